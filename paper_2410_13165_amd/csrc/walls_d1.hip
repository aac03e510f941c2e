// Wall kernels of d = 1 (one run-time wall variant).
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(1, false)
LBM_WALL_INST(1, true)

}  // namespace lbm
