// Wall kernels of d = 1 and 4 (one run-time variant each).
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(1, false)
LBM_WALL_INST(1, true)
LBM_WALL_INST(4, false)
LBM_WALL_INST(4, true)

}  // namespace lbm
