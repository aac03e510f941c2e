// Wall kernels of d = 4 with analytic wall data (one run-time wall variant).
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(4, false)

}  // namespace lbm
