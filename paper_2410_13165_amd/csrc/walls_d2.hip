// Wall kernels of d = 2.
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(2, false)
LBM_WALL_INST(2, true)

}  // namespace lbm
