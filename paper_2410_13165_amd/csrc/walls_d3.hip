// Wall kernels of d = 3 with analytic wall data.
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(3, false)

}  // namespace lbm
