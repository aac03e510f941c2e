// Wall kernels of d = 3 with tangential wall data (Remark 1).
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(3, true)

}  // namespace lbm
