// Wall kernels of d = 4 with tangential wall data (Remark 1; one run-time wall variant).
#include "walls.hpp"

namespace lbm {

LBM_WALL_INST(4, true)

}  // namespace lbm
