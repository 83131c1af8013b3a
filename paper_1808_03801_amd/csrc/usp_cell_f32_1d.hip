// cell kernel instantiations: F32 particle state, 1-D
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(float, 1, false)
USP_CELL_W6(float, 1)
}  // namespace usp
