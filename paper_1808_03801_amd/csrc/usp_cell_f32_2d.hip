// cell kernel instantiations: F32 particle state, 2-D
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(float, 2, false)
USP_CELL_W6(float, 2)
}  // namespace usp
