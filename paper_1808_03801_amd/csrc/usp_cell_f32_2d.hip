// cell kernel instantiations: F32 particle state, 2-D
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(float, 2, false)
}  // namespace usp
