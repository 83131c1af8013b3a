// cell kernel instantiations: F64 particle state, 1-D
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(double, 1, false)
USP_CELL_W6(double, 1)
}  // namespace usp
