// cell kernel instantiations: F64 particle state, 2-D
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(double, 2, false)
USP_CELL_W6(double, 2)
}  // namespace usp
