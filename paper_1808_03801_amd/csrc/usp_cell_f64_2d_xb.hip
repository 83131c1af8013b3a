// cell kernel instantiations: F64 particle state, 2-D, open faces and the plate
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(double, 2, true)
}  // namespace usp
