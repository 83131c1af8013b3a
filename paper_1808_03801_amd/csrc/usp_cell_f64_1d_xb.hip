// cell kernel instantiations: F64 particle state, 1-D, open faces and the plate
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(double, 1, true)
}  // namespace usp
