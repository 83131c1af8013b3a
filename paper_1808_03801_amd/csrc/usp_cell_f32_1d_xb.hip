// cell kernel instantiations: F32 particle state, 1-D, open faces and the plate
#include "usp_cell_impl.h"

namespace usp {
USP_CELL_ALL(float, 1, true)
}  // namespace usp
