// Stencil kernels of dimension 3, order 4: dispatch and the 48- and 64-row bins (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(3, 4, )
CC_ROW_BIN(3, 4, 48, )
CC_ROW_BIN(3, 4, 64, )
}  // namespace cutcell
