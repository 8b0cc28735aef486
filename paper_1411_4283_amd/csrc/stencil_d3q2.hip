// Stencil kernels of dimension 3, order 2 (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(3, 2, )
CC_ROW_BINS_ALL(3, 2, )
}  // namespace cutcell
