// Stencil kernels of dimension 2, order 4 (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(2, 4, )
CC_ROW_BINS_ALL(2, 4, )
}  // namespace cutcell
