// Stencil kernels of dimension 2, order 2 (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(2, 2, )
CC_ROW_BINS_ALL(2, 2, )
}  // namespace cutcell
