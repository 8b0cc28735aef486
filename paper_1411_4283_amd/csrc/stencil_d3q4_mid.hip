// Stencil kernels of dimension 3, order 4: the 80- and 96-row bins (with the 88-row half) (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_ROW_BIN(3, 4, 80, )
CC_ROW_BIN(3, 4, 96, )
}  // namespace cutcell
