// Stencil kernels of dimension 3, order 4: the 112- and 128-row bins (the kernels are
// split over several files so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_ROW_BIN(3, 4, 112, )
CC_ROW_BIN(3, 4, 128, )
}  // namespace cutcell
