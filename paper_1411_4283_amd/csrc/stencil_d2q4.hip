// Stencil kernels of dimension 2, order 4 (one translation unit per (dimension, order),
// so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(2, 4, )
}  // namespace cutcell
