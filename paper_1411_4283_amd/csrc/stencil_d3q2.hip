// Stencil kernels of dimension 3, order 2 (one translation unit per (dimension, order),
// so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(3, 2, )
}  // namespace cutcell
