// Stencil kernels of dimension 2, order 2 (one translation unit per (dimension, order),
// so that they compile in parallel).
#include "stencil_impl.hpp"

namespace cutcell {
CC_DISPATCH(2, 2, )
}  // namespace cutcell
