"""MI355X (gfx950) flux-stencil library for the higher-order cut-cell finite-volume
Poisson method of Devendran, Graves and Johansen (arXiv:1411.4283).

The method runs in libcutcell.so (HIP kernels behind the C ABI of include/cutcell.h);
this package is its Python binding.  Importing it does not load the library; the first
call does, and fails loudly if the library has not been built.
"""

from .api import Builder, DeviceGeometry, Stencils, apply, build_stencils, make_opts  # noqa: F401
from ._lib import CutcellError, LIB_PATH, load  # noqa: F401
from .api import Transpose, apply_adjoint, build_transpose  # noqa: F401,E402
from .autograd import CutCellOperator, OperatorApply, StencilBuild  # noqa: F401,E402
from .api import Laplacian, SolveResult, apply_laplacian, build_laplacian, solve  # noqa: F401,E402
from .api import hessenberg_eigs, ritz  # noqa: F401,E402
from .api import Packed, apply_packed, pack  # noqa: F401,E402
