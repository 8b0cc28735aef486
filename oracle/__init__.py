"""Plain CPU oracle for the cut-cell flux-stencil method of Devendran, Graves and
Johansen, "A higher-order finite-volume discretization method for Poisson's equation
in cut cell geometries" (arXiv:1411.4283).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP library;
the only common dependency is the seeded input generator ``cutgeom``.

The oracle follows the paper's definitions directly, face by face, in numpy: the FP64
moments are the inputs, and each stencil is formed from them in x87 extended precision
(numpy.longdouble) -- offsets, weights, re-centred rows, a plain Householder QR and the
minimum-norm solve -- then rounded to FP64.  Every function cites the passage it
implements.
"""

from .stencils import (  # noqa: F401
    Enumeration,
    enumerate_geometry,
    neighbours,
    neighbours_all,
    face_system,
    face_stencil,
    face_condition,
    face_centre,
    face_centre_h,
    face_system_ld,
    householder_qr,
    min_norm_solve,
    flux_vector,
    eb_normal_flux,
    recentre,
    row_weights,
    volumes_within,
    build,
    apply,
    STATUS_OK,
    STATUS_INSUFFICIENT_ROWS,
    STATUS_RANK_DEFICIENT,
    STATUS_NONFINITE,
)
from .adjoint import apply_adjoint, stencils_backward  # noqa: F401,E402
from .solve import operator_matrix, solve  # noqa: F401,E402
