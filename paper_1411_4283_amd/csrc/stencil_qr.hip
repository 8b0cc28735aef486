// Launches of the Householder QR path (stencil_qr.hpp): the faces the Gram path leaves to
// it, or every face when the caller asks for this factorisation.
#include "stencil_qr.hpp"

namespace cutcell {

int solve_qr_faces(const Work& w, const cutcell_opts& o, const int32_t* list, const int32_t* count_dev,
                   long long count_host, const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status,
                   hipStream_t st) {
  if (!count_dev && count_host <= 0) return CUTCELL_OK;
  int dev = 0, cus = 256;
  CC_HIP(hipGetDevice(&dev));
  CC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  long long grid = std::min<long long>(4LL * cus, w.qr_slots);   // 4 per CU (shared memory, registers)
  if (!count_dev) grid = std::min(grid, count_host);
  double hscale = 1.0;
  for (int d = 0; d < o.dim - 2; ++d) hscale *= o.h;   // h^(D-2)
  StencilArgs A = stencil_args(w, hscale, w.perm, 0, row_ptr, col);
  A.h = o.h;
  A.wpow = o.weight_custom ? o.weight_power : 5.0;
  const bool neu = o.eb_bc == CUTCELL_BC_NEUMANN;
  const dim3 g((unsigned)grid), b(64);
#define CC_QR(DD, QQ)                                                                                           \
  if (o.dim == DD && o.order == QQ) {                                                                           \
    if (neu)                                                                                                    \
      hipLaunchKernelGGL((k_stencil_qr<DD, QQ, true>), g, b, 0, st, A, list, count_dev, count_host, w.qr_b, val, \
                         status, w.flagged);                                                                            \
    else                                                                                                        \
      hipLaunchKernelGGL((k_stencil_qr<DD, QQ, false>), g, b, 0, st, A, list, count_dev, count_host, w.qr_b, val, \
                         status, w.flagged);                                                                    \
    CC_HIP(hipGetLastError());                                                                                  \
    return CUTCELL_OK;                                                                                          \
  }
  CC_QR(2, 2) CC_QR(2, 4) CC_QR(3, 2) CC_QR(3, 4)
#undef CC_QR
  return fail(CUTCELL_E_UNSUPPORTED, "order/dimension");
}

}  // namespace cutcell
