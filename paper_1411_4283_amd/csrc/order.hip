// Processing order of the faces (the permutation the stencil kernels walk).  Faces are
// grouped by bucket (16-row bins, then faces with fewer rows than monomials, then template
// copies), a row bin's faces by part (at most 8, 12, 16 rows above the bin below), and
// inside that ordered by the cell they sit at -- a grid face's low-side
// cell (the last cell for faces on the high box side), an EB face's cut cell -- so that
// the faces of all directions around the same cells are solved together and share the
// rows' moments in one L2.  One stable 64-bit radix sort of (bucket, part, geometry, cell).
// The stencils do not depend on the order.
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace cutcell {

constexpr int kKeyBits = 45;   // 40 bits of (geometry, cell), 5 of (bucket, part)
static_assert(3 * kNBuckets <= 32, "bucket and part must fit in 5 key bits");

__global__ void k_face_keys(GridDims g, long long n_face, int M, const int32_t* __restrict__ fcode,
                            const int32_t* __restrict__ fref, const GeomPtrs* __restrict__ geoms,
                            const int32_t* __restrict__ nrows, const int32_t* __restrict__ tmpl,
                            unsigned long long* __restrict__ keys, int32_t* __restrict__ vals) {
  const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f >= n_face) return;
  const int32_t code = fcode[f];
  const int gi = code >> 4, kind = (code >> 2) & 3, dn = code & 3;
  long long cell;
  if (kind == 0) {
    const long long loc = fref[f] - g.foff[dn];
    const int m0 = g.n[0] + (dn == 0), m1 = g.n[1] + (dn == 1);
    int j[3] = {(int)(loc % m0), (int)((loc / m0) % m1), (int)(loc / ((long long)m0 * m1))};
    if (j[dn] > g.n[dn] - 1) j[dn] = g.n[dn] - 1;
    cell = j[0] + (long long)g.n[0] * (j[1] + (long long)g.n[1] * j[2]);
  } else {
    cell = geoms[gi].eb_cell[fref[f]];
  }
  const int b = face_bucket(f, M, nrows, tmpl);
  const unsigned long long bh = (unsigned long long)(3 * b + face_part(b, f, nrows));
  keys[f] = (bh << 40) | (unsigned long long)((long long)gi * g.ncell + cell);
  vals[f] = (int32_t)f;
}

size_t order_temp_bytes(long long n_items) {
  size_t temp = 0;
  if (n_items > 0)
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const unsigned long long*)nullptr,
                                             (unsigned long long*)nullptr, (const int32_t*)nullptr, (int32_t*)nullptr,
                                             (int)n_items, 0, kKeyBits, (hipStream_t)0);
  return temp;
}

int order_faces(const Work& w, long long n_face, int M, const int32_t* tmpl, hipStream_t st) {
  if (n_face <= 0) return CUTCELL_OK;
  if (order_temp_bytes(n_face) > w.osort_bytes) return fail(CUTCELL_E_WORKSPACE, "face-order scratch too small");
  const int T = 256;
  hipLaunchKernelGGL(k_face_keys, dim3((unsigned)((n_face + T - 1) / T)), dim3(T), 0, st, w.dims, n_face, M, w.fcode,
                     w.fref, w.geoms, w.nrows, tmpl, w.okey, w.oval);
  size_t bytes = w.osort_bytes;
  CC_HIP(hipcub::DeviceRadixSort::SortPairs(w.osort_tmp, bytes, w.okey, w.okey_out, w.oval, w.perm, (int)n_face, 0,
                                            kKeyBits, st));
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
