// Host side of the stencil solves: launches per bin (the kernels are in stencil_impl.hpp,
// instantiated per dimension and order in stencil_d*q*.hip), the faces with fewer rows
// than monomials, the template copies, and the launch-schedule autotuner.
#include "stencil_impl.hpp"

namespace cutcell {

// Faces with fewer rows than monomials: zero stencil, status INSUFFICIENT_ROWS -- except,
// under Neumann EB conditions, the EB faces, whose one-row stencil is their area
// |A_f| = h^(D-1) m^0 (the flux is the prescribed data).
__global__ void k_insufficient(const int32_t* __restrict__ perm, long long n, const int64_t* __restrict__ row_ptr,
                               double* val, int8_t* status, int32_t* flagged, const int32_t* __restrict__ fcode,
                               const int32_t* __restrict__ fref, const GeomPtrs* __restrict__ geoms, int neumann,
                               double hd1, int M) {
  long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t F = perm[t];
  const int32_t code = fcode[F];
  if (neumann && ((code >> 2) & 3) == 1) {
    const double area = hd1 * geoms[code >> 4].eb_mom[(long long)fref[F] * M];
    const bool ok = isfinite(area);
    val[row_ptr[F]] = ok ? area : 0.0;
    status[F] = ok ? CUTCELL_STATUS_OK : CUTCELL_STATUS_NONFINITE;
    if (!ok) atomicAdd(flagged, 1);
    return;
  }
  for (int64_t j = row_ptr[F]; j < row_ptr[F + 1]; ++j) val[j] = 0.0;
  status[F] = CUTCELL_STATUS_INSUFFICIENT_ROWS;
  atomicAdd(flagged, 1);
}

// Faces whose system is bitwise that of their template face: the template's values (the
// same rows in the same order) and status.  One wave per face.
__global__ __launch_bounds__(64) void k_copy_template(const int32_t* __restrict__ perm, long long n,
                                                      const int32_t* __restrict__ tmpl,
                                                      const int64_t* __restrict__ row_ptr, double* val, int8_t* status,
                                                      int32_t* flagged) {
  const long long t = blockIdx.x;
  if (t >= n) return;
  const int32_t F = perm[t];
  const int32_t T = tmpl[F];
  const int64_t a = row_ptr[F], b = row_ptr[T];
  const int N = (int)(row_ptr[F + 1] - a);
  for (int i = threadIdx.x; i < N; i += 64) val[a + i] = val[b + i];
  if (threadIdx.x == 0) {
    const int8_t s = status[T];
    status[F] = s;
    if (s != CUTCELL_STATUS_OK) atomicAdd(flagged, 1);
  }
}

// faces with fewer rows than monomials carry no gradient
__global__ void k_insufficient_backward(const int32_t* __restrict__ perm, long long n,
                                        const int64_t* __restrict__ row_ptr, int M, BackwardArgs B) {
  long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t F = perm[t];
  for (int64_t j = row_ptr[F]; j < row_ptr[F + 1]; ++j) {
    B.nz_rz[2 * j] = 0.0;
    B.nz_rz[2 * j + 1] = 0.0;
    if (B.weight_bar) B.weight_bar[j] = 0.0;
  }
  for (int p = 0; p < 2 * M; ++p) B.face_yw[(long long)F * 2 * M + p] = 0.0;
  for (int k = 0; k < 4; ++k) {
    B.owner_grad[(long long)F * 4 + k] = 0.0;
    B.face_x0[(long long)F * 4 + k] = 0.0;
  }
}

static int run_bins(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                    const int32_t* col, double* val, int8_t* status, hipStream_t st, const BackwardArgs* bw,
                    const BinSchedule* sched, int only_bin = -1) {
  double hscale = 1.0;
  for (int d = 0; d < o.dim - 2; ++d) hscale *= o.h;   // h^(D-2)
  const bool neu = o.eb_bc == CUTCELL_BC_NEUMANN;
  const bool qr_all = !bw && o.factorization == CUTCELL_FACTOR_QR;
  const bool route = o.factorization != CUTCELL_FACTOR_GRAM;
  BinSchedule sc[kMaxBins];
  for (int b = 0; b < kMaxBins; ++b) {
    sc[b] = sched[b];
    sc[b].route = route;
  }
  int rc = CUTCELL_E_UNSUPPORTED;
  if (!bw) hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.qr_count, 1LL, 0);
  if (qr_all) {
    // every face of the row bins (or of bin only_bin) by Householder QR
    long long first = 0, n = 0;
    for (int b = 0; b < kMaxBins; ++b) {
      if (only_bin < 0 || b == only_bin) n += bin_count[b];
      else if (b < only_bin) first += bin_count[b];
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.qr_count, 1LL, (int32_t)n);
    rc = solve_qr_faces(w, o, w.perm + first, nullptr, n, row_ptr, col, val, status, st);
    if (rc != CUTCELL_OK) return rc;
  } else {
#define CC_RB(DD, QQ) \
  if (o.dim == DD && o.order == QQ) \
    rc = dispatch_row_bins<DD, QQ>(w, hscale, bin_count, row_ptr, col, val, status, st, bw, sc, only_bin, neu, o.h, \
                                   o.weight_custom ? o.weight_power : 5.0);
    CC_RB(2, 2) CC_RB(2, 4) CC_RB(3, 2) CC_RB(3, 4)
#undef CC_RB
    if (rc == CUTCELL_E_UNSUPPORTED) return fail(CUTCELL_E_UNSUPPORTED, "order/dimension");
    if (rc != CUTCELL_OK) return rc;
    // the faces the Gram path left to Householder QR (their count is on the device)
    if (!bw && route) {
      rc = solve_qr_faces(w, o, w.qr_list, w.qr_count, 0, row_ptr, col, val, status, st);
      if (rc != CUTCELL_OK) return rc;
    }
  }
  // after the bins: faces with fewer rows than monomials, and the template copies (the
  // templates are solved by then: same stream)
  const int M = binom(o.order + o.dim, o.dim);
  long long start = 0;
  for (int b = 0; b < kMaxBins; ++b) start += bin_count[b];
  const long long ninsuf = (only_bin < 0) ? bin_count[kMaxBins] : 0;
  const long long ncopy = (only_bin < 0 && !bw) ? bin_count[kMaxBins + 1] : 0;
  if (ncopy > 0)
    hipLaunchKernelGGL(k_copy_template, dim3((unsigned)ncopy), dim3(64), 0, st, w.perm + start + bin_count[kMaxBins],
                       ncopy, w.tmpl, row_ptr, val, status, w.flagged);
  if (ninsuf > 0 && bw)
    hipLaunchKernelGGL(k_insufficient_backward, dim3((unsigned)((ninsuf + 255) / 256)), dim3(256), 0, st,
                       w.perm + start, ninsuf, row_ptr, M, *bw);
  else if (ninsuf > 0)
    hipLaunchKernelGGL(k_insufficient, dim3((unsigned)((ninsuf + 255) / 256)), dim3(256), 0, st, w.perm + start,
                       ninsuf, row_ptr, val, status, w.flagged, w.fcode, w.fref, w.geoms, (int)neu,
                       o.dim == 3 ? o.h * o.h : o.h, M);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

static void schedules_from(const cutcell_tuning* t, BinSchedule* sc) {
  for (int b = 0; b < kMaxBins; ++b) {
    sc[b] = BinSchedule{};
    if (t) {
      sc[b].xcd = t->xcd_chunks[b] > 1 ? t->xcd_chunks[b] : 1;
      sc[b].per_xcd = t->blocks_per_xcd[b] > 0 ? t->blocks_per_xcd[b] : 0;
      sc[b].split = (t->split[b] >= 0 && t->split[b] <= 3) ? t->split[b] : 0;
    }
  }
}

int solve_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, long long n_face,
                   const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status, hipStream_t st) {
  (void)n_face;
  BinSchedule sc[kMaxBins];
  schedules_from(o.tuning, sc);
  return run_bins(w, o, bin_count, row_ptr, col, val, status, st, nullptr, sc);
}

int backward_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                      const int32_t* col, const BackwardArgs& bw, hipStream_t st) {
  BinSchedule sc[kMaxBins];
  schedules_from(nullptr, sc);
  return run_bins(w, o, bin_count, row_ptr, col, nullptr, nullptr, st, &bw, sc);
}

// Times every candidate of every non-empty bin on these faces (HIP events, best of
// `reps`) and keeps the fastest: the five launch schedules, crossed with the split modes
// the bin's compiled kernel widths allow; then solves all bins with the choices, so
// val/status hold the same stencils as an untuned build.
int tune_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                  const int32_t* col, double* val, int8_t* status, hipStream_t st, cutcell_tuning* out, int reps,
                  double* best_ms) {
  int dev = 0, cus = 256;
  CC_HIP(hipGetDevice(&dev));
  CC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int X = kXcds;
  const int resident = std::max(1, cus / X) * 4;   // workgroups per XCD at one wave per SIMD
  const BinSchedule launch[] = {{1, 0}, {X, 0}, {X, resident}, {X, 2 * resident}, {1, X * resident}};
  const int nlaunch = (int)(sizeof(launch) / sizeof(launch[0]));
  hipEvent_t e0, e1;
  CC_HIP(hipEventCreate(&e0));
  CC_HIP(hipEventCreate(&e1));
  BinSchedule sc[kMaxBins];
  schedules_from(nullptr, sc);
  for (int b = 0; b < kMaxBins; ++b) {
    best_ms[b] = -1.0;
    if (bin_count[b] == 0) continue;
    double best = 1e300;
    // split modes that differ for this bin: 1 (whole bin at its width) always; 2 with a
    // NPAD - 8 instance, 3 with a NPAD - 4 one, 0 with both
    const int nm = narrow_mask_of(o.dim, o.order, b);
    int splits[4], nsplit = 0;
    splits[nsplit++] = 1;
    if (nm & 1) splits[nsplit++] = 2;
    if (nm & 2) splits[nsplit++] = 3;
    if ((nm & 3) == 3) splits[nsplit++] = 0;
    for (int c = 0; c < nlaunch * nsplit; ++c) {
      BinSchedule cand = launch[c % nlaunch];
      cand.split = splits[c / nlaunch];
      BinSchedule trial[kMaxBins];
      for (int i = 0; i < kMaxBins; ++i) trial[i] = cand;
      double tmin = 1e300;
      for (int r = 0; r < reps; ++r) {
        CC_HIP(hipEventRecord(e0, st));
        int rc = run_bins(w, o, bin_count, row_ptr, col, val, status, st, nullptr, trial, b);
        if (rc) return rc;
        CC_HIP(hipEventRecord(e1, st));
        CC_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CC_HIP(hipEventElapsedTime(&ms, e0, e1));
        tmin = std::min(tmin, (double)ms);
      }
      if (tmin < best) {
        best = tmin;
        sc[b] = cand;
      }
    }
    best_ms[b] = best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int b = 0; b < kMaxBins; ++b) {
    out->xcd_chunks[b] = sc[b].xcd;
    out->blocks_per_xcd[b] = sc[b].per_xcd;
    out->split[b] = sc[b].split;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.flagged, 1LL, 0);
  return run_bins(w, o, bin_count, row_ptr, col, val, status, st, nullptr, sc);
}

}  // namespace cutcell
