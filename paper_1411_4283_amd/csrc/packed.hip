// Compressed stencils for repeated applies: the stencil of a face that was copied from a
// template face (Sec. 4 names standard interior stencils as the natural next step; the
// regular faces' stencils of Fig. 2b are all the same up to a shift) is stored as the
// template's slot plus one Phi index per run of consecutive columns, instead of its own
// columns and values: its values are the slot's (a copy of the template's row), its
// columns base[run] + position in the run.
//
// A face is packed only where this reproduces its CSR row exactly: the same row count as
// its template, columns consecutive wherever the template's are, and values equal bit
// for bit.  The apply gives the plain apply's result bit for bit: both kinds of face are
// summed in the order the CSR flux pass (k_flux) adds a face's products -- entry j in
// lane (phase + j) mod 64, ascending per lane, then the same butterfly -- where the phase
// is the face's row offset from the first face of its group there.  One launch takes the
// CSR pass's groups of faces (packed faces skipped, their entries never loaded), then the
// packed faces.
//
// On MI355X this does not beat the plain apply although it reads 41% fewer bytes on the
// 64^3 fourth-order workload: both kinds of wave are bound by the latency of their
// dependent loads (row bounds, entries, Phi gathers), not by HBM bandwidth, and the
// packed faces add gathers (run bases) of their own.  It is kept for the bytes, exact.
#include "gather.hpp"
#include "scan.hpp"

namespace cutcell {

namespace {

inline unsigned nblocks(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// the template of face f, or -1 when it has none usable
__device__ __forceinline__ int32_t template_of(const int32_t* __restrict__ tmpl, long long f, long long n_face) {
  const int32_t t = tmpl[f];
  return (t >= 0 && t < n_face && t != f) ? t : -1;
}

// a run of the template's columns starts at entry j
__device__ __forceinline__ bool run_head(const int32_t* __restrict__ col, int64_t rt, int j) {
  return j == 0 || col[rt + j] != col[rt + j - 1] + 1;
}

__global__ void k_pack_mark(long long n_face, const int32_t* __restrict__ tmpl, int32_t* is_tmpl) {
  const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f >= n_face) return;
  const int32_t t = template_of(tmpl, f, n_face);
  if (t >= 0) is_tmpl[t] = 1;   // every writer stores the same value
}

// runs and rows of each template face: the maxima size the tables
__global__ void k_pack_tinfo(long long n_face, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ is_tmpl, int32_t* maxima) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n_face || !is_tmpl[t]) return;
  const int64_t rt = row_ptr[t];
  const int n = (int)(row_ptr[t + 1] - rt);
  int runs = 0;
  for (int j = 0; j < n; ++j) runs += run_head(col, rt, j);
  atomicMax(&maxima[0], runs);
  atomicMax(&maxima[1], n);
}

// one wave per face: does its row reproduce from its template's?
__global__ __launch_bounds__(256) void k_pack_check(long long n_face, const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    const int32_t* __restrict__ tmpl, int32_t* __restrict__ ok) {
  const long long f = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (f >= n_face) return;
  const int32_t t = template_of(tmpl, f, n_face);
  bool good = t >= 0;
  if (good) {
    const int64_t rf = row_ptr[f], rt = row_ptr[t];
    const int n = (int)(row_ptr[f + 1] - rf);
    good = n > 0 && n == (int)(row_ptr[t + 1] - rt) && n <= 0x7fff;
    if (good) {
      bool bad = false;
      for (int j = lane; j < n; j += 64) {
        if (!run_head(col, rt, j) && col[rf + j] != col[rf + j - 1] + 1) bad = true;
        if (__double_as_longlong(val[rf + j]) != __double_as_longlong(val[rt + j])) bad = true;
      }
      good = !__any(bad);
    }
  }
  if (lane == 0) ok[f] = good ? 1 : 0;
}

// per template: its face and, per entry, run index | position in the run << 16
__global__ void k_pack_slots(long long n_face, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ is_tmpl, const int32_t* __restrict__ slot_of, int max_rows,
                             int32_t* __restrict__ slot_face, int32_t* __restrict__ slot_tab) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n_face || !is_tmpl[t]) return;
  const int s = slot_of[t];
  slot_face[s] = (int32_t)t;
  const int64_t rt = row_ptr[t];
  const int n = (int)(row_ptr[t + 1] - rt);
  int32_t* tab = slot_tab + (long long)s * max_rows;
  int r = -1, head = 0;
  for (int j = 0; j < n; ++j) {
    if (run_head(col, rt, j)) {
      ++r;
      head = j;
    }
    tab[j] = r | ((j - head) << 16);
  }
  for (int j = n; j < max_rows; ++j) tab[j] = 0;
}

// per face: packed or not and its phase; per packed face its slot and the first column of
// each run
__global__ void k_pack_fill(long long n_face, int GF, const int64_t* __restrict__ row_ptr,
                            const int32_t* __restrict__ col, const int32_t* __restrict__ tmpl,
                            const int32_t* __restrict__ ok, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ slot_of, int max_runs, uint8_t* __restrict__ flag,
                            uint8_t* __restrict__ phase, int32_t* __restrict__ face, int32_t* __restrict__ slot,
                            int32_t* __restrict__ base) {
  const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f >= n_face) return;
  const int64_t rf = row_ptr[f];
  phase[f] = (uint8_t)((rf - row_ptr[f - f % GF]) & 63);
  flag[f] = ok[f] ? 1 : 0;
  if (!ok[f]) return;
  const long long i = pos[f];
  const int32_t t = tmpl[f];
  face[i] = (int32_t)f;
  slot[i] = slot_of[t];
  const int64_t rt = row_ptr[t];
  const int n = (int)(row_ptr[f + 1] - rf);
  int32_t* b = base + i * max_runs;
  int r = 0;
  for (int j = 0; j < n; ++j)
    if (run_head(col, rt, j)) b[r++] = col[rf + j];
  for (; r < max_runs; ++r) b[r] = 0;
}

// 64-bit ds_bpermute: v of lane src
__device__ __forceinline__ double pull_f64(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src * 4, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src * 4, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

constexpr int kQ = 8;   // faces per wave of k_apply_compact

// butterfly over the wave, as k_flux ends
__device__ __forceinline__ double wave_sum(double a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  return a;
}

// kQ packed faces.  Consecutive packed faces nearly always share a slot (faces run by
// direction, then lattice index): then the slot's table and values are loaded once, in
// lane = j order, each face's run bases with one coalesced load (a lane per run), and
// per face only Phi is gathered; each lane then pulls its products from lane j0.  Other
// waves take each face on its own.
__device__ __forceinline__ void packed_faces(const PackedArgs& P, long long i0, int lane,
                                             const double* __restrict__ phi, double* __restrict__ flux) {
#pragma clang fp contract(off)
  const int s0 = P.slot[i0];
  bool one_slot = i0 + kQ <= P.n_packed;
#pragma unroll
  for (int q = 1; q < kQ; ++q) one_slot = one_slot && (i0 + q >= P.n_packed || P.slot[i0 + q] == s0);
  const int n0 = P.slot_rows[s0];
  if (one_slot && n0 <= 128 && P.max_runs <= 64) {
    const long long so = (long long)s0 * P.max_rows;
    const bool in0 = lane < n0, in1 = lane + 64 < n0;
    const int32_t tb0 = in0 ? P.slot_tab[so + lane] : 0, tb1 = in1 ? P.slot_tab[so + lane + 64] : 0;
    const double v0 = in0 ? P.slot_val[so + lane] : 0.0, v1 = in1 ? P.slot_val[so + lane + 64] : 0.0;
    int32_t br[kQ];
    uint8_t ph[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      br[q] = lane < P.max_runs ? P.base[(i0 + q) * P.max_runs + lane] : 0;
      ph[q] = P.phase[P.face[i0 + q]];
    }
    double o = 0.0;
    int32_t fo = -1;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int32_t c0 = __shfl(br[q], tb0 & 0xffff, 64) + (tb0 >> 16);
      const int32_t c1 = __shfl(br[q], tb1 & 0xffff, 64) + (tb1 >> 16);
      const double p0 = in0 ? v0 * phi[c0] : 0.0;
      const double p1 = in1 ? v1 * phi[c1] : 0.0;
      const int j0 = (lane - ph[q]) & 63;
      const double a0 = pull_f64(p0, j0), a1 = pull_f64(p1, j0);
      double acc = 0.0;
      if (j0 < n0) acc += a0;
      if (j0 + 64 < n0) acc += a1;
      acc = wave_sum(acc);
      if (lane == q) {
        o = acc;
        fo = P.face[i0 + q];
      }
    }
    if (lane < kQ) flux[fo] = o;
    return;
  }
  for (int q = 0; q < kQ && i0 + q < P.n_packed; ++q) {
    const long long i = i0 + q;
    const int32_t f = P.face[i], s = P.slot[i];
    const int n = P.slot_rows[s];
    const long long so = (long long)s * P.max_rows;
    const int32_t* b = P.base + i * P.max_runs;
    double acc = 0.0;
    for (int j = (lane - P.phase[f]) & 63; j < n; j += 64) {
      const int32_t tb = P.slot_tab[so + j];
      const double p = P.slot_val[so + j] * phi[b[tb & 0xffff] + (tb >> 16)];
      acc += p;
    }
    acc = wave_sum(acc);
    if (lane == 0) flux[f] = acc;
  }
}

// The CSR pass's groups (packed faces skipped), then the packed faces, in one launch.
template <int GF, int U>
__global__ __launch_bounds__(256) void k_apply_packed(PackedArgs P, long long n_face,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const double* __restrict__ val,
                                                      const double* __restrict__ phi, double* __restrict__ flux) {
  const long long w = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const long long w1 = (n_face + GF - 1) / GF;
  if (w < w1) flux_group<GF, U, true>(w, lane, n_face, row_ptr, col, val, phi, flux, P.flag);
  else if ((w - w1) * kQ < P.n_packed) packed_faces(P, (w - w1) * kQ, lane, phi, flux);
}

// the slots' row counts and values (copies of the templates' rows, zero-padded)
__global__ void k_pack_slot_vals(int n_slot, int max_rows, const int32_t* __restrict__ slot_face,
                                 const int64_t* __restrict__ row_ptr, const double* __restrict__ val,
                                 int32_t* __restrict__ slot_rows, double* __restrict__ slot_val) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)n_slot * max_rows) return;
  const int s = (int)(k / max_rows), j = (int)(k % max_rows);
  const int32_t t = slot_face[s];
  const int64_t rt = row_ptr[t];
  const int n = (int)(row_ptr[t + 1] - rt);
  if (j == 0) slot_rows[s] = n;
  slot_val[k] = j < n ? val[rt + j] : 0.0;
}

struct PackWs {
  int32_t* is_tmpl;
  int32_t* slot_of;
  int32_t* ok;
  int32_t* pos;
  int32_t* scan_tmp;
  int32_t* totals;   // [2]: templates, packed faces
  int32_t* maxima;   // [2]: runs, rows per template
};

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

PackWs pack_layout(long long n_face, char* ws) {
  const long long n1 = n_face > 0 ? n_face : 1;
  PackWs p;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = ws + off;
    off += al256(b);
    return q;
  };
  p.is_tmpl = (int32_t*)take(sizeof(int32_t) * n1);
  p.slot_of = (int32_t*)take(sizeof(int32_t) * n1);
  p.ok = (int32_t*)take(sizeof(int32_t) * n1);
  p.pos = (int32_t*)take(sizeof(int32_t) * n1);
  p.scan_tmp = (int32_t*)take(sizeof(int32_t) * (scan_tiles(n1) + 1));
  p.totals = (int32_t*)take(sizeof(int32_t) * 2);
  p.maxima = (int32_t*)take(sizeof(int32_t) * 2);
  return p;
}

// marks the templates, numbers them, checks every face against its template and numbers
// the packed faces; returns (on the host) the counts and maxima
int pack_prepare(long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
                 const int32_t* tmpl, const PackWs& p, int32_t* totals, int32_t* maxima, hipStream_t st) {
  const int T = 256;
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(n_face, T)), dim3(T), 0, st, p.is_tmpl, n_face, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, p.totals, 2LL, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, p.maxima, 2LL, 0);
  hipLaunchKernelGGL(k_pack_mark, dim3(nblocks(n_face, T)), dim3(T), 0, st, n_face, tmpl, p.is_tmpl);
  int rc = exclusive_scan<int32_t, int32_t>(p.is_tmpl, n_face, n_face, 1, p.slot_of, n_face, p.totals, p.scan_tmp,
                                            st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_pack_tinfo, dim3(nblocks(n_face, T)), dim3(T), 0, st, n_face, row_ptr, col, p.is_tmpl,
                     p.maxima);
  hipLaunchKernelGGL(k_pack_check, dim3(nblocks(n_face * 64, T)), dim3(T), 0, st, n_face, row_ptr, col, val, tmpl,
                     p.ok);
  rc = exclusive_scan<int32_t, int32_t>(p.ok, n_face, n_face, 1, p.pos, n_face, p.totals + 1, p.scan_tmp, st);
  if (rc) return rc;
  CC_HIP(hipMemcpyAsync(totals, p.totals, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(maxima, p.maxima, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace

size_t pack_temp_bytes(long long n_face) {
  const long long n1 = n_face > 0 ? n_face : 1;
  return 4 * al256(sizeof(int32_t) * n1) + al256(sizeof(int32_t) * (scan_tiles(n1) + 1)) + 2 * al256(8);
}

int pack_count(long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
               const int32_t* tmpl, char* ws, size_t ws_bytes, long long* n_packed, int* n_slot, int* max_runs,
               int* max_rows, hipStream_t st) {
  *n_packed = 0;
  *n_slot = *max_runs = *max_rows = 0;
  if (n_face <= 0) return CUTCELL_OK;
  if (ws_bytes < pack_temp_bytes(n_face)) return fail(CUTCELL_E_WORKSPACE, "pack workspace too small");
  int32_t totals[2], maxima[2];
  int rc = pack_prepare(n_face, row_ptr, col, val, tmpl, pack_layout(n_face, ws), totals, maxima, st);
  if (rc) return rc;
  *n_slot = totals[0];
  *n_packed = totals[1];
  *max_runs = maxima[0];
  *max_rows = maxima[1];
  return CUTCELL_OK;
}

int pack_fill(int D, long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
              const int32_t* tmpl, char* ws, size_t ws_bytes, const PackedSizes& ps, const PackedOut& out,
              hipStream_t st) {
  if (n_face <= 0) return CUTCELL_OK;
  if (ws_bytes < pack_temp_bytes(n_face)) return fail(CUTCELL_E_WORKSPACE, "pack workspace too small");
  const PackWs p = pack_layout(n_face, ws);
  int32_t totals[2], maxima[2];
  int rc = pack_prepare(n_face, row_ptr, col, val, tmpl, p, totals, maxima, st);
  if (rc) return rc;
  if (totals[0] != ps.n_slot || totals[1] != ps.n_packed || maxima[0] != ps.max_runs || maxima[1] != ps.max_rows)
    return fail(CUTCELL_E_CAPACITY, "packed sizes do not match these stencils (call cutcell_pack_count first)");
  const int T = 256;
  if (ps.n_slot > 0) {
    hipLaunchKernelGGL(k_pack_slots, dim3(nblocks(n_face, T)), dim3(T), 0, st, n_face, row_ptr, col, p.is_tmpl,
                       p.slot_of, ps.max_rows, out.slot_face, out.slot_tab);
    hipLaunchKernelGGL(k_pack_slot_vals, dim3(nblocks((long long)ps.n_slot * ps.max_rows, T)), dim3(T), 0, st,
                       ps.n_slot, ps.max_rows, out.slot_face, row_ptr, val, out.slot_rows, out.slot_val);
  }
  hipLaunchKernelGGL(k_pack_fill, dim3(nblocks(n_face, T)), dim3(T), 0, st, n_face,
                     D == 3 ? kFluxFaces3 : kFluxFaces2, row_ptr, col, tmpl, p.ok, p.pos, p.slot_of, ps.max_runs,
                     out.flag, out.phase, out.face, out.slot, out.base);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int apply_packed(int D, long long n_face, long long n_vol, const int64_t* row_ptr, const int32_t* col,
                 const double* val, const int32_t* vol_face, const double* vol_scale, const PackedArgs& pk,
                 const double* phi, double* lphi, double* flux, hipStream_t st) {
  if (n_face > 0) {
    constexpr int T = 256;
    const int GF = D == 3 ? kFluxFaces3 : kFluxFaces2;
    const long long waves = (n_face + GF - 1) / GF + (pk.n_packed + kQ - 1) / kQ;
    const dim3 grid(nblocks(waves * 64, T));
    if (D == 3)
      hipLaunchKernelGGL((k_apply_packed<kFluxFaces3, kFluxRounds3>), grid, dim3(T), 0, st, pk, n_face, row_ptr, col,
                         val, phi, flux);
    else
      hipLaunchKernelGGL((k_apply_packed<kFluxFaces2, kFluxRounds2>), grid, dim3(T), 0, st, pk, n_face, row_ptr, col,
                         val, phi, flux);
    CC_HIP(hipGetLastError());
  }
  return divergence(D, n_vol, vol_face, vol_scale, flux, lphi, st);
}

}  // namespace cutcell
