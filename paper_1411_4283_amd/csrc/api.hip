// Host entry points of the C ABI declared in include/cutcell.h.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "solve.hpp"
#include "scan.hpp"

namespace cutcell {

static thread_local std::string g_last_error;

// ---- optional per-phase timing of cutcell_build_stencils (hipEvents on its stream) ------
constexpr int kPhases = 6;   // enumerate, count+scan, fill, bin, solve, tables
static thread_local bool g_profiling = false;
static thread_local double g_phase_ms[kPhases] = {-1, -1, -1, -1, -1, -1};
static thread_local int64_t g_last_reused = 0;
static thread_local int64_t g_last_qr = 0;
static thread_local int64_t g_last_bins[kMaxBins] = {0, 0, 0, 0, 0, 0, 0, 0};

struct PhaseTimer {
  hipEvent_t ev[kPhases + 1];
  int n = 0;
  bool on;
  hipStream_t st;
  PhaseTimer(hipStream_t s, bool allowed = true) : on(g_profiling && allowed), st(s) {
    if (!on) return;
    for (int i = 0; i <= kPhases; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) on = false;
  }
  void mark() {
    if (on && n <= kPhases) (void)hipEventRecord(ev[n++], st);
  }
  void finish() {
    if (!on) return;
    (void)hipEventSynchronize(ev[n - 1]);
    for (int i = 0; i < kPhases; ++i) {
      float ms = 0.f;
      g_phase_ms[i] = (i + 1 < n && hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) ? ms : -1.0;
    }
  }
  ~PhaseTimer() {
    if (!on) return;
    for (int i = 0; i <= kPhases; ++i) (void)hipEventDestroy(ev[i]);
  }
};

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// ---- the static scratch of cutcell_build_stencils_noalloc ---------------------------------
// One array per GPU, in this file's code object (the runtime places it on every device when
// the library is loaded).  In host code `scratch` is only a stand-in for the symbol: its
// device address comes from hipGetSymbolAddress, once per device with that device current,
// and is what kernels and copies are given.
constexpr size_t kStaticScratchBytes = CUTCELL_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static int static_scratch(void** out) {
  static std::mutex mu;
  static std::vector<void*> ptrs;   // device address of `scratch`, per device
  int dev = 0;
  CC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* p = nullptr;
    CC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(CUTCELL_E_HIP, "hipGetSymbolAddress returned no address for the static scratch");
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return CUTCELL_OK;
}

size_t layout_work(const cutcell_opts& o, int G, char* base, Work* w) {
  Work t{};
  t.dims = make_dims(o);
  t.G = G;
  const GridDims& g = t.dims;
  t.L = g.ncell + g.nboxslot + g.NF;
  t.maxface = g.NF + g.ncell;
  const long long tilesL = scan_tiles(t.L);
  const long long totface = (long long)G * t.maxface;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  t.flags = (int32_t*)take(sizeof(int32_t) * G * t.L);
  t.excl = (int32_t*)take(sizeof(int32_t) * G * t.L);
  t.seg_total = (int32_t*)take(sizeof(int32_t) * G);
  t.scan_tmp = (int32_t*)take(sizeof(int32_t) * G * tilesL);
  t.vol_id = (int32_t*)take(sizeof(int32_t) * G * g.ncell);
  t.eb_id = (int32_t*)take(sizeof(int32_t) * G * g.ncell);
  t.face_id = (int32_t*)take(sizeof(int32_t) * G * g.NF);
  t.box_id = (int32_t*)take(sizeof(int32_t) * G * g.NF);
  t.box_lf = (int32_t*)take(sizeof(int32_t) * G * std::max<long long>(g.nboxslot, 1));
  t.vol_cell = (int32_t*)take(sizeof(int32_t) * G * g.ncell);
  t.cellinfo = (uint8_t*)take(sizeof(uint8_t) * G * g.ncell);
  t.ballreg = (uint8_t*)take(sizeof(uint8_t) * G * g.ncell);
  t.ballreg_tmp = (uint8_t*)take(sizeof(uint8_t) * G * g.ncell);
  t.canon = (uint8_t*)take(sizeof(uint8_t) * G * g.ncell);
  t.ref_cell = (int32_t*)take(sizeof(int32_t) * G);
  t.tface = (int32_t*)take(sizeof(int32_t) * 3 * G);
  t.tmpl = (int32_t*)take(sizeof(int32_t) * totface);
  t.okey = (unsigned long long*)take(sizeof(unsigned long long) * totface);
  t.okey_out = (unsigned long long*)take(sizeof(unsigned long long) * totface);
  t.oval = (int32_t*)take(sizeof(int32_t) * totface);
  t.osort_bytes = order_temp_bytes(totface);
  t.osort_tmp = take(t.osort_bytes);
  t.counts = (int64_t*)take(sizeof(int64_t) * 4 * G);
  t.offs = (int64_t*)take(sizeof(int64_t) * 3 * (G + 1));
  t.fcode = (int32_t*)take(sizeof(int32_t) * totface);
  t.fref = (int32_t*)take(sizeof(int32_t) * totface);
  t.nrows = (int32_t*)take(sizeof(int32_t) * totface);
  t.scan64 = (int64_t*)take(sizeof(int64_t) * (scan_tiles(totface) + 1));
  t.rp_tmp = (int64_t*)take(sizeof(int64_t) * (totface + 1));
  t.perm = (int32_t*)take(sizeof(int32_t) * totface);
  t.bins = (int32_t*)take(sizeof(int32_t) * kBinWords);
  t.flagged = (int32_t*)take(sizeof(int32_t) * 2);
  t.qr_count = (int32_t*)take(sizeof(int32_t));
  t.qr_list = (int32_t*)take(sizeof(int32_t) * totface);
  {
    const int M = binom(o.order + o.dim, o.dim);
    t.qr_slots = (int)std::min<long long>(kQrSlots, std::max<long long>(totface, 1));
    t.qr_b = (double*)take(sizeof(double) * t.qr_slots * 2 * kMaxRows * (M | 1));
    // ballot masks of the neighbour window, (2R + 2)(2R + 1)^(D-1) cells, per face
    long long nw = 2 * o.path_radius + 2;
    for (int d = 1; d < o.dim; ++d) nw *= 2 * o.path_radius + 1;
    t.nbmask = (unsigned long long*)take(sizeof(unsigned long long) * totface * ((nw + 63) / 64));
  }
  t.geoms = (GeomPtrs*)take(sizeof(GeomPtrs) * G);
  t.bytes = off;
  if (w) *w = t;
  return off;
}

static int validate(const cutcell_geom* geoms, int G, const cutcell_opts* o) {
  if (!o) return fail(CUTCELL_E_INVALID_ARG, "opts is NULL");
  if (o->dim != 2 && o->dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (o->order != 2 && o->order != 4) return fail(CUTCELL_E_UNSUPPORTED, "order must be 2 or 4");
  if (o->path_radius < 1 || o->path_radius > 4) return fail(CUTCELL_E_UNSUPPORTED, "path_radius must be in [1, 4]");
  if (!(o->h > 0)) return fail(CUTCELL_E_INVALID_ARG, "h must be positive");
  if (o->weight_custom != 0 && o->weight_custom != 1)
    return fail(CUTCELL_E_INVALID_ARG, "weight_custom must be 0 or 1");
  if (o->weight_custom && !(o->weight_power >= 0.0 && o->weight_power <= 16.0))
    return fail(CUTCELL_E_INVALID_ARG, "weight_power must be in [0, 16]");
  if (o->reuse_templates != 0 && o->reuse_templates != 1)
    return fail(CUTCELL_E_INVALID_ARG, "reuse_templates must be 0 or 1");
  if (o->factorization != CUTCELL_FACTOR_AUTO && o->factorization != CUTCELL_FACTOR_QR &&
      o->factorization != CUTCELL_FACTOR_GRAM)
    return fail(CUTCELL_E_INVALID_ARG, "factorization must be CUTCELL_FACTOR_AUTO, _QR or _GRAM");
  if (o->eb_bc != CUTCELL_BC_DIRICHLET && o->eb_bc != CUTCELL_BC_NEUMANN)
    return fail(CUTCELL_E_INVALID_ARG, "eb_bc must be CUTCELL_BC_DIRICHLET or CUTCELL_BC_NEUMANN");
  if (o->tuning)
    for (int b = 0; b < kMaxBins; ++b)
      if (o->tuning->xcd_chunks[b] < 0 || o->tuning->xcd_chunks[b] > 64 || o->tuning->blocks_per_xcd[b] < 0 ||
          o->tuning->blocks_per_xcd[b] > (1 << 24))
        return fail(CUTCELL_E_INVALID_ARG, "tuning entries out of range");
  for (int d = 0; d < o->dim; ++d)
    if (o->n[d] < 1 || o->n[d] > (1 << 14)) return fail(CUTCELL_E_INVALID_ARG, "n[d] out of range");
  long long ncell = 1;
  for (int d = 0; d < o->dim; ++d) ncell *= o->n[d];
  if (G < 1 || G > (1 << 20)) return fail(CUTCELL_E_INVALID_ARG, "n_geom out of range");
  if ((long long)G * (ncell * 4 + 64) > (1LL << 31)) return fail(CUTCELL_E_UNSUPPORTED, "batch too large for 32-bit indices");
  if (!geoms) return fail(CUTCELL_E_INVALID_ARG, "geoms is NULL");
  for (int i = 0; i < G; ++i) {
    const cutcell_geom& g = geoms[i];
    if (!g.vol_mom) return fail(CUTCELL_E_INVALID_ARG, "vol_mom is NULL");
    for (int d = 0; d < o->dim; ++d)
      if (!g.face_mom[d]) return fail(CUTCELL_E_INVALID_ARG, "face_mom[d] is NULL");
    if (g.n_eb < 0 || g.n_eb > ncell) return fail(CUTCELL_E_INVALID_ARG, "n_eb out of range");
    if (g.n_eb > 0 && (!g.eb_cell || !g.eb_mom || !g.eb_nmom)) return fail(CUTCELL_E_INVALID_ARG, "EB arrays are NULL");
  }
  return CUTCELL_OK;
}

// EB cells must be strictly ascending, inside the grid and in volumes (checked on the
// device before anything indexes with them)
__global__ void k_check_eb(int G, long long ncell, int M, const GeomPtrs* __restrict__ geoms, int32_t* bad) {
  const int gi = blockIdx.y;
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const GeomPtrs gp = geoms[gi];
  if (e >= gp.n_eb) return;
  const int32_t c = gp.eb_cell[e];
  bool ok = c >= 0 && c < ncell;
  if (ok && e > 0) ok = gp.eb_cell[e - 1] < c;
  if (ok) ok = gp.vol_mom[(long long)c * M] > 0.0;
  if (!ok) atomicOr(bad, 1);
}

struct Prepared {
  Work w;
  std::vector<int64_t> counts, offs;
  int64_t n_vol = 0, n_eb = 0, n_box = 0, n_phi = 0, n_face = 0;
};

static int prepare(const cutcell_geom* geoms, int G, const cutcell_opts* o, void* ws, size_t ws_bytes, hipStream_t st,
                   Prepared* P) {
  int rc = validate(geoms, G, o);
  if (rc) return rc;
  const size_t need = layout_work(*o, G, nullptr, nullptr);
  if (!ws || ws_bytes < need)
    return fail(CUTCELL_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  layout_work(*o, G, (char*)ws, &P->w);
  const Work& w = P->w;
  std::vector<GeomPtrs> gp(G);
  for (int i = 0; i < G; ++i) {
    gp[i].vol_mom = geoms[i].vol_mom;
    for (int d = 0; d < 3; ++d) gp[i].face_mom[d] = (d < o->dim) ? geoms[i].face_mom[d] : nullptr;
    gp[i].eb_cell = geoms[i].eb_cell;
    gp[i].eb_mom = geoms[i].eb_mom;
    gp[i].eb_nmom = geoms[i].eb_nmom;
    gp[i].n_eb = geoms[i].n_eb;
  }
  CC_HIP(hipMemcpyAsync(w.geoms, gp.data(), sizeof(GeomPtrs) * G, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.flagged, 2LL, 0);
  const int M = binom(o->order + o->dim, o->dim);
  int maxeb = 0;
  for (int i = 0; i < G; ++i) maxeb = std::max(maxeb, geoms[i].n_eb);
  if (maxeb > 0)
    hipLaunchKernelGGL(k_check_eb, dim3((unsigned)((maxeb + 255) / 256), G), dim3(256), 0, st, G, w.dims.ncell, M,
                       w.geoms, w.flagged + 1);
  rc = enumerate_batch(w, *o, st);
  if (rc) return rc;
  P->counts.assign(4 * G, 0);
  P->offs.assign(3 * (G + 1), 0);
  int32_t bad = 0;
  CC_HIP(hipMemcpyAsync(P->counts.data(), w.counts, sizeof(int64_t) * 4 * G, hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(P->offs.data(), w.offs, sizeof(int64_t) * 3 * (G + 1), hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(&bad, w.flagged + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (bad) return fail(CUTCELL_E_INVALID_ARG, "eb_cell must be strictly ascending cells with kappa > 0");
  for (int i = 0; i < G; ++i) {
    P->n_vol += P->counts[4 * i + 0];
    P->n_eb += P->counts[4 * i + 1];
    P->n_box += P->counts[4 * i + 2];
  }
  P->n_phi = P->offs[G];
  P->n_face = P->offs[2 * (G + 1) + G];
  if (P->n_phi >= (1LL << 31)) return fail(CUTCELL_E_UNSUPPORTED, "more than 2^31 Phi rows");
  return CUTCELL_OK;
}

// counts rows per face, scans them into row_ptr (int64); returns nnz and max rows
static int count_rows(const Prepared& P, const cutcell_opts* o, int64_t* row_ptr, int64_t* nnz, int32_t* maxrows,
                      hipStream_t st) {
  const Work& w = P.w;
  int rc = neighbour_rows(w, *o, P.n_face, nullptr, nullptr, false, st);
  if (rc) return rc;
  rc = max_rows(w, P.n_face, st);
  if (rc) return rc;
  int64_t total = 0;
  if (P.n_face > 0) {
    rc = exclusive_scan<int32_t, int64_t>(w.nrows, P.n_face, P.n_face, 1, row_ptr, P.n_face, row_ptr ? row_ptr + P.n_face : nullptr,
                                          w.scan64, st);
    if (rc) return rc;
  }
  int32_t mr = 0;
  const int64_t zero = 0;
  CC_HIP(hipMemcpyAsync(&mr, w.bins + 2 * kNBuckets, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (row_ptr && P.n_face > 0)
    CC_HIP(hipMemcpyAsync(&total, row_ptr + P.n_face, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  else if (row_ptr)   // no faces: row_ptr = [0]
    CC_HIP(hipMemcpyAsync(row_ptr, &zero, sizeof(int64_t), hipMemcpyHostToDevice, st));
  CC_HIP(hipStreamSynchronize(st));
  *nnz = total;
  *maxrows = mr;
  return CUTCELL_OK;
}


// Scratch of cutcell_stencils_backward after the forward workspace.
struct BackWork {
  GradPtrs* grads;     // [G]
  double* face_yw;     // [n_face][2M]
  double* face_x0;     // [n_face][4]
  double* owner_grad;  // [n_face][4]
  double* nz_rz;       // [nnz][2]
  size_t bytes;
};

static size_t layout_backward(const cutcell_opts& o, int G, long long n_face, long long nnz, char* base, BackWork* b) {
  const int M = binom(o.order + o.dim, o.dim);
  size_t off = layout_work(o, G, nullptr, nullptr);
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  BackWork t{};
  t.grads = (GradPtrs*)take(sizeof(GradPtrs) * G);
  t.face_yw = (double*)take(sizeof(double) * 2 * M * std::max<long long>(n_face, 1));
  t.face_x0 = (double*)take(sizeof(double) * 4 * std::max<long long>(n_face, 1));
  t.owner_grad = (double*)take(sizeof(double) * 4 * std::max<long long>(n_face, 1));
  t.nz_rz = (double*)take(sizeof(double) * 2 * std::max<long long>(nnz, 1));
  t.bytes = off;
  if (b) *b = t;
  return off;
}

static void fill_zero(double* p, long long n, hipStream_t st) {
  if (p && n > 0) hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, 0.0);
}

static bool stencils_complete(const cutcell_stencils* s) {
  return s && s->row_ptr && s->col && s->val && s->status && s->vol_face && s->vol_scale;
}

static bool transpose_complete(const cutcell_transpose* t) { return t && t->col_ptr && t->nz && t->nz_face; }

}  // namespace cutcell

using namespace cutcell;

extern "C" {

size_t cutcell_workspace_bytes(const cutcell_opts* opts, int32_t n_geom) {
  if (!opts || n_geom < 1 || (opts->dim != 2 && opts->dim != 3)) return 0;
  return layout_work(*opts, n_geom, nullptr, nullptr);
}

int cutcell_query(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts, void* workspace,
                  size_t workspace_bytes, cutcell_sizes* sizes, cutcell_stream_t stream) {
  if (!sizes) return fail(CUTCELL_E_INVALID_ARG, "sizes is NULL");
  hipStream_t st = (hipStream_t)stream;
  Prepared P;
  int rc = prepare(geoms, n_geom, opts, workspace, workspace_bytes, st, &P);
  if (rc) return rc;
  int64_t nnz = 0;
  int32_t mr = 0;
  rc = count_rows(P, opts, P.w.rp_tmp, &nnz, &mr, st);
  if (rc) return rc;
  sizes->n_vol = P.n_vol;
  sizes->n_eb = P.n_eb;
  sizes->n_box = P.n_box;
  sizes->n_phi = P.n_phi;
  sizes->n_face = P.n_face;
  sizes->nnz = nnz;
  sizes->max_rows = mr;
  sizes->n_geom = n_geom;
  if (mr > kMaxRows)
    return fail(CUTCELL_E_UNSUPPORTED, "a face has " + std::to_string(mr) + " rows; at most " +
                                           std::to_string(kMaxRows) + " are supported");
  return CUTCELL_OK;
}

static int build_common(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                        const cutcell_sizes* sizes, cutcell_stencils* out, void* workspace, size_t workspace_bytes,
                        cutcell_stream_t stream, cutcell_tuning* tune_out, int reps, double* best_ms,
                        bool timing_allowed = true) {
  if (!sizes || !out) return fail(CUTCELL_E_INVALID_ARG, "sizes/out is NULL");
  if (!out->row_ptr || !out->col || !out->val || !out->status || !out->vol_face || !out->vol_scale ||
      !out->phi_off || !out->vol_off || !out->face_off)
    return fail(CUTCELL_E_INVALID_ARG, "an output array is NULL");
  hipStream_t st = (hipStream_t)stream;
  PhaseTimer timer(st, timing_allowed);
  timer.mark();
  Prepared P;
  int rc = prepare(geoms, n_geom, opts, workspace, workspace_bytes, st, &P);
  if (rc) return rc;
  timer.mark();
  if (sizes->n_geom != n_geom || sizes->n_face != P.n_face || sizes->n_vol != P.n_vol || sizes->n_phi != P.n_phi)
    return fail(CUTCELL_E_CAPACITY, "sizes do not match these inputs (call cutcell_query first)");
  const Work& w = P.w;
  int64_t nnz = 0;
  int32_t mr = 0;
  rc = count_rows(P, opts, out->row_ptr, &nnz, &mr, st);
  if (rc) return rc;
  timer.mark();
  if (nnz != sizes->nnz) return fail(CUTCELL_E_CAPACITY, "nnz differs from sizes->nnz");
  if (mr > kMaxRows)
    return fail(CUTCELL_E_UNSUPPORTED, "a face has " + std::to_string(mr) + " rows; at most " +
                                           std::to_string(kMaxRows) + " are supported");
  rc = neighbour_rows(w, *opts, P.n_face, out->row_ptr, out->col, true, st);
  if (rc) return rc;
  timer.mark();
  const int M = binom(opts->order + opts->dim, opts->dim);
  if (opts->reuse_templates) {
    rc = find_templates(w, *opts, P.n_face, st);
    if (rc) return rc;
  }
  rc = bin_faces(w, P.n_face, M, opts->reuse_templates ? w.tmpl : nullptr, st);
  if (rc) return rc;
  timer.mark();
  int32_t bc[kBinWords];
  CC_HIP(hipMemcpyAsync(bc, w.bins, sizeof(bc), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  g_last_reused = bc[kMaxBins + 1];
  for (int b = 0; b < kMaxBins; ++b) g_last_bins[b] = bc[b];
  if (tune_out) {
    double bm[kMaxBins];
    rc = tune_stencils(w, *opts, bc, out->row_ptr, out->col, out->val, out->status, st, tune_out, reps, bm);
    if (best_ms)
      for (int b = 0; b < kMaxBins; ++b) best_ms[b] = bm[b];
  } else {
    rc = solve_stencils(w, *opts, bc, P.n_face, out->row_ptr, out->col, out->val, out->status, st);
  }
  if (rc) return rc;
  timer.mark();
  rc = volume_tables(w, *opts, P.n_vol, out->vol_face, out->vol_scale, st);
  if (rc) return rc;
  if (out->tmpl && P.n_face > 0) {   // each face's template, -1 where it was solved itself
    if (opts->reuse_templates)
      CC_HIP(hipMemcpyAsync(out->tmpl, w.tmpl, sizeof(int32_t) * P.n_face, hipMemcpyDeviceToDevice, st));
    else
      hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((P.n_face + 255) / 256)), dim3(256), 0, st, out->tmpl, P.n_face,
                         -1);
  }
  timer.mark();
  const size_t ob = sizeof(int64_t) * (n_geom + 1);
  CC_HIP(hipMemcpyAsync(out->phi_off, w.offs, ob, hipMemcpyDeviceToDevice, st));
  CC_HIP(hipMemcpyAsync(out->vol_off, w.offs + (n_geom + 1), ob, hipMemcpyDeviceToDevice, st));
  CC_HIP(hipMemcpyAsync(out->face_off, w.offs + 2 * (n_geom + 1), ob, hipMemcpyDeviceToDevice, st));
  int32_t flagged = 0, nqr = 0;
  CC_HIP(hipMemcpyAsync(&flagged, w.flagged, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipMemcpyAsync(&nqr, w.qr_count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  CC_HIP(hipGetLastError());
  g_last_qr = nqr;
  timer.finish();
  return flagged ? CUTCELL_W_FLAGGED_FACES : CUTCELL_OK;
}

int cutcell_build_stencils(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                           const cutcell_sizes* sizes, cutcell_stencils* out, void* workspace, size_t workspace_bytes,
                           cutcell_stream_t stream) {
  return build_common(geoms, n_geom, opts, sizes, out, workspace, workspace_bytes, stream, nullptr, 0, nullptr);
}

int cutcell_build_stencils_noalloc(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                                   const cutcell_sizes* sizes, cutcell_stencils* out, cutcell_stream_t stream) {
  int rc = validate(geoms, n_geom, opts);
  if (rc) return rc;
  const size_t need = layout_work(*opts, n_geom, nullptr, nullptr);
  if (need > kStaticScratchBytes)
    return fail(CUTCELL_E_WORKSPACE, "the build needs " + std::to_string(need) + " bytes of scratch; the static " +
                                         "scratch holds " + std::to_string(kStaticScratchBytes));
  void* ws = nullptr;
  rc = static_scratch(&ws);
  if (rc) return rc;
  return build_common(geoms, n_geom, opts, sizes, out, ws, kStaticScratchBytes, stream, nullptr, 0, nullptr, false);
}

int cutcell_autotune(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts, const cutcell_sizes* sizes,
                     cutcell_stencils* out, void* workspace, size_t workspace_bytes, int32_t reps,
                     cutcell_tuning* tuning, double* best_ms, cutcell_stream_t stream) {
  if (!tuning) return fail(CUTCELL_E_INVALID_ARG, "tuning is NULL");
  if (reps < 1 || reps > 100) return fail(CUTCELL_E_INVALID_ARG, "reps must be in [1, 100]");
  if (!opts) return fail(CUTCELL_E_INVALID_ARG, "opts is NULL");
  cutcell_opts o = *opts;
  o.tuning = nullptr;
  return build_common(geoms, n_geom, &o, sizes, out, workspace, workspace_bytes, stream, tuning, reps, best_ms);
}

void cutcell_set_profiling(int enable) { g_profiling = enable != 0; }

int64_t cutcell_last_reused_faces(void) { return g_last_reused; }

int cutcell_last_bin_faces(int64_t* counts, int32_t n) {
  if (!counts || n < 0) return fail(CUTCELL_E_INVALID_ARG, "counts is NULL");
  for (int b = 0; b < n && b < kMaxBins; ++b) counts[b] = g_last_bins[b];
  return kMaxBins;
}

int64_t cutcell_last_qr_faces(void) { return g_last_qr; }

int cutcell_last_profile(double* ms, int32_t n) {
  if (!ms || n < 0) return fail(CUTCELL_E_INVALID_ARG, "ms is NULL");
  for (int i = 0; i < n && i < kPhases; ++i) ms[i] = g_phase_ms[i];
  return kPhases;
}

int cutcell_apply(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_, const double* phi,
                  double* lphi, double* flux, cutcell_stream_t stream) {
  if (!sizes) return fail(CUTCELL_E_INVALID_ARG, "sizes is NULL");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (sizes->n_vol == 0 && sizes->n_face == 0) return CUTCELL_OK;   // nothing to apply (arrays may be NULL)
  if (!st_ || !phi || !lphi || !flux) return fail(CUTCELL_E_INVALID_ARG, "NULL argument (flux is required)");
  if (!st_->row_ptr || !st_->col || !st_->val || !st_->vol_face || !st_->vol_scale)
    return fail(CUTCELL_E_INVALID_ARG, "stencil arrays are NULL");
  return apply_operator(dim, sizes->n_face, sizes->n_vol, st_->row_ptr, st_->col, st_->val, st_->vol_face,
                        st_->vol_scale, phi, lphi, flux, nullptr, (hipStream_t)stream);
}

size_t cutcell_solve_workspace_bytes(const cutcell_sizes* sizes, int32_t restart) {
  if (!sizes || restart < 1 || restart > 1024 || sizes->n_vol < 0 || sizes->n_phi < 0 || sizes->n_face < 0) return 0;
  return solve_workspace_bytes(sizes->n_vol, sizes->n_phi, sizes->n_face, restart);
}

size_t cutcell_pack_workspace_bytes(const cutcell_sizes* sizes) {
  if (!sizes || sizes->n_face < 0 || sizes->n_face >= (1LL << 31)) return 0;
  return pack_temp_bytes(sizes->n_face);
}

int cutcell_pack_count(const cutcell_sizes* sizes, const cutcell_stencils* st_, cutcell_packed_sizes* out,
                       void* workspace, size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !out) return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (sizes->n_face < 0 || sizes->n_face >= (1LL << 31)) return fail(CUTCELL_E_INVALID_ARG, "bad sizes");
  long long np = 0;
  int ns = 0, mr = 0, mw = 0;
  if (sizes->n_face > 0) {
    if (!st_ || !st_->row_ptr || !st_->col || !st_->val || !st_->tmpl || !workspace)
      return fail(CUTCELL_E_INVALID_ARG, "NULL argument (the stencils need their tmpl array)");
    const int rc = pack_count(sizes->n_face, st_->row_ptr, st_->col, st_->val, st_->tmpl, (char*)workspace,
                              workspace_bytes, &np, &ns, &mr, &mw, (hipStream_t)stream);
    if (rc) return rc;
  }
  out->n_packed = np;
  out->n_slot = ns;
  out->max_runs = mr;
  out->max_rows = mw;
  return CUTCELL_OK;
}

int cutcell_pack_fill(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_,
                      const cutcell_packed_sizes* psizes, cutcell_packed* out, void* workspace,
                      size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !psizes || !out) return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (sizes->n_face < 0 || sizes->n_face >= (1LL << 31)) return fail(CUTCELL_E_INVALID_ARG, "bad sizes");
  if (psizes->n_packed < 0 || psizes->n_packed > sizes->n_face)
    return fail(CUTCELL_E_CAPACITY, "packed sizes do not match these stencils (call cutcell_pack_count first)");
  if (sizes->n_face == 0) return CUTCELL_OK;
  if (!st_ || !st_->row_ptr || !st_->col || !st_->val || !st_->tmpl || !workspace || !out->flag || !out->phase)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument (the stencils need their tmpl array)");
  if (psizes->n_packed > 0 && (!out->face || !out->slot || !out->base))
    return fail(CUTCELL_E_INVALID_ARG, "packed face arrays are NULL");
  if (psizes->n_slot > 0 && (!out->slot_face || !out->slot_rows || !out->slot_tab || !out->slot_val))
    return fail(CUTCELL_E_INVALID_ARG, "slot arrays are NULL");
  PackedSizes ps{psizes->n_packed, psizes->n_slot, psizes->max_runs, psizes->max_rows};
  PackedOut o{out->flag, out->phase, out->face, out->slot, out->base, out->slot_face, out->slot_rows, out->slot_tab,
              out->slot_val};
  return pack_fill(dim, sizes->n_face, st_->row_ptr, st_->col, st_->val, st_->tmpl, (char*)workspace,
                   workspace_bytes, ps, o, (hipStream_t)stream);
}

int cutcell_apply_packed(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_,
                         const cutcell_packed_sizes* psizes, const cutcell_packed* pk, const double* phi, double* lphi,
                         double* flux, cutcell_stream_t stream) {
  if (!sizes || !psizes) return fail(CUTCELL_E_INVALID_ARG, "sizes is NULL");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (sizes->n_vol == 0 && sizes->n_face == 0) return CUTCELL_OK;   // nothing to apply (arrays may be NULL)
  if (!st_ || !phi || !lphi || !flux || !pk || !pk->flag || !pk->phase)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (!st_->row_ptr || !st_->col || !st_->val || !st_->vol_face || !st_->vol_scale)
    return fail(CUTCELL_E_INVALID_ARG, "stencil arrays are NULL");
  if (psizes->n_packed < 0 || psizes->n_packed > sizes->n_face ||
      (psizes->n_packed > 0 && (!pk->face || !pk->slot || !pk->base || !pk->slot_rows || !pk->slot_tab ||
                                !pk->slot_val || psizes->max_runs < 1 || psizes->max_rows < 1 || psizes->n_slot < 1)))
    return fail(CUTCELL_E_INVALID_ARG, "packed arrays or sizes are inconsistent");
  PackedArgs a;
  a.n_packed = psizes->n_packed;
  a.n_slot = psizes->n_slot;
  a.max_runs = psizes->max_runs;
  a.max_rows = psizes->max_rows;
  a.flag = pk->flag;
  a.phase = pk->phase;
  a.face = pk->face;
  a.slot = pk->slot;
  a.base = pk->base;
  a.slot_rows = pk->slot_rows;
  a.slot_tab = pk->slot_tab;
  a.slot_val = pk->slot_val;
  return apply_packed(dim, sizes->n_face, sizes->n_vol, st_->row_ptr, st_->col, st_->val, st_->vol_face,
                      st_->vol_scale, a, phi, lphi, flux, (hipStream_t)stream);
}

size_t cutcell_laplacian_workspace_bytes(const cutcell_sizes* sizes) {
  if (!sizes || sizes->n_vol < 0) return 0;
  return laplacian_temp_bytes(sizes->n_vol);
}

int cutcell_laplacian_count(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_, int64_t* row_ptr,
                            int64_t* nnz, void* workspace, size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !row_ptr || !nnz || !workspace)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (sizes->n_vol < 0 || sizes->n_vol >= (1LL << 31)) return fail(CUTCELL_E_INVALID_ARG, "bad sizes");
  return laplacian_count(dim, sizes->n_vol, st_->row_ptr, st_->col, st_->val, st_->vol_face, st_->vol_scale, row_ptr,
                         nnz, (char*)workspace, workspace_bytes, (hipStream_t)stream);
}

int cutcell_laplacian_fill(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_,
                           const cutcell_laplacian* lap, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !lap || !lap->row_ptr || !lap->col || !lap->val)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  return laplacian_fill(dim, sizes->n_vol, st_->row_ptr, st_->col, st_->val, st_->vol_face, st_->vol_scale,
                        lap->row_ptr, lap->col, lap->val, (hipStream_t)stream);
}

int cutcell_apply_laplacian(const cutcell_sizes* sizes, int32_t dim, const cutcell_laplacian* lap, const double* phi,
                            double* lphi, cutcell_stream_t stream) {
  if (!sizes) return fail(CUTCELL_E_INVALID_ARG, "sizes is NULL");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (sizes->n_vol == 0) return CUTCELL_OK;   // nothing to apply (arrays may be NULL)
  if (!lap || !lap->row_ptr || !lap->col || !lap->val || !phi || !lphi)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  return apply_laplacian(dim, sizes->n_vol, lap->row_ptr, lap->col, lap->val, phi, lphi, (hipStream_t)stream);
}

int cutcell_solve(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_, const cutcell_laplacian* lap,
                  const double* phi_bc, const double* rhs, double* x, int32_t restart, int32_t max_iters, double rtol,
                  void* workspace, size_t workspace_bytes, int32_t* iters, double* relres, cutcell_stream_t stream) {
  if (!sizes) return fail(CUTCELL_E_INVALID_ARG, "sizes is NULL");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (restart < 1 || restart > 1024) return fail(CUTCELL_E_INVALID_ARG, "restart must be in [1, 1024]");
  if (max_iters < 0) return fail(CUTCELL_E_INVALID_ARG, "max_iters must be >= 0");
  if (!(rtol >= 0.0)) return fail(CUTCELL_E_INVALID_ARG, "rtol must be >= 0");
  if (sizes->n_vol == 0) {   // nothing to solve (arrays may be NULL)
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return CUTCELL_OK;
  }
  if (!stencils_complete(st_) || !st_->phi_off || !st_->vol_off || !phi_bc || !rhs || !x || !workspace)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (sizes->n_geom < 1 || sizes->n_vol < 0 || sizes->n_phi >= (1LL << 31))
    return fail(CUTCELL_E_INVALID_ARG, "bad sizes");
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  if (sizes->n_vol == 0) return CUTCELL_OK;
  SolveOp op{dim, sizes->n_vol, sizes->n_phi, sizes->n_face, st_->row_ptr, st_->col, st_->val, st_->vol_face,
             st_->vol_scale, (hipStream_t)stream};
  if (lap) {
    if (!lap->row_ptr || !lap->col || !lap->val) return fail(CUTCELL_E_INVALID_ARG, "lap arrays are NULL");
    op.lap_ptr = lap->row_ptr;
    op.lap_col = lap->col;
    op.lap_val = lap->val;
  }
  int it = 0;
  const int rc = solve_poisson(op, sizes->n_geom, st_->phi_off, st_->vol_off, phi_bc, rhs, x, restart, max_iters,
                               rtol, (char*)workspace, workspace_bytes, &it, relres);
  if (iters) *iters = it;
  return rc;
}

int cutcell_hessenberg_eigs(int32_t n, const double* H, int32_t ld, double* re, double* im) {
  if (n < 0 || ld < n || (n > 0 && (!H || !re || !im))) return fail(CUTCELL_E_INVALID_ARG, "bad arguments");
  if (n > 4096) return fail(CUTCELL_E_UNSUPPORTED, "n must be at most 4096");
  if (hessenberg_eigs(n, H, ld, re, im)) return fail(CUTCELL_E_BREAKDOWN, "Hessenberg QR did not converge");
  return CUTCELL_OK;
}

size_t cutcell_ritz_workspace_bytes(const cutcell_sizes* sizes, int32_t steps, int32_t mode, int32_t inner_restart) {
  if (!sizes || steps < 1 || steps > 1024 || (mode != 0 && mode != 1) ||
      (mode == 1 && (inner_restart < 1 || inner_restart > 1024)))
    return 0;
  return ritz_workspace_bytes(sizes->n_vol, sizes->n_phi, sizes->n_face, steps, mode == 1 ? inner_restart : 0);
}

int cutcell_ritz(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_, const cutcell_laplacian* lap,
                 int32_t mode, int32_t steps, double inner_rtol, int32_t inner_restart, int32_t inner_max_iters,
                 double* ritz_re, double* ritz_im, double* ritz_res, int32_t* n_ritz, void* workspace,
                 size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !st_->phi_off || !st_->vol_off || !ritz_re || !ritz_im || !n_ritz ||
      !workspace)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  if (mode != 0 && mode != 1) return fail(CUTCELL_E_INVALID_ARG, "mode must be 0 or 1");
  if (steps < 1 || steps > 1024) return fail(CUTCELL_E_INVALID_ARG, "steps must be in [1, 1024]");
  if (mode == 1 && (inner_restart < 1 || inner_restart > 1024 || inner_max_iters < 1 || !(inner_rtol > 0.0)))
    return fail(CUTCELL_E_INVALID_ARG, "bad inner solve parameters");
  if (sizes->n_geom < 1 || sizes->n_vol < 1 || sizes->n_phi >= (1LL << 31)) return fail(CUTCELL_E_INVALID_ARG, "bad sizes");
  *n_ritz = 0;
  SolveOp op{dim, sizes->n_vol, sizes->n_phi, sizes->n_face, st_->row_ptr, st_->col, st_->val, st_->vol_face,
             st_->vol_scale, (hipStream_t)stream};
  if (lap) {
    if (!lap->row_ptr || !lap->col || !lap->val) return fail(CUTCELL_E_INVALID_ARG, "lap arrays are NULL");
    op.lap_ptr = lap->row_ptr;
    op.lap_col = lap->col;
    op.lap_val = lap->val;
  }
  int nr = 0;
  const int rc = ritz_values(op, sizes->n_geom, st_->phi_off, st_->vol_off, mode, steps, inner_rtol, inner_restart,
                             inner_max_iters, ritz_re, ritz_im, ritz_res, nullptr, &nr, (char*)workspace,
                             workspace_bytes);
  *n_ritz = nr;
  return rc;
}

size_t cutcell_transpose_workspace_bytes(const cutcell_sizes* sizes) {
  if (!sizes || sizes->nnz < 0 || sizes->nnz >= (1LL << 31)) return 0;
  return transpose_temp_bytes(sizes->nnz, sizes->n_phi);
}

int cutcell_build_transpose(const cutcell_sizes* sizes, const cutcell_stencils* st_, cutcell_transpose* out,
                            void* workspace, size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !transpose_complete(out))
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  if (sizes->nnz >= (1LL << 31)) return fail(CUTCELL_E_UNSUPPORTED, "the transpose needs nnz < 2^31");
  return build_transpose(sizes->n_face, sizes->n_phi, sizes->nnz, st_->row_ptr, st_->col, out->col_ptr, out->nz,
                         out->nz_face, (char*)workspace, workspace_bytes, (hipStream_t)stream);
}

int cutcell_apply_adjoint(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st_,
                          const cutcell_transpose* tr, const double* phi, const double* flux,
                          const double* lphi_bar, double* phi_bar, double* val_bar, double* scale_bar,
                          double* flux_bar, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !transpose_complete(tr) || !lphi_bar || !phi_bar || !flux_bar)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument (lphi_bar, phi_bar and flux_bar are required)");
  if (val_bar && !phi) return fail(CUTCELL_E_INVALID_ARG, "val_bar needs phi");
  if (scale_bar && !flux) return fail(CUTCELL_E_INVALID_ARG, "scale_bar needs the forward flux");
  if (dim != 2 && dim != 3) return fail(CUTCELL_E_UNSUPPORTED, "dim must be 2 or 3");
  Transpose t{tr->col_ptr, tr->nz, tr->nz_face};
  return apply_adjoint(dim, sizes->n_face, sizes->n_vol, sizes->n_phi, st_->row_ptr, st_->col, st_->val,
                       st_->vol_face, st_->vol_scale, t, phi, flux, lphi_bar, phi_bar, val_bar, scale_bar, flux_bar,
                       (hipStream_t)stream);
}

size_t cutcell_backward_workspace_bytes(const cutcell_opts* opts, const cutcell_sizes* sizes) {
  if (!opts || !sizes || sizes->n_geom < 1 || (opts->dim != 2 && opts->dim != 3) ||
      (opts->order != 2 && opts->order != 4))
    return 0;
  return layout_backward(*opts, sizes->n_geom, sizes->n_face, sizes->nnz, nullptr, nullptr);
}

int cutcell_stencils_backward(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                              const cutcell_sizes* sizes, const cutcell_stencils* st_, const cutcell_transpose* tr,
                              const double* val_bar, const double* scale_bar, const cutcell_geom_grad* grads,
                              double* weight_bar, void* workspace, size_t workspace_bytes, cutcell_stream_t stream) {
  if (!sizes || !stencils_complete(st_) || !transpose_complete(tr) || !val_bar || !grads)
    return fail(CUTCELL_E_INVALID_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = validate(geoms, n_geom, opts);
  if (rc) return rc;
  if (opts->eb_bc != CUTCELL_BC_DIRICHLET)
    return fail(CUTCELL_E_UNSUPPORTED, "the stencil adjoint supports Dirichlet EB conditions only");
  for (int i = 0; i < n_geom; ++i) {
    if (!grads[i].vol_mom) return fail(CUTCELL_E_INVALID_ARG, "grads[i].vol_mom is NULL");
    for (int d = 0; d < opts->dim; ++d)
      if (!grads[i].face_mom[d]) return fail(CUTCELL_E_INVALID_ARG, "grads[i].face_mom[d] is NULL");
    if (geoms[i].n_eb > 0 && (!grads[i].eb_mom || !grads[i].eb_nmom))
      return fail(CUTCELL_E_INVALID_ARG, "grads[i] EB arrays are NULL");
  }
  const size_t need = layout_backward(*opts, n_geom, sizes->n_face, sizes->nnz, nullptr, nullptr);
  if (!workspace || workspace_bytes < need)
    return fail(CUTCELL_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  Prepared P;
  rc = prepare(geoms, n_geom, opts, workspace, workspace_bytes, st, &P);
  if (rc) return rc;
  if (sizes->n_geom != n_geom || sizes->n_face != P.n_face || sizes->n_vol != P.n_vol || sizes->n_phi != P.n_phi)
    return fail(CUTCELL_E_CAPACITY, "sizes do not match these inputs");
  const Work& w = P.w;
  BackWork b;
  layout_backward(*opts, n_geom, sizes->n_face, sizes->nnz, (char*)workspace, &b);
  const int D = opts->dim, Q = opts->order;
  const int M = binom(Q + D, D), Mf = binom(Q + D - 1, D - 1), M1 = binom(Q - 1 + D, D);
  // every gradient starts at zero: cells without a volume, faces without a flux, ...
  std::vector<GradPtrs> gp(n_geom);
  for (int i = 0; i < n_geom; ++i) {
    const int64_t neb = geoms[i].n_eb;
    gp[i].vol_mom = grads[i].vol_mom;
    fill_zero(gp[i].vol_mom, w.dims.ncell * M, st);
    for (int d = 0; d < 3; ++d) {
      gp[i].face_mom[d] = (d < D) ? grads[i].face_mom[d] : nullptr;
      if (d < D) fill_zero(gp[i].face_mom[d], w.dims.nface[d] * Mf, st);
    }
    gp[i].eb_mom = grads[i].eb_mom;
    gp[i].eb_nmom = grads[i].eb_nmom;
    if (neb > 0) {
      fill_zero(gp[i].eb_mom, neb * M, st);
      fill_zero(gp[i].eb_nmom, neb * D * M1, st);
    }
  }
  CC_HIP(hipMemcpyAsync(b.grads, gp.data(), sizeof(GradPtrs) * n_geom, hipMemcpyHostToDevice, st));
  // bin the faces by their row counts again
  rc = rows_per_face(w, P.n_face, st_->row_ptr, st);
  if (rc) return rc;
  rc = max_rows(w, P.n_face, st);
  if (rc) return rc;
  rc = bin_faces(w, P.n_face, M, nullptr, st);
  if (rc) return rc;
  int32_t bc[kBinWords];
  CC_HIP(hipMemcpyAsync(bc, w.bins, sizeof(bc), hipMemcpyDeviceToHost, st));
  CC_HIP(hipStreamSynchronize(st));
  if (bc[2 * kNBuckets] > kMaxRows) return fail(CUTCELL_E_INVALID_ARG, "row_ptr does not come from a build");
  BackwardArgs ba{};
  ba.val_bar = val_bar;
  ba.face_yw = b.face_yw;
  ba.face_x0 = b.face_x0;
  ba.nz_rz = b.nz_rz;
  ba.weight_bar = weight_bar;
  ba.owner_grad = b.owner_grad;
  ba.grads = b.grads;
  ba.fwd_status = st_->status;
  rc = backward_stencils(w, *opts, bc, st_->row_ptr, st_->col, ba, st);
  if (rc) return rc;
  ReduceArgs R{};
  R.g = w.dims;
  R.G = n_geom;
  R.n_phi = P.n_phi;
  R.offs = w.offs;
  R.counts = w.counts;
  R.geoms = w.geoms;
  R.grads = b.grads;
  R.vol_cell_ws = w.vol_cell;
  R.box_lf_ws = w.box_lf;
  R.tr = Transpose{tr->col_ptr, tr->nz, tr->nz_face};
  R.face_yw = b.face_yw;
  R.face_x0 = b.face_x0;
  R.nz_rz = b.nz_rz;
  R.owner_grad = b.owner_grad;
  R.vol_face = st_->vol_face;
  R.vol_scale = st_->vol_scale;
  R.scale_bar = scale_bar;
  rc = reduce_moments(*opts, R, st);
  if (rc) return rc;
  CC_HIP(hipStreamSynchronize(st));
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

const char* cutcell_last_error(void) { return g_last_error.c_str(); }

int cutcell_abi_version(void) { return CUTCELL_ABI_VERSION; }

}  // extern "C"
