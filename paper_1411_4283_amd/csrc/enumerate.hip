// Enumeration of volumes, boundary faces and flux faces (Sec. 2.1), path-radius
// neighbour rows (Sec. 2.4) and row-count binning.
#include "kernels.hpp"
#include "scan.hpp"

namespace cutcell {

__global__ void k_fill_i32(int32_t* p, long long n, int32_t v) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double* p, long long n, double v) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// row counts of an existing CSR, for binning the faces again (the adjoint)
__global__ void k_rows_per_face(long long n_face, const int64_t* __restrict__ row_ptr, int32_t* __restrict__ nrows) {
  long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f < n_face) {
    const int64_t n = row_ptr[f + 1] - row_ptr[f];
    nrows[f] = (n < 0 || n > (int64_t)kMaxRows) ? kMaxRows + 1 : (int32_t)n;
  }
}

static inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// lattice face lf (in the concatenated lattice) -> direction and coordinates
__device__ __forceinline__ int lattice_dir(const GridDims& g, long long lf) {
  return (lf >= g.foff[1]) + (lf >= g.foff[2]);
}

// (32-bit arithmetic: a geometry's lattice has fewer than 2^31 faces, checked on entry)
__device__ __forceinline__ void lattice_coords(const GridDims& g, int d, long long lf, int* j) {
  const int loc = (int)(lf - g.foff[d]);
  const int m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
  j[0] = loc % m0;
  j[1] = (loc / m0) % m1;
  j[2] = loc / (m0 * m1);
}

__device__ __forceinline__ long long lattice_index(const GridDims& g, int d, const int* j) {
  int m0 = g.n[0] + (d == 0), m1 = g.n[1] + (d == 1);
  return g.foff[d] + j[0] + (long long)m0 * (j[1] + (long long)m1 * j[2]);
}

__device__ __forceinline__ long long cell_index(const GridDims& g, const int* i) {
  return i[0] + (long long)g.n[0] * (i[1] + (long long)g.n[1] * i[2]);
}

// box slot s (cells next to the box boundary, grouped by (d, side), ascending cell index
// inside a group) -> direction, side and the box face's lattice index
__device__ __forceinline__ long long box_slot_face(const GridDims& g, long long s, int* dd, int* side) {
  int k = 0;
  while (k < 5 && s >= g.boxoff[k + 1]) ++k;
  const int d = k / 2, sd = k % 2;
  long long t = s - g.boxoff[k];
  int a = (d == 0) ? 1 : 0;           // the two other directions, ascending
  int b = (d == 2) ? 1 : 2;
  int i[3] = {0, 0, 0};
  i[a] = (int)(t % g.n[a]);
  i[b] = (int)(t / g.n[a]);
  i[d] = sd ? g.n[d] : 0;             // lattice coordinate of the boundary face
  *dd = d;
  *side = sd;
  return lattice_index(g, d, i);
}

__global__ void k_enum_flags(GridDims g, int M, int Mf, const GeomPtrs* __restrict__ geoms, int32_t* flags,
                             long long L) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= L) return;
  const int gi = blockIdx.y;
  const GeomPtrs gp = geoms[gi];
  int32_t f = 0;
  if (i < g.ncell) {
    f = gp.vol_mom[i * M] > 0.0;
  } else if (i < g.ncell + g.nboxslot) {
    int d, side;
    long long lf = box_slot_face(g, i - g.ncell, &d, &side);
    f = gp.face_mom[d][(lf - g.foff[d]) * Mf] > 0.0;
  } else {
    long long lf = i - g.ncell - g.nboxslot;
    int d = lattice_dir(g, lf);
    f = gp.face_mom[d][(lf - g.foff[d]) * Mf] > 0.0;
  }
  flags[gi * L + i] = f;
}

__global__ void k_enum_counts(GridDims g, int G, long long L, const int32_t* __restrict__ excl,
                              const int32_t* __restrict__ seg_total, const GeomPtrs* __restrict__ geoms,
                              int64_t* counts, int64_t* offs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t* phi_off = offs;
  int64_t* vol_off = offs + (G + 1);
  int64_t* face_off = offs + 2 * (G + 1);
  phi_off[0] = vol_off[0] = face_off[0] = 0;
  for (int gi = 0; gi < G; ++gi) {
    const int32_t* e = excl + gi * L;
    int64_t n_vol = e[g.ncell];
    int64_t n_box = (int64_t)e[g.ncell + g.nboxslot] - e[g.ncell];
    int64_t n_gface = (int64_t)seg_total[gi] - e[g.ncell + g.nboxslot];
    int64_t n_eb = geoms[gi].n_eb;
    counts[4 * gi + 0] = n_vol;
    counts[4 * gi + 1] = n_eb;
    counts[4 * gi + 2] = n_box;
    counts[4 * gi + 3] = n_gface;
    phi_off[gi + 1] = phi_off[gi] + n_vol + n_eb + n_box;
    vol_off[gi + 1] = vol_off[gi] + n_vol;
    face_off[gi + 1] = face_off[gi] + n_gface + n_eb;
  }
}

__global__ void k_enum_maps(GridDims g, int G, long long L, long long maxface, const int32_t* __restrict__ flags,
                            const int32_t* __restrict__ excl, const int64_t* __restrict__ offs, int32_t* vol_id,
                            int32_t* vol_cell, int32_t* box_id, int32_t* box_lf, int32_t* face_id, int32_t* fcode,
                            int32_t* fref) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= L) return;
  const int gi = blockIdx.y;
  const int32_t f = flags[gi * L + i];
  const int32_t e = excl[gi * L + i];
  if (i < g.ncell) {
    vol_id[gi * g.ncell + i] = f ? e : -1;
    if (f) vol_cell[gi * g.ncell + e] = (int32_t)i;
  } else if (i < g.ncell + g.nboxslot) {
    if (!f) return;
    int d, side;
    long long lf = box_slot_face(g, i - g.ncell, &d, &side);
    int32_t b = e - excl[gi * L + g.ncell];
    box_id[gi * g.NF + lf] = b;
    box_lf[gi * g.nboxslot + b] = (int32_t)lf;
  } else {
    long long lf = i - g.ncell - g.nboxslot;
    int32_t loc = f ? e - excl[gi * L + g.ncell + g.nboxslot] : -1;
    face_id[gi * g.NF + lf] = loc;
    if (f) {
      long long F = offs[2 * (G + 1) + gi] + loc;
      fcode[F] = face_code(gi, 0, lattice_dir(g, lf));
      fref[F] = (int32_t)lf;
    }
  }
}

__global__ void k_enum_eb(GridDims g, int G, const GeomPtrs* __restrict__ geoms, const int64_t* __restrict__ counts,
                          const int64_t* __restrict__ offs, int32_t* eb_id, int32_t* fcode, int32_t* fref) {
  const int gi = blockIdx.y;
  long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const GeomPtrs gp = geoms[gi];
  if (e >= gp.n_eb) return;
  int32_t c = gp.eb_cell[e];
  if (c < 0 || c >= g.ncell) return;   // rejected by the argument check; never index with it
  eb_id[gi * g.ncell + c] = (int32_t)e;
  long long F = offs[2 * (G + 1) + gi] + counts[4 * gi + 3] + e;
  fcode[F] = face_code(gi, 1, 0);
  fref[F] = (int32_t)e;
}

// one byte per cell for the neighbour search: bit 0 volume, bit 1 + 2d + s the grid face
// on side s (0 low, 1 high) of direction d has alpha > 0, bit 7 the cell has an EB face
__global__ void k_cellinfo(GridDims g, const int32_t* __restrict__ vol_id, const int32_t* __restrict__ eb_id,
                           const int32_t* __restrict__ face_id, uint8_t* __restrict__ info) {
  const int gi = blockIdx.y;
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const long long o = (long long)gi * g.ncell + c;
  unsigned v = vol_id[o] >= 0 ? 1u : 0u;
  if (v) {
    int x[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    for (int d = 0; d < g.D; ++d)
      for (int s = 0; s < 2; ++s) {
        int j[3] = {x[0], x[1], x[2]};
        j[d] += s;
        if (face_id[(long long)gi * g.NF + lattice_index(g, d, j)] >= 0) v |= 1u << (1 + 2 * d + s);
      }
    if (eb_id[o] >= 0) v |= 0x80u;
  }
  info[o] = (uint8_t)v;
}

// Regular cells for the neighbour fast path: reg0 = a volume without an EB face whose 2D
// faces are all flux faces and which does not touch the box boundary; then R erosions,
// reg_{k+1}(c) = reg_k(c) and reg_k of its 2D neighbours, so reg_R(c) = 1 iff every cell
// within L1 distance R of c is regular.  For such cells the path-distance ball of radius
// R is the L1 ball and touches no EB or box face.
__global__ void k_regular0(GridDims g, const uint8_t* __restrict__ info, uint8_t* __restrict__ reg) {
  const int gi = blockIdx.y;
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const long long o = (long long)gi * g.ncell + c;
  const unsigned full = (1u << (1 + 2 * g.D)) - 1u;   // volume bit and all open-face bits
  bool r = info[o] == full;
  const int x[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  for (int d = 0; d < g.D; ++d) r = r && x[d] >= 1 && x[d] <= g.n[d] - 2;
  reg[o] = r ? 1 : 0;
}

__global__ void k_erode(GridDims g, const uint8_t* __restrict__ in, uint8_t* __restrict__ out) {
  const int gi = blockIdx.y;
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const long long o = (long long)gi * g.ncell + c;
  bool r = in[o] != 0;   // a regular cell is interior, so its neighbours exist
  if (r) {
    const long long st[3] = {1, g.n[0], (long long)g.n[0] * g.n[1]};
    for (int d = 0; d < g.D; ++d) r = r && in[o - st[d]] && in[o + st[d]];
  }
  out[o] = r ? 1 : 0;
}

int enumerate_batch(const Work& w, const cutcell_opts& o, hipStream_t st) {
  const GridDims& g = w.dims;
  const int D = o.dim, Q = o.order;
  const int M = binom(Q + D, D), Mf = binom(Q + D - 1, D - 1);
  const int T = 256;
  hipLaunchKernelGGL(k_enum_flags, dim3(blocks_for(w.L, T), w.G), dim3(T), 0, st, g, M, Mf, w.geoms, w.flags, w.L);
  int rc = exclusive_scan<int32_t, int32_t>(w.flags, w.L, w.L, w.G, w.excl, w.L, w.seg_total, w.scan_tmp, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_enum_counts, dim3(1), dim3(64), 0, st, g, w.G, w.L, w.excl, w.seg_total, w.geoms, w.counts,
                     w.offs);
  const long long nmap = (long long)w.G * g.NF;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(nmap, T)), dim3(T), 0, st, w.box_id, nmap, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for((long long)w.G * g.ncell, T)), dim3(T), 0, st, w.eb_id,
                     (long long)w.G * g.ncell, -1);
  hipLaunchKernelGGL(k_enum_maps, dim3(blocks_for(w.L, T), w.G), dim3(T), 0, st, g, w.G, w.L, w.maxface, w.flags,
                     w.excl, w.offs, w.vol_id, w.vol_cell, w.box_id, w.box_lf, w.face_id, w.fcode, w.fref);
  hipLaunchKernelGGL(k_enum_eb, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, w.G, w.geoms, w.counts, w.offs,
                     w.eb_id, w.fcode, w.fref);
  hipLaunchKernelGGL(k_cellinfo, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, w.vol_id, w.eb_id, w.face_id,
                     w.cellinfo);
  // the result must end in w.ballreg: start in the buffer that R erosions leave it in
  uint8_t* bufs[2] = {w.ballreg, w.ballreg_tmp};
  int cur = (o.path_radius % 2 == 0) ? 0 : 1;
  hipLaunchKernelGGL(k_regular0, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, w.cellinfo, bufs[cur]);
  for (int r = 0; r < o.path_radius; ++r) {
    hipLaunchKernelGGL(k_erode, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, bufs[cur], bufs[1 - cur]);
    cur = 1 - cur;
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// ---------------------------------------------------------------------------------------
// neighbours: breadth-first search by path distance inside a window around the face

template <int D, int R>
struct Win {
  static constexpr int EN = 2 * R + 2;                       // extent along the face normal
  static constexpr int ET = 2 * R + 1;                       // transverse extent
  static constexpr int NW = EN * (D >= 2 ? ET : 1) * (D >= 3 ? ET : 1);
  static constexpr int K = (NW + 63) / 64;                   // window cells per lane
};

// Rows of a face between two ball-regular cells a (low) and a + e_d: the union of the L1
// balls of radius R around them, as offsets from a in ascending cell-index order (z, y, x).
template <int D, int R>
struct RegularRows {
  static constexpr int kMax = 2 * (2 * R + 2) * (2 * R + 1) * (D == 3 ? 2 * R + 1 : 1);
  int n = 0;
  int8_t off[3][kMax][3] = {};
  constexpr RegularRows() {
    for (int dn = 0; dn < D; ++dn) {
      int cnt = 0;
      const int zlo = (D == 3) ? -R : 0, zhi = (D == 3) ? R + (dn == 2) : 0;
      for (int z = zlo; z <= zhi; ++z)
        for (int y = -R; y <= R + (dn == 1); ++y)
          for (int x = -R; x <= R + (dn == 0); ++x) {
            const int o[3] = {x, y, z};
            int l0 = 0, l1 = 0;
            for (int ax = 0; ax < 3; ++ax) {
              const int v = o[ax], w = o[ax] - (ax == dn);
              l0 += v < 0 ? -v : v;
              l1 += w < 0 ? -w : w;
            }
            if (l0 <= R || l1 <= R) {
              off[dn][cnt][0] = (int8_t)x;
              off[dn][cnt][1] = (int8_t)y;
              off[dn][cnt][2] = (int8_t)z;
              ++cnt;
            }
          }
      n = cnt;
    }
  }
};

template <int D, int R>
inline constexpr RegularRows<D, R> kRegularRows{};

template <int D, int R, bool FILL>
__global__ __launch_bounds__(64) void k_neighbours(GridDims g, int G, long long n_face,
                                                   const int32_t* __restrict__ fcode, const int32_t* __restrict__ fref,
                                                   const GeomPtrs* __restrict__ geoms, const int32_t* __restrict__ vol_id,
                                                   const int32_t* __restrict__ eb_id, const int32_t* __restrict__ face_id,
                                                   const int32_t* __restrict__ box_id, const int64_t* __restrict__ counts,
                                                   const int64_t* __restrict__ offs, const uint8_t* __restrict__ cellinfo,
                                                   const uint8_t* __restrict__ ballreg, int32_t* nrows,
                                                   const int64_t* __restrict__ row_ptr, int32_t* col, int neumann,
                                                   unsigned long long* __restrict__ nbmask) {
  using W = Win<D, R>;
  __shared__ int8_t dist[W::NW];
  const long long F = blockIdx.x;
  if (F >= n_face) return;
  const int lane = threadIdx.x;
  const int32_t code = fcode[F];
  const int gi = code >> 4, kind = (code >> 2) & 3, dn = code & 3;
  const int32_t ref = fref[F];
  // a Neumann EB face's flux is its data: one row, its own Phi entry
  if (kind == 1 && neumann) {
    if (lane == 0) {
      if (!FILL) nrows[F] = 1;
      else col[row_ptr[F]] = (int32_t)(offs[gi] + counts[4 * gi + 0] + ref);
    }
    return;
  }

  const int32_t* vid = vol_id + gi * g.ncell;
  // fast path: a grid face between two ball-regular cells has the fixed L1-ball rows
  if (kind == 0) {
    int j[3];
    lattice_coords(g, dn, ref, j);
    if (j[dn] >= 1 && j[dn] <= g.n[dn] - 1) {
      const long long b = cell_index(g, j);
      const long long st[3] = {1, g.n[0], (long long)g.n[0] * g.n[1]};
      const long long a = b - st[dn];
      const uint8_t* reg = ballreg + (long long)gi * g.ncell;
      if (reg[a] && reg[b]) {
        constexpr auto& P = kRegularRows<D, R>;
        if (!FILL) {
          if (lane == 0) nrows[F] = P.n;
          return;
        }
        const long long pos = row_ptr[F];
        const int64_t phi0 = offs[gi];
        for (int i = lane; i < P.n; i += 64) {
          const long long c = a + P.off[dn][i][0] + st[1] * P.off[dn][i][1] + st[2] * P.off[dn][i][2];
          col[pos + i] = (int32_t)(phi0 + vid[c]);
        }
        return;
      }
    }
  }
  const int32_t* eid = eb_id + gi * g.ncell;
  const int32_t* bid = box_id + gi * g.NF;

  // window origin and extents; the adjacent cells sit at normal index R (and R + 1)
  int org[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int nrm = dn;
  if (kind == 0) {
    int j[3];
    lattice_coords(g, dn, ref, j);
    for (int ax = 0; ax < D; ++ax) {
      ext[ax] = (ax == dn) ? W::EN : W::ET;
      org[ax] = (ax == dn) ? j[ax] - R - 1 : j[ax] - R;
    }
  } else {
    const int32_t c = geoms[gi].eb_cell[ref];
    int ci[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
    nrm = 0;
    for (int ax = 0; ax < D; ++ax) {
      ext[ax] = (ax == 0) ? W::EN : W::ET;
      org[ax] = ci[ax] - R;
    }
  }
  const int NW = ext[0] * ext[1] * ext[2];

  // the fill pass takes the rows the count pass found (its ballot masks, one word per 64
  // window cells, at the face's own slot) instead of searching again
  const bool reuse = FILL && nbmask;

  // per-lane window cells: global cell, info byte (volume, open faces, EB); open bits
  // are kept only toward neighbours inside the window and the box
  const uint8_t* inf = cellinfo + (long long)gi * g.ncell;
  long long cell[W::K];
  bool isvol[W::K];
  unsigned open[W::K];
  unsigned info[W::K];
  int wpos[W::K][3];
  int xk[W::K][3];      // grid coordinates of the window cells
#pragma unroll
  for (int k = 0; k < W::K; ++k) {
    const int w = lane + 64 * k;
    isvol[k] = false;
    open[k] = 0;
    info[k] = 0;
    cell[k] = -1;
    xk[k][0] = xk[k][1] = xk[k][2] = -1;
    if (w >= NW) continue;
    // window coordinates with compile-time divisors (the long extent is along nrm)
    int wc[3];
    if (nrm == 0) {
      wc[0] = w % W::EN; wc[1] = (w / W::EN) % W::ET; wc[2] = w / (W::EN * W::ET);
    } else if (nrm == 1) {
      wc[0] = w % W::ET; wc[1] = (w / W::ET) % W::EN; wc[2] = w / (W::ET * W::EN);
    } else {
      wc[0] = w % W::ET; wc[1] = (w / W::ET) % W::ET; wc[2] = w / (W::ET * W::ET);
    }
    if (D == 2) wc[2] = 0;
    int x[3];
    bool inbox = true;
    for (int ax = 0; ax < 3; ++ax) {
      wpos[k][ax] = wc[ax];
      x[ax] = org[ax] + wc[ax];
      xk[k][ax] = x[ax];
      if (ax < D && (x[ax] < 0 || x[ax] >= g.n[ax])) inbox = false;
    }
    if (!inbox) continue;
    cell[k] = cell_index(g, x);
    if (reuse) continue;   // rows from the count pass: no search
    info[k] = inf[cell[k]];
    isvol[k] = info[k] & 1u;
    for (int ax = 0; ax < D; ++ax)
      for (int s = 0; s < 2; ++s) {
        const int wn = wc[ax] + (s ? 1 : -1);
        const int xn = x[ax] + (s ? 1 : -1);
        if (wn >= 0 && wn < ext[ax] && xn >= 0 && xn < g.n[ax] && ((info[k] >> (1 + 2 * ax + s)) & 1u))
          open[k] |= 1u << (2 * ax + s);
      }
  }
  bool inS[W::K];
  if (reuse) {
    const unsigned long long* mk = nbmask + F * W::K;
#pragma unroll
    for (int k = 0; k < W::K; ++k) inS[k] = (mk[k] >> lane) & 1ull;
  } else {
  // distances: 0 at the adjacent volumes, R + 1 ("far") elsewhere
#pragma unroll
  for (int k = 0; k < W::K; ++k) {
    const int w = lane + 64 * k;
    if (w >= NW) continue;
    bool adj = isvol[k];
    for (int ax = 0; ax < D; ++ax) {
      if (ax == nrm)
        adj = adj && ((wpos[k][ax] == R) || (kind == 0 && wpos[k][ax] == R + 1));
      else
        adj = adj && (wpos[k][ax] == R);
    }
    dist[w] = adj ? 0 : (R + 1);
  }
  __syncthreads();
  for (int r = 1; r <= R; ++r) {
    int8_t nd[W::K];
#pragma unroll
    for (int k = 0; k < W::K; ++k) {
      const int w = lane + 64 * k;
      nd[k] = -1;
      if (w >= NW || !isvol[k] || dist[w] <= R) continue;
      const int st[3] = {1, ext[0], ext[0] * ext[1]};
      for (int ax = 0; ax < D; ++ax)
        for (int s = 0; s < 2; ++s)
          if ((open[k] >> (2 * ax + s)) & 1u) {
            int wn = w + (s ? st[ax] : -st[ax]);
            if (dist[wn] == r - 1) nd[k] = (int8_t)r;
          }
    }
#pragma unroll
    for (int k = 0; k < W::K; ++k)
      if (nd[k] > 0) dist[lane + 64 * k] = nd[k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < W::K; ++k) {
    const int w = lane + 64 * k;
    inS[k] = (w < NW) && isvol[k] && dist[w] <= R;
  }
  }

  const int64_t* cnt = counts + 4 * gi;
  const int64_t phi0 = offs[gi];
  if (!FILL) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < W::K; ++k) {
      if (!inS[k]) continue;
      c += 1 + (int)(info[k] >> 7);
      const int* x = xk[k];
      for (int ax = 0; ax < D; ++ax)
        for (int s = 0; s < 2; ++s)
          if (x[ax] == (s ? g.n[ax] - 1 : 0) && ((info[k] >> (1 + 2 * ax + s)) & 1u)) c += 1;   // box face
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane == 0) nrows[F] = c;
    if (nbmask) {   // leave the rows for the fill pass
      unsigned long long* mk = nbmask + F * W::K;
#pragma unroll
      for (int k = 0; k < W::K; ++k) {
        const unsigned long long m = __ballot(inS[k]);
        if (lane == k) mk[k] = m;
      }
    }
    return;
  }
  // fill in ascending Phi order: volumes, EB faces, box faces by (d, side)
  long long pos = row_ptr[F];
  const unsigned long long below = lanes_below(lane);
#pragma unroll
  for (int k = 0; k < W::K; ++k) {
    bool p = inS[k];
    unsigned long long m = __ballot(p);
    if (p) col[pos + __popcll(m & below)] = (int32_t)(phi0 + vid[cell[k]]);
    pos += __popcll(m);
  }
#pragma unroll
  for (int k = 0; k < W::K; ++k) {
    bool p = inS[k] && eid[cell[k]] >= 0;
    unsigned long long m = __ballot(p);
    if (p) col[pos + __popcll(m & below)] = (int32_t)(phi0 + cnt[0] + eid[cell[k]]);
    pos += __popcll(m);
  }
  for (int ax = 0; ax < D; ++ax)
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int k = 0; k < W::K; ++k) {
        int32_t b = -1;
        if (inS[k]) {
          const int* x = xk[k];
          if (x[ax] == (s ? g.n[ax] - 1 : 0)) {
            int j[3] = {x[0], x[1], x[2]};
            j[ax] += s;
            b = bid[lattice_index(g, ax, j)];
          }
        }
        bool p = b >= 0;
        unsigned long long m = __ballot(p);
        if (p) col[pos + __popcll(m & below)] = (int32_t)(phi0 + cnt[0] + cnt[1] + b);
        pos += __popcll(m);
      }
    }
}

template <int D, int R>
static void launch_neighbours(const Work& w, long long n_face, const int64_t* row_ptr, int32_t* col, bool fill,
                              int neumann, hipStream_t st) {
  // the count pass leaves each searched face's rows (as ballot masks) for the fill pass
  if (fill)
    hipLaunchKernelGGL((k_neighbours<D, R, true>), dim3((unsigned)n_face), dim3(64), 0, st, w.dims, w.G, n_face,
                       w.fcode, w.fref, w.geoms, w.vol_id, w.eb_id, w.face_id, w.box_id, w.counts, w.offs, w.cellinfo,
                       w.ballreg, w.nrows, row_ptr, col, neumann, w.nbmask);
  else
    hipLaunchKernelGGL((k_neighbours<D, R, false>), dim3((unsigned)n_face), dim3(64), 0, st, w.dims, w.G, n_face,
                       w.fcode, w.fref, w.geoms, w.vol_id, w.eb_id, w.face_id, w.box_id, w.counts, w.offs, w.cellinfo,
                       w.ballreg, w.nrows, row_ptr, col, neumann, w.nbmask);
}

int neighbour_rows(const Work& w, const cutcell_opts& o, long long n_face, const int64_t* row_ptr, int32_t* col,
                   bool fill, hipStream_t st) {
  if (n_face <= 0) return CUTCELL_OK;
  const int D = o.dim, R = o.path_radius;
  const int neumann = o.eb_bc == CUTCELL_BC_NEUMANN;
#define CC_NB(DD, RR) \
  if (D == DD && R == RR) { launch_neighbours<DD, RR>(w, n_face, row_ptr, col, fill, neumann, st); }
  CC_NB(2, 1) CC_NB(2, 2) CC_NB(2, 3) CC_NB(2, 4) CC_NB(3, 1) CC_NB(3, 2) CC_NB(3, 3) CC_NB(3, 4)
#undef CC_NB
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// ---------------------------------------------------------------------------------------
// volume -> faces table and the 1/|V| scale of the divergence

__global__ void k_volume_tables(GridDims g, int G, int M, double hD, const GeomPtrs* __restrict__ geoms,
                                const int32_t* __restrict__ vol_id, const int32_t* __restrict__ eb_id,
                                const int32_t* __restrict__ face_id, const int64_t* __restrict__ counts,
                                const int64_t* __restrict__ offs, int32_t* vol_face, double* vol_scale) {
  const int gi = blockIdx.y;
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int32_t v = vol_id[gi * g.ncell + c];
  if (v < 0) return;
  const int D = g.D;
  const long long V = offs[(G + 1) + gi] + v;
  const long long F0 = offs[2 * (G + 1) + gi];
  int x[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  const int S = 2 * D + 1;
  for (int d = 0; d < D; ++d)
    for (int s = 0; s < 2; ++s) {
      int j[3] = {x[0], x[1], x[2]};
      j[d] += s;
      int32_t f = face_id[gi * g.NF + lattice_index(g, d, j)];
      vol_face[V * S + 2 * d + s] = (f >= 0) ? (int32_t)(F0 + f) : -1;
    }
  int32_t e = eb_id[gi * g.ncell + c];
  vol_face[V * S + 2 * D] = (e >= 0) ? (int32_t)(F0 + counts[4 * gi + 3] + e) : -1;
  vol_scale[V] = 1.0 / (geoms[gi].vol_mom[c * M] * hD);
}

int volume_tables(const Work& w, const cutcell_opts& o, long long n_vol_total, int32_t* vol_face, double* vol_scale,
                  hipStream_t st) {
  if (n_vol_total <= 0) return CUTCELL_OK;
  const int M = binom(o.order + o.dim, o.dim);
  double hD = 1.0;
  for (int d = 0; d < o.dim; ++d) hD *= o.h;
  hipLaunchKernelGGL(k_volume_tables, dim3(blocks_for(w.dims.ncell, 256), w.G), dim3(256), 0, st, w.dims, w.G, M, hD,
                     w.geoms, w.vol_id, w.eb_id, w.face_id, w.counts, w.offs, vol_face, vol_scale);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

// ---------------------------------------------------------------------------------------
// binning by row count: buckets of 16 rows (N <= 16, ..., <= 128) and one bucket for
// faces with fewer rows than monomials; perm lists faces bucket by bucket

// per-block histograms in LDS (buckets, then parts 0 and 1 of the row bins), one global
// atomic per counter per block
__global__ __launch_bounds__(256) void k_bin_count(long long n_face, int M, const int32_t* __restrict__ nrows,
                                                   const int32_t* __restrict__ tmpl, int32_t* bins) {
  constexpr int NP = 2 * kMaxBins;
  __shared__ int32_t h[kNBuckets + NP];
  if (threadIdx.x < kNBuckets + NP) h[threadIdx.x] = 0;
  __syncthreads();
  long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f < n_face) {
    const int b = face_bucket(f, M, nrows, tmpl);
    atomicAdd(&h[b], 1);
    const int part = face_part(b, f, nrows);
    if (part < 2) atomicAdd(&h[kNBuckets + part * kMaxBins + b], 1);
  }
  __syncthreads();
  if (threadIdx.x < kNBuckets && h[threadIdx.x]) atomicAdd(&bins[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x < NP && h[kNBuckets + threadIdx.x])
    atomicAdd(&bins[kPartWords + threadIdx.x], h[kNBuckets + threadIdx.x]);
}

__global__ void k_bin_starts(int32_t* bins) {
  if (threadIdx.x != 0) return;
  int s = 0;
  for (int b = 0; b < kNBuckets; ++b) {
    bins[kNBuckets + b] = s;
    s += bins[b];
  }
}

// largest row count (block reduction, one atomic per block)
__global__ __launch_bounds__(256) void k_max_rows(long long n_face, const int32_t* __restrict__ nrows, int32_t* out) {
  __shared__ int32_t sm[256];
  long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  sm[threadIdx.x] = (f < n_face) ? nrows[f] : 0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, sm[0]);
}

int max_rows(const Work& w, long long n_face, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.bins + 2 * kNBuckets, 1LL, 0);
  if (n_face > 0)
    hipLaunchKernelGGL(k_max_rows, dim3(blocks_for(n_face, 256)), dim3(256), 0, st, n_face, w.nrows,
                       w.bins + 2 * kNBuckets);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int rows_per_face(const Work& w, long long n_face, const int64_t* row_ptr, hipStream_t st) {
  if (n_face > 0)
    hipLaunchKernelGGL(k_rows_per_face, dim3(blocks_for(n_face, 256)), dim3(256), 0, st, n_face, row_ptr, w.nrows);
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

int bin_faces(const Work& w, long long n_face, int M, const int32_t* tmpl, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.bins, (long long)(2 * kNBuckets), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.bins + kPartWords, (long long)(2 * kMaxBins), 0);
  if (n_face <= 0) return CUTCELL_OK;
  hipLaunchKernelGGL(k_bin_count, dim3(blocks_for(n_face, 256)), dim3(256), 0, st, n_face, M, w.nrows, tmpl, w.bins);
  hipLaunchKernelGGL(k_bin_starts, dim3(1), dim3(64), 0, st, w.bins);
  CC_HIP(hipGetLastError());
  return order_faces(w, n_face, M, tmpl, st);
}

// ---------------------------------------------------------------------------------------
// Template reuse.  A face between two cells whose every neighbour within the path radius
// is a plain interior volume has the fixed row pattern of the fast path above; if all of
// those cells and their faces also carry exactly the reference cell's moments, its system
// (rows about x0 -- the offsets are exact small half-integers --, weights and F) is bit
// for bit that of any other such face of the same direction, and so is its stencil.  One
// face per (geometry, direction) is solved; the others copy its values.

constexpr int32_t kNone = 0x7fffffff;

__global__ void k_ref_cell(GridDims g, const uint8_t* __restrict__ ballreg, int32_t* ref) {
  const int gi = blockIdx.y;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  if (ballreg[(long long)gi * g.ncell + c]) atomicMin(&ref[gi], (int32_t)c);
}

__device__ __forceinline__ bool same_bits(const double* a, const double* b, int n) {
  bool s = true;
  for (int i = 0; i < n; ++i) s = s && (__double_as_longlong(a[i]) == __double_as_longlong(b[i]));
  return s;
}

// plain interior volume (as for ball regularity) whose volume moments and the moments of
// its 2D faces equal the reference cell's bit for bit
__global__ void k_canon0(GridDims g, int M, int Mf, const GeomPtrs* __restrict__ geoms,
                         const uint8_t* __restrict__ info, const int32_t* __restrict__ ref, uint8_t* __restrict__ out) {
  const int gi = blockIdx.y;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const long long o = (long long)gi * g.ncell + c;
  const unsigned full = (1u << (1 + 2 * g.D)) - 1u;
  bool r = info[o] == full;
  const int x[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((long long)g.n[0] * g.n[1]))};
  for (int d = 0; d < g.D; ++d) r = r && x[d] >= 1 && x[d] <= g.n[d] - 2;
  const int32_t rc = ref[gi];
  r = r && rc != kNone;
  if (r) {
    const GeomPtrs gp = geoms[gi];
    r = same_bits(gp.vol_mom + c * M, gp.vol_mom + (long long)rc * M, M);
    const int xr[3] = {(int)(rc % g.n[0]), (int)((rc / g.n[0]) % g.n[1]), (int)(rc / ((long long)g.n[0] * g.n[1]))};
    for (int d = 0; d < g.D && r; ++d)
      for (int s = 0; s < 2 && r; ++s) {
        int j[3] = {x[0], x[1], x[2]}, jr[3] = {xr[0], xr[1], xr[2]};
        j[d] += s;
        jr[d] += s;
        const long long lf = lattice_index(g, d, j) - g.foff[d], lr = lattice_index(g, d, jr) - g.foff[d];
        r = same_bits(gp.face_mom[d] + lf * Mf, gp.face_mom[d] + lr * Mf, Mf);
      }
  }
  out[o] = r ? 1 : 0;
}

// a grid face between two cells that are canonical out to the path radius
__device__ __forceinline__ bool template_face(const GridDims& g, const int32_t* fcode, const int32_t* fref,
                                             const uint8_t* canon, long long F, int* gi_out, int* dn_out) {
  const int32_t code = fcode[F];
  const int gi = code >> 4, kind = (code >> 2) & 3, dn = code & 3;
  *gi_out = gi;
  *dn_out = dn;
  if (kind != 0) return false;
  int j[3];
  lattice_coords(g, dn, fref[F], j);
  if (j[dn] < 1 || j[dn] > g.n[dn] - 1) return false;
  const long long b = cell_index(g, j);
  const long long st[3] = {1, g.n[0], (long long)g.n[0] * g.n[1]};
  const uint8_t* cn = canon + (long long)gi * g.ncell;
  return cn[b - st[dn]] && cn[b];
}

// The first template-able face of each (geometry, direction).  Faces of a wave are
// consecutive and nearly always of one (geometry, direction): the wave's lowest such lane
// stands for the lanes of its key (their minimum, faces ascending with the lane), and only
// lanes of another key add their own atomic -- one atomic per wave instead of one per
// face on three addresses per geometry.
__global__ void k_tmpl_pick(GridDims g, long long n_face, const int32_t* __restrict__ fcode,
                            const int32_t* __restrict__ fref, const uint8_t* __restrict__ canon, int32_t* tface) {
  const long long F = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  int gi = 0, dn = 0;
  const bool q = F < n_face && template_face(g, fcode, fref, canon, F, &gi, &dn);
  const unsigned long long m = __ballot(q);
  if (m == 0) return;
  const int lane = threadIdx.x & 63, leader = __ffsll((long long)m) - 1;
  const int key = 3 * gi + dn;
  const int lkey = __shfl(key, leader, 64);
  if (q && (lane == leader || key != lkey)) atomicMin(&tface[key], (int32_t)F);
}

__global__ void k_tmpl_assign(GridDims g, long long n_face, const int32_t* __restrict__ fcode,
                              const int32_t* __restrict__ fref, const uint8_t* __restrict__ canon,
                              const int32_t* __restrict__ tface, int32_t* __restrict__ tmpl) {
  const long long F = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (F >= n_face) return;
  int gi, dn;
  const bool q = template_face(g, fcode, fref, canon, F, &gi, &dn);
  const int32_t t = q ? tface[3 * gi + dn] : kNone;
  tmpl[F] = (q && t != (int32_t)F) ? t : -1;
}

int find_templates(const Work& w, const cutcell_opts& o, long long n_face, hipStream_t st) {
  const GridDims& g = w.dims;
  const int D = o.dim, Q = o.order;
  const int M = binom(Q + D, D), Mf = binom(Q + D - 1, D - 1);
  const int T = 256;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, w.ref_cell, (long long)w.G, kNone);
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(3LL * w.G, 64)), dim3(64), 0, st, w.tface, 3LL * w.G, kNone);
  hipLaunchKernelGGL(k_ref_cell, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, w.ballreg, w.ref_cell);
  // R erosions must leave the result in w.canon (ping-pong with ballreg_tmp)
  uint8_t* bufs[2] = {w.canon, w.ballreg_tmp};
  int cur = (o.path_radius % 2 == 0) ? 0 : 1;
  hipLaunchKernelGGL(k_canon0, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, M, Mf, w.geoms, w.cellinfo,
                     w.ref_cell, bufs[cur]);
  for (int r = 0; r < o.path_radius; ++r) {
    hipLaunchKernelGGL(k_erode, dim3(blocks_for(g.ncell, T), w.G), dim3(T), 0, st, g, bufs[cur], bufs[1 - cur]);
    cur = 1 - cur;
  }
  if (n_face > 0) {
    hipLaunchKernelGGL(k_tmpl_pick, dim3(blocks_for(n_face, T)), dim3(T), 0, st, g, n_face, w.fcode, w.fref, w.canon,
                       w.tface);
    hipLaunchKernelGGL(k_tmpl_assign, dim3(blocks_for(n_face, T)), dim3(T), 0, st, g, n_face, w.fcode, w.fref,
                       w.canon, w.tface, w.tmpl);
  }
  CC_HIP(hipGetLastError());
  return CUTCELL_OK;
}

}  // namespace cutcell
