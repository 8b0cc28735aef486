// Device workspace layout and kernel launchers shared by the host entry points.
#pragma once

#include "common.hpp"

namespace cutcell {

// flux-face code: geometry << 4 | kind << 2 | direction (kind 0 grid/box, 1 EB)
__host__ __device__ inline int32_t face_code(int g, int kind, int d) { return (g << 4) | (kind << 2) | d; }

constexpr int kMaxBins = 8;     // row-count bins of 16 rows: N <= 16, 32, ..., 128
constexpr int kBinRows = 16;
constexpr int kMaxRows = kMaxBins * kBinRows;
constexpr int kNBuckets = kMaxBins + 2;   // then faces with N < M, then template copies
constexpr int kPartWords = 2 * kNBuckets + 1;      // counts, cursors, max rows; then per row bin
constexpr int kBinWords = kPartWords + 2 * kMaxBins;  // the faces of its part 0 and of its part 1
constexpr int kXcds = 8;        // MI355X: workgroups are dealt to 8 XCDs (own L2 each) in turn
constexpr int kQrSlots = 1024;  // workgroups of the QR path, each with a slot of workspace

// Per-batch workspace: pointers into the caller's buffer.
struct Work {
  GridDims dims;
  int G;
  long long L;          // enumeration flag space per geometry: cells | box slots | lattice faces
  long long maxface;    // flux-face capacity per geometry (lattice faces + one EB per cell)
  int32_t* flags;       // [G][L]
  int32_t* excl;        // [G][L]
  int32_t* seg_total;   // [G]
  int32_t* scan_tmp;    // [G][tiles(L)]
  int32_t* vol_id;      // [G][ncell]  local volume index or -1
  int32_t* eb_id;       // [G][ncell]  local EB index or -1
  int32_t* face_id;     // [G][NF]     local flux-face index or -1
  int32_t* box_id;      // [G][NF]     local box-face index or -1
  int32_t* box_lf;      // [G][nboxslot] lattice face of each local box face
  int32_t* vol_cell;    // [G][ncell]  cell of each local volume
  uint8_t* cellinfo;    // [G][ncell]  volume / open-face / EB bits for the neighbour search
  uint8_t* ballreg;     // [G][ncell]  1: every cell within path radius is a plain interior volume
  uint8_t* ballreg_tmp; // [G][ncell]  erosion ping-pong buffer
  uint8_t* canon;       // [G][ncell]  1: every cell within path radius has the reference moments
  int32_t* ref_cell;    // [G]         the reference (ball-regular) cell, or INT32_MAX
  int32_t* tface;       // [G][3]      template face per direction, or INT32_MAX
  int32_t* tmpl;        // [G*maxface] template of each face whose stencil is copied, else -1
  unsigned long long* okey;      // [G*maxface] processing-order keys (bucket, then cell)
  unsigned long long* okey_out;  // [G*maxface]
  int32_t* oval;        // [G*maxface] face ids to sort
  char* osort_tmp;      // radix-sort scratch
  size_t osort_bytes;
  int64_t* counts;      // [G][4]      n_vol, n_eb, n_box, n_gface
  int64_t* offs;        // [3][G+1]    phi_off, vol_off, face_off
  int32_t* fcode;       // [G*maxface] per global flux face
  int32_t* fref;        // [G*maxface] lattice face (grid/box) or EB index
  int32_t* nrows;       // [G*maxface]
  int64_t* scan64;      // int64 scan tiles over G*maxface
  int64_t* rp_tmp;      // [G*maxface + 1] row offsets when the caller has none (query)
  int32_t* perm;        // [G*maxface]
  int32_t* bins;        // [kBinWords] bucket counts, bucket cursors, max rows, part counts
  int32_t* flagged;     // [2] flagged faces, bad EB input
  int32_t* qr_count;    // [1] faces left to the Householder QR path
  int32_t* qr_list;     // [G*maxface] those faces
  double* qr_b;         // [qr_slots][2][kMaxRows * MS] the QR path's exact B per workgroup
  unsigned long long* nbmask;  // [G*maxface][window words] rows the count pass found (searched faces)
  int qr_slots;         // min(kQrSlots, G*maxface)
  GeomPtrs* geoms;      // [G]
  size_t bytes;
};

size_t layout_work(const cutcell_opts& o, int G, char* base, Work* w);

// Outputs of the per-face stencil adjoint (k_stencil_backward) and their layout.
// device copy of the per-geometry gradient pointers (layouts as the inputs)
struct GradPtrs {
  double* vol_mom;
  double* face_mom[3];
  double* eb_mom;
  double* eb_nmom;
};

struct BackwardArgs {
  const double* val_bar;        // [nnz]
  double* face_yw;              // [n_face][2][M]   y and w
  double* face_x0;              // [n_face][4]      x0 / h
  double* nz_rz;                // [nnz][2]         (W r, W z) of each row
  double* weight_bar;           // [nnz] or null
  double* owner_grad;           // [n_face][4]      EB faces: d/d vol_mom[owner][0..D]; 0 otherwise
  const GradPtrs* grads;        // [G]  the face-moment and EB normal-moment gradients are
                                //      written here directly (Fbar)
  const int8_t* fwd_status;     // [n_face] status of the forward build
};

// Transposed (CSC) structure of the stencils: the nonzeros of each Phi entry in
// ascending CSR position, with the face each belongs to.
struct Transpose {
  const int64_t* col_ptr;   // [n_phi + 1]
  const int32_t* nz;        // [nnz]
  const int32_t* nz_face;   // [nnz]
};

// enumeration (Sec. 2.1): flags, maps, global face table, counts and offsets
int enumerate_batch(const Work& w, const cutcell_opts& o, hipStream_t st);
// neighbour rows (Sec. 2.4): count (fill = false) or write col[] (fill = true)
int neighbour_rows(const Work& w, const cutcell_opts& o, long long n_face, const int64_t* row_ptr, int32_t* col,
                   bool fill, hipStream_t st);
// volume -> face table and 1/(kappa h^D)
int volume_tables(const Work& w, const cutcell_opts& o, long long n_vol_total, int32_t* vol_face,
                  double* vol_scale, hipStream_t st);
// binning by row count and the stencil solves (Sec. 2.2.1)
// `tmpl` (or null): faces with tmpl >= 0 go to the template-copy bucket
int bin_faces(const Work& w, long long n_face, int M, const int32_t* tmpl, hipStream_t st);
// processing order: faces grouped by bucket, inside a bucket by the cell they sit at
size_t order_temp_bytes(long long n_items);
int order_faces(const Work& w, long long n_face, int M, const int32_t* tmpl, hipStream_t st);

// bucket of face f: a 16-row bin, the faces with fewer rows than monomials, or the copies
__host__ __device__ inline int face_bucket(long long f, int M, const int32_t* nrows, const int32_t* tmpl) {
  if (tmpl && tmpl[f] >= 0) return kMaxBins + 1;
  const int N = nrows[f];
  return (N < M) ? kMaxBins : ((N - 1) / kBinRows < kMaxBins - 1 ? (N - 1) / kBinRows : kMaxBins - 1);
}
// part of face f in row bin `bucket` (rows 16 bucket + 1 .. 16 bucket + 16): 0 for at most
// 8 rows above the bin's lower edge, 1 for at most 12, else 2 (and 2 outside the row bins).
// The parts come in this order in the bin, and parts 0 and 1 may be solved by narrower
// kernel instances.
__host__ __device__ inline int face_part(int bucket, long long f, const int32_t* nrows) {
  if (bucket >= kMaxBins) return 2;
  const int above = nrows[f] - kBinRows * bucket;
  return above <= kBinRows / 2 ? 0 : (above <= 3 * kBinRows / 4 ? 1 : 2);
}
// faces whose systems are bitwise those of one solved face per (geometry, direction)
int find_templates(const Work& w, const cutcell_opts& o, long long n_face, hipStream_t st);
int max_rows(const Work& w, long long n_face, hipStream_t st);
int solve_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count /* host */, long long n_face,
                   const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status, hipStream_t st);
// Arguments of the per-Phi-entry sum of the rows' moment gradients.
struct ReduceArgs {
  GridDims g;
  int G;
  long long n_phi;
  const int64_t* offs;        // [3][G+1] phi_off, vol_off, face_off
  const int64_t* counts;      // [G][4]
  const GeomPtrs* geoms;
  const GradPtrs* grads;
  const int32_t* vol_cell_ws;
  const int32_t* box_lf_ws;
  Transpose tr;
  const double* face_yw;
  const double* face_x0;
  const double* nz_rz;
  const double* owner_grad;
  const int32_t* vol_face;    // [n_vol][2D+1]
  const double* vol_scale;    // [n_vol]
  const double* scale_bar;    // [n_vol] or null
};

// the Householder QR path (stencil_qr.hip): faces list[0 .. n), n = *count_dev if given,
// else count_host
int solve_qr_faces(const Work& w, const cutcell_opts& o, const int32_t* list, const int32_t* count_dev,
                   long long count_host, const int64_t* row_ptr, const int32_t* col, double* val, int8_t* status,
                   hipStream_t st);
int tune_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                  const int32_t* col, double* val, int8_t* status, hipStream_t st, cutcell_tuning* out, int reps,
                  double* best_ms);
int backward_stencils(const Work& w, const cutcell_opts& o, const int32_t* bin_count, const int64_t* row_ptr,
                      const int32_t* col, const BackwardArgs& bw, hipStream_t st);
int rows_per_face(const Work& w, long long n_face, const int64_t* row_ptr, hipStream_t st);
int reduce_moments(const cutcell_opts& o, const ReduceArgs& R, hipStream_t st);
// transpose of the stencils and the apply adjoint
size_t transpose_temp_bytes(long long nnz, long long n_phi);
int build_transpose(long long n_face, long long n_phi, long long nnz, const int64_t* row_ptr, const int32_t* col,
                    int64_t* col_ptr, int32_t* nz, int32_t* nz_face, char* ws, size_t ws_bytes, hipStream_t st);
int apply_adjoint(int D, long long n_face, long long n_vol, long long n_phi, const int64_t* row_ptr,
                  const int32_t* col, const double* val, const int32_t* vol_face, const double* vol_scale,
                  const Transpose& tr, const double* phi, const double* flux, const double* lbar, double* phi_bar,
                  double* val_bar, double* scale_bar, double* fbar, hipStream_t st);
// operator apply (Sec. 2.2, Sec. 3.3): face fluxes, their divergence, and both
constexpr int kFluxFaces3 = 4, kFluxRounds3 = 6;   // faces per wave and rounds of the CSR flux pass, 3D
constexpr int kFluxFaces2 = 8, kFluxRounds2 = 4;   // and 2D
int flux_faces(int D, long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
               const double* phi, double* flux, hipStream_t st);
int divergence(int D, long long n_vol, const int32_t* vol_face, const double* vol_scale, const double* flux,
               double* lphi, hipStream_t st);
int apply_operator(int D, long long n_face, long long n_vol, const int64_t* row_ptr, const int32_t* col,
                   const double* val, const int32_t* vol_face, const double* vol_scale, const double* phi,
                   double* lphi, double* flux, double* flux_tmp, hipStream_t st);

// the compressed form of the stencils (packed.hip)
struct PackedSizes {
  long long n_packed;
  int n_slot, max_runs, max_rows;
};
struct PackedOut {          // the arrays pack_fill writes
  uint8_t* flag;            // [n_face] 1: the face is packed
  uint8_t* phase;           // [n_face] lane of its first entry in the CSR flux pass
  int32_t* face;            // [n_packed]
  int32_t* slot;            // [n_packed]
  int32_t* base;            // [n_packed][max_runs]
  int32_t* slot_face;       // [n_slot]
  int32_t* slot_rows;       // [n_slot]
  int32_t* slot_tab;        // [n_slot][max_rows]
  double* slot_val;         // [n_slot][max_rows]
};
struct PackedArgs {         // what the apply reads
  long long n_packed;
  int n_slot, max_runs, max_rows;
  const uint8_t* flag;
  const uint8_t* phase;
  const int32_t* face;
  const int32_t* slot;
  const int32_t* base;
  const int32_t* slot_rows;
  const int32_t* slot_tab;
  const double* slot_val;
};
size_t pack_temp_bytes(long long n_face);
int pack_count(long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
               const int32_t* tmpl, char* ws, size_t ws_bytes, long long* n_packed, int* n_slot, int* max_runs,
               int* max_rows, hipStream_t st);
int pack_fill(int D, long long n_face, const int64_t* row_ptr, const int32_t* col, const double* val,
              const int32_t* tmpl, char* ws, size_t ws_bytes, const PackedSizes& ps, const PackedOut& out,
              hipStream_t st);
int apply_packed(int D, long long n_face, long long n_vol, const int64_t* row_ptr, const int32_t* col,
                 const double* val, const int32_t* vol_face, const double* vol_scale, const PackedArgs& pk,
                 const double* phi, double* lphi, double* flux, hipStream_t st);

__global__ void k_fill_i32(int32_t* p, long long n, int32_t v);
__global__ void k_fill_f64(double* p, long long n, double v);

}  // namespace cutcell
