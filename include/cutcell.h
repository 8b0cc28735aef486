/*
 * cutcell.h -- C ABI of the MI355X (gfx950) flux-stencil library for the higher-order
 * cut-cell finite-volume Poisson method of D. Devendran, D. T. Graves and H. Johansen,
 * "A higher-order finite-volume discretization method for Poisson's equation in cut cell
 * geometries" (arXiv:1411.4283).
 *
 * The library builds, for every face of a single-valued cut-cell grid, the weighted
 * least-squares flux stencil  s = W (A^T W)^+ F  (Sec. 2.2.1, eq. 'stencil equation
 * solution') and applies the flux-divergence operator L(Phi) those stencils define
 * (Sec. 2.2, eq. 'laplacian over V'; Sec. 3.3).
 *
 * ---------------------------------------------------------------------------------------
 * Conventions
 *
 *  Grid.  Cells [i h, (i+1) h] of the box [0, n_d h]^D, indexed linearly with x fastest:
 *    c = i0 + n0*(i1 + n1*i2).  Grid faces of direction d form a lattice with n_d + 1
 *    points along d (the other extents as for cells), indexed the same way; face j lies
 *    on x_d = j_d h between cells j - e_d and j.
 *  Monomials.  Multi-indices p with |p| <= Q in graded order: degree ascending; inside a
 *    degree p_1 descending, then p_2 descending (the last exponent varies fastest).
 *    M = C(Q+D, D) (6, 15 or 35), Mf = C(Q+D-1, D-1) transverse face monomials (in the
 *    D-1 directions other than d, in increasing direction order), M1 = C(Q-1+D, D).
 *  Moments (Sec. 2.1, eqs. 'volume moment', 'face moment', 'face moment with normal'),
 *    scaled: with xi = (x - c)/h about the Cartesian centre c of the cell (or face),
 *      vol_mom[c][p]      = int_V  xi^p dV / h^D        (vol_mom[c][0] = kappa)
 *      face_mom[d][f][q]  = int_A  xi^q dA / h^(D-1)    (transverse q; [0] = alpha)
 *      eb_mom[e][p]       = int_EB xi^p dA / h^(D-1)    about the cut cell's centre
 *      eb_nmom[e][d][q]   = int_EB xi^q n_d dA / h^(D-1), |q| <= Q-1, n out of the fluid
 *    A cell with kappa > 0 is a volume; kappa = 0 is covered.  A grid face with
 *    alpha > 0 is a flux face.  Single-valued cells only (one volume and at most one
 *    EB face per cell).
 *  Phi (eq. 'def of phi vec').  [volumes | EB faces | box faces]: volumes by cell index,
 *    EB faces in input order (eb_cell ascending), box faces (grid faces on the box
 *    boundary with alpha > 0) by (direction d, side low=0/high=1, adjacent cell index).
 *    In a batch, geometry g's block starts at phi_off[g] and the blocks follow in order.
 *  Flux faces (CSR rows).  Per geometry: grid faces with alpha > 0 by (d, lattice index),
 *    box faces included, then the EB faces in input order; geometries follow in order.
 *    Reference normal +e_d for grid faces, out of the fluid for EB faces.
 *  Neighbours (Sec. 2.4).  The volumes within path distance R_n (steps through grid
 *    faces with alpha > 0) of the face's adjacent volumes, then every EB face and box
 *    face those volumes touch; col[] lists their Phi indices in ascending order.
 *  Centring (Sec. 2.4).  x0 = face centre for grid faces; for an EB face the centroid
 *    of the cut volume.  Weights W_i = 1 if d_i < 1/2 else (2 d_i)^-5, d_i = |x_i - x0|/h,
 *    x_i the Cartesian centre of the row's cell (volume and EB rows) or face (box rows);
 *    cutcell_opts.weight_custom / weight_power replace the exponent 5 for weight studies.
 *  Values.  val[] holds the physical stencil s = h^(D-2) W (A~^T W)^+ F~, so
 *    flux_f = sum_j val[j] Phi[col[j]] approximates int_f grad(phi).n dA, and
 *    L_v = (1/(kappa_v h^D)) sum_f sigma_vf flux_f with sigma = +1 when the face's
 *    reference normal points out of v.
 *
 *  Boundary data (Sec. 2.2.1).  Under Dirichlet EB conditions an EB entry of Phi is the
 *    average of phi over the face and its row is b_p = m^p(x0)/m^0 (eq. 'Dir moment eq
 *    for cp').  Under Neumann EB conditions (cutcell_opts.eb_bc) it is the average of
 *    grad(phi).n over the face (n out of the fluid) and its row is the normal-derivative
 *    row b_p = sum_d p_d m^(p-e_d)_d(x0) / m^0 (eq. 'Neu moment eq for cp'), whose values
 *    carry h^(D-1) instead of h^(D-2); the flux of a Neumann EB face is its data: its
 *    stencil is the single entry |A_f| (physical area) on its own Phi entry.  Box faces
 *    are Dirichlet.
 *  Memory.  Every array argument is DEVICE memory owned by the caller, except the
 *    structs themselves and cutcell_sizes, which live on the host.  The library keeps no
 *    state between calls and allocates no device memory: scratch comes from the caller's
 *    workspace (sizes from the *_workspace_bytes functions).  Work is enqueued on `stream`
 *    (a hipStream_t; 0 = the null stream).  cutcell_query, cutcell_build_stencils and
 *    cutcell_stencils_backward synchronise `stream` before returning (they read counts
 *    back); cutcell_apply, cutcell_build_transpose and cutcell_apply_adjoint do not.
 *
 *  Derivatives.  The paper defines the forward maps only; the adjoints below are their
 *    exact derivatives (up to rounding).  For a scalar loss l, *_bar denotes dl/d(.).
 *    Results are deterministic: no floating-point atomics, fixed summation orders.
 *
 *  Empty inputs.  A batch may have no fluid at all (no volumes, no faces): the build
 *    then writes only offsets, and cutcell_apply, cutcell_apply_laplacian and cutcell_solve
 *    return CUTCELL_OK at once, accepting NULL for the arrays whose sizes are zero.
 *  Errors.  Every entry point returns CUTCELL_OK (0), CUTCELL_W_FLAGGED_FACES (> 0:
 *    success, some faces got a nonzero status) or a negative CUTCELL_E_* code; the
 *    message of the last error on the calling thread is cutcell_last_error().  The
 *    library never aborts.  A face whose system cannot be solved gets a status code and
 *    val = 0 on its row.
 * ---------------------------------------------------------------------------------------
 */
#ifndef CUTCELL_H
#define CUTCELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CUTCELL_ABI_VERSION 12

enum {
  CUTCELL_OK = 0,
  CUTCELL_W_FLAGGED_FACES = 1,
  CUTCELL_W_NOT_CONVERGED = 2, /* cutcell_solve: the iteration limit came first; x holds
                                  the last iterate                                    */
  CUTCELL_E_INVALID_ARG = -1,  /* null pointer, bad size, inconsistent sizes          */
  CUTCELL_E_UNSUPPORTED = -2,  /* D not in {2,3}, Q not in {2,4}, R_n out of [1, 4],
                                  a face with more rows than the largest kernel bin   */
  CUTCELL_E_WORKSPACE = -3,    /* workspace missing or smaller than required          */
  CUTCELL_E_HIP = -4,          /* a HIP runtime call failed (message kept)            */
  CUTCELL_E_CAPACITY = -5,     /* output arrays smaller than the sizes require        */
  CUTCELL_E_BREAKDOWN = -6     /* cutcell_solve: the residual became non-finite        */
};

/* Per-face status.  Sec. 2.2.1 assumes enough neighbours for a full-rank system; a face
 * without them gets val = 0 and one of these codes. */
enum {
  CUTCELL_STATUS_OK = 0,
  CUTCELL_STATUS_INSUFFICIENT_ROWS = 1, /* fewer rows than monomials (N < M)            */
  CUTCELL_STATUS_RANK_DEFICIENT = 2,    /* min |R_kk| <= 1e-12 max |R_kk| for the
                                           Householder R factor of the column-
                                           equilibrated W A                             */
  CUTCELL_STATUS_NONFINITE = 3          /* a non-finite moment or weight in the system  */
};

typedef void* cutcell_stream_t; /* hipStream_t */

/* Launch schedule and kernel widths of the stencil solves, per row-count bin b (faces
 * with 16 b < N <= 16 (b + 1) rows).  Results do not depend on it (every face is solved
 * the same way, padding rows are exact zeros); only the order in which workgroups take
 * faces, and the kernel width they run at, do.
 *   xcd_chunks[b]     1: faces in bin order over the workgroups; 8: the bin is cut into
 *                     8 contiguous chunks, one per XCD (MI355X deals workgroups to its 8
 *                     XCDs in turn, each with its own L2), so faces that share rows share
 *                     an L2.
 *   blocks_per_xcd[b] 0: one workgroup per face; > 0: a persistent grid of
 *                     xcd_chunks * blocks_per_xcd workgroups that walk their chunk.
 *   split[b]          which kernel widths take the bin's faces with at most 16 (b+1) - 8
 *                     rows (part 0) and at most 16 (b+1) - 4 rows (part 1), where such
 *                     narrower instances are compiled (they hold more waves per CU): 0
 *                     parts 0 and 1 each at its own width (the default); 1 the whole bin
 *                     at 16 (b+1) rows; 2 part 0 narrower only; 3 parts 0 and 1 at
 *                     16 (b+1) - 4.
 * cutcell_autotune fills it by timing candidates on the caller's workload. */
typedef struct {
  int32_t xcd_chunks[8];
  int32_t blocks_per_xcd[8];
  int32_t split[8];
} cutcell_tuning;

typedef struct {
  int32_t dim;          /* D: 2 or 3                                                   */
  int32_t n[3];         /* cells per direction (n[2] ignored when D = 2)               */
  double h;             /* grid spacing                                                */
  int32_t order;        /* Q: 2 or 4 (interpolant degree Q, P = Q + 1; Sec. 2.3)       */
  int32_t path_radius;  /* R_n, 1..4 (the paper uses 2 for Q = 2 and 3 for Q = 4)      */
  const cutcell_tuning* tuning;  /* host pointer, or NULL for one workgroup per face in
                                    bin order                                          */
  int32_t eb_bc;        /* CUTCELL_BC_DIRICHLET or CUTCELL_BC_NEUMANN on every EB face
                           (box faces are always Dirichlet); see "Boundary data" above  */
  int32_t reuse_templates; /* 1: solve one face per (geometry, direction) among the faces
                           whose systems are bitwise identical -- grid faces whose cells
                           within the path radius (plus one) are plain interior volumes
                           carrying, with their faces, exactly the moments of a reference
                           cell -- and copy its stencil to the others.  The output is bit
                           for bit that of a build without reuse; only the work differs
                           (cutcell_last_reused_faces counts the copies).  0: solve every
                           face, as the paper does.                                     */
  int32_t weight_custom;   /* 0: the paper's weights W = (2d)^-5 beyond half a cell
                           (Sec. 2.4); 1: W = (2d)^-weight_power instead (weight studies;
                           0 gives unweighted least squares)                            */
  double weight_power;  /* used when weight_custom = 1; in [0, 16]                      */
  int32_t factorization; /* how the least-squares systems are solved (Sec. 2.2.1, eq.
                           'stencil equation solution'; the stencil is the same either
                           way, to the tolerance below):
                           CUTCELL_FACTOR_AUTO: the Gram matrix of the column-equilibrated
                             W A (matrix cores), inverted by Gauss-Jordan, with one step of
                             refinement (its residual in compensated arithmetic when the
                             estimated cond(W A) exceeds about 3e3; the rows of cells with
                             kappa < 1e-3 in double-double); a face whose smallest pivot is
                             at most 1e-4 of the largest, whose estimated cond(W A) exceeds
                             3e4, or whose refinement step moved the stencil by more than
                             1e-6 of its size, is solved again by the QR path;
                           CUTCELL_FACTOR_QR: every face by the QR path -- Householder QR
                             of W A held in shared memory, with the rows and the
                             refinement residuals of the augmented system in
                             double-double arithmetic, so the stencil is correct to FP64
                             rounding while cond(W A) * eps < 1;
                           CUTCELL_FACTOR_GRAM: every face on the Gram path, none sent to
                             QR (rank deficiency from its pivots); accurate to about
                             eps cond(W A) while the refinement converges -- for callers
                             that want every face by one method (e.g. finite differences
                             of the stencils, where a face changing path between the
                             perturbed builds would show as noise).                     */
} cutcell_opts;

enum { CUTCELL_BC_DIRICHLET = 0, CUTCELL_BC_NEUMANN = 1 };
enum { CUTCELL_FACTOR_AUTO = 0, CUTCELL_FACTOR_QR = 1, CUTCELL_FACTOR_GRAM = 2 };

/* One geometry: device arrays in the layouts above. */
typedef struct {
  const double* vol_mom;     /* [ncell][M]                                             */
  const double* face_mom[3]; /* [nface_d][Mf] for d < D                                */
  int32_t n_eb;              /* number of EB faces                                     */
  const int32_t* eb_cell;    /* [n_eb] strictly ascending cell indices                 */
  const double* eb_mom;      /* [n_eb][M]                                              */
  const double* eb_nmom;     /* [n_eb][D][M1]                                          */
} cutcell_geom;

/* Totals over the batch (host struct, filled by cutcell_query). */
typedef struct {
  int64_t n_vol, n_eb, n_box, n_phi, n_face, nnz;
  int32_t max_rows;     /* largest row count N of any face                             */
  int32_t n_geom;
} cutcell_sizes;

/* Build outputs: device arrays allocated by the caller with the sizes from
 * cutcell_query (n_geom entries plus one for the offset arrays). */
typedef struct {
  int64_t* row_ptr;     /* [n_face + 1]                                                */
  int32_t* col;         /* [nnz]   Phi indices (global over the batch), ascending per row */
  double* val;          /* [nnz]   physical stencil values                             */
  int8_t* status;       /* [n_face] CUTCELL_STATUS_*                                   */
  int32_t* vol_face;    /* [n_vol][2D+1] flux faces of each volume: for d < D the low
                           face (slot 2d) and high face (slot 2d+1), then the EB face;
                           -1 where there is none                                       */
  double* vol_scale;    /* [n_vol] 1 / (kappa_v h^D)                                    */
  int64_t* phi_off;     /* [n_geom + 1] start of each geometry's Phi block              */
  int64_t* vol_off;     /* [n_geom + 1] start of each geometry's volumes                */
  int64_t* face_off;    /* [n_geom + 1] start of each geometry's flux faces             */
  int32_t* tmpl;        /* [n_face] or NULL (then not written): the face whose stencil this
                           face's was copied from (cutcell_opts.reuse_templates), -1 for a
                           face solved itself -- the input of cutcell_pack_count           */
} cutcell_stencils;

/* Bytes of device workspace the calls below need for this grid and batch size. */
size_t cutcell_workspace_bytes(const cutcell_opts* opts, int32_t n_geom);

/* Enumerates volumes, boundary faces and flux faces (Sec. 2.1) and counts each face's
 * neighbour rows (Sec. 2.4) for a batch of n_geom geometries that share `opts`; fills
 * *sizes.  Synchronises `stream`. */
int cutcell_query(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                  void* workspace, size_t workspace_bytes, cutcell_sizes* sizes,
                  cutcell_stream_t stream);

/* Builds every face's stencil s = W (A^T W)^+ F (Sec. 2.2.1 and Sec. 2.4) into *out,
 * whose arrays must hold `sizes` (from cutcell_query on the same inputs).  Returns
 * CUTCELL_W_FLAGGED_FACES when some face got a nonzero status.  Synchronises `stream`. */
int cutcell_build_stencils(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                           const cutcell_sizes* sizes, cutcell_stencils* out,
                           void* workspace, size_t workspace_bytes, cutcell_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cutcell_build_stencils with the
 * library's own scratch in place of the caller's workspace.  The scratch is one static
 * device array of CUTCELL_STATIC_SCRATCH_BYTES per GPU, held from the library's loading to
 * the end of the process; a batch whose workspace (cutcell_workspace_bytes) is larger is
 * refused with CUTCELL_E_WORKSPACE before any work (256 MiB holds one geometry up to 64^3 at
 * order 4, which needs about 198 MiB).  The call allocates nothing and records no profiling events.  Every call on one
 * GPU uses that GPU's array, which keeps the last call's contents (the build clears what it
 * needs), so calls that overlap on one GPU -- other threads, other streams -- race and must
 * be serialised by the caller.  `sizes` comes from cutcell_query (with a workspace of the
 * caller's, e.g. at set-up).  Outputs and return codes as cutcell_build_stencils.
 * Synchronises `stream`. */
#define CUTCELL_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
int cutcell_build_stencils_noalloc(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                                   const cutcell_sizes* sizes, cutcell_stencils* out, cutcell_stream_t stream);

/* Builds the stencils like cutcell_build_stencils and, on the way, times every candidate
 * schedule of each row-count bin (best of `reps` runs, HIP events on `stream`), writing the
 * fastest to *tuning and each bin's best time in milliseconds to best_ms[8] (-1 for empty
 * bins; may be NULL).  opts->tuning is ignored.  Synchronises `stream`. */
int cutcell_autotune(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                     const cutcell_sizes* sizes, cutcell_stencils* out, void* workspace, size_t workspace_bytes,
                     int32_t reps, cutcell_tuning* tuning, double* best_ms, cutcell_stream_t stream);

/* Applies the operator (Sec. 2.2, eq. 'laplacian over V'; Sec. 3.3):
 *   flux[f] = sum_j val[j] phi[col[j]]   (output, [n_face]; also the pass's scratch)
 *   lphi[v] = vol_scale[v] * sum over v's faces of sigma * flux
 * phi: [n_phi], lphi: [n_vol].  Asynchronous on `stream`. */
int cutcell_apply(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                  const double* phi, double* lphi, double* flux, cutcell_stream_t stream);

/* Compressed stencils for repeated applies (Sec. 4, standard interior stencils; Fig. 2b):
 * a face whose stencil was copied from a template face (cutcell_opts.reuse_templates) is
 * stored as its template's slot plus one Phi index per run of consecutive columns -- its
 * values are the slot's (a copy of the template's row), its columns base[run] + position
 * in the run -- instead of its own columns and values.  cutcell_pack_count checks every
 * face against its template (st->tmpl) and packs it only where that reproduces its CSR
 * row exactly (row count, columns, values bit for bit); the others stay CSR rows of `st`,
 * which must stay as they are while the packed form is used. */
typedef struct {
  int64_t n_packed;   /* faces stored as a slot plus run bases                           */
  int32_t n_slot;     /* template faces                                                  */
  int32_t max_runs;   /* runs of consecutive columns per template, at most               */
  int32_t max_rows;   /* rows per template, at most                                      */
} cutcell_packed_sizes;

typedef struct {
  uint8_t* flag;      /* [n_face] 1: the face is packed                                  */
  uint8_t* phase;     /* [n_face] lane of the face's first entry in cutcell_apply's flux
                         pass (its row offset from the first face of its group, mod 64)  */
  int32_t* face;      /* [n_packed] the packed faces, ascending                          */
  int32_t* slot;      /* [n_packed] the slot of each one's template                      */
  int32_t* base;      /* [n_packed][max_runs] Phi index of each run's first entry        */
  int32_t* slot_face; /* [n_slot] the template face of each slot                         */
  int32_t* slot_rows; /* [n_slot] its row count                                          */
  int32_t* slot_tab;  /* [n_slot][max_rows] per entry: run | (position in the run) << 16 */
  double* slot_val;   /* [n_slot][max_rows] its values                                   */
} cutcell_packed;

/* Bytes of workspace cutcell_pack_count and cutcell_pack_fill need. */
size_t cutcell_pack_workspace_bytes(const cutcell_sizes* sizes);

/* Counts the faces that pack and sizes the tables into *out.  st->tmpl is required.
 * Synchronises `stream`. */
int cutcell_pack_count(const cutcell_sizes* sizes, const cutcell_stencils* st, cutcell_packed_sizes* out,
                       void* workspace, size_t workspace_bytes, cutcell_stream_t stream);

/* Fills *out (arrays sized from *psizes, as cutcell_pack_count returned them for the same
 * stencils; CUTCELL_E_CAPACITY if they no longer match) for applies in dimension `dim`
 * (the phases follow that dimension's flux pass).  Synchronises `stream`. */
int cutcell_pack_fill(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                      const cutcell_packed_sizes* psizes, cutcell_packed* out, void* workspace,
                      size_t workspace_bytes, cutcell_stream_t stream);

/* cutcell_apply on the compressed stencils (pk from cutcell_pack_fill on `st`, same dim):
 * flux and lphi equal cutcell_apply's bit for bit -- every face's products are added in
 * the order cutcell_apply adds them.  One launch takes the faces left as CSR rows of `st`
 * (cutcell_apply's groups, packed faces skipped) and the packed ones.  Asynchronous on
 * `stream`. */
int cutcell_apply_packed(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                         const cutcell_packed_sizes* psizes, const cutcell_packed* pk, const double* phi,
                         double* lphi, double* flux, cutcell_stream_t stream);

/* Transposed structure of the stencils (for the adjoints): for every Phi entry k, the
 * CSR positions j with col[j] = k, ascending, in nz[col_ptr[k] .. col_ptr[k+1]), and the
 * face (CSR row) of each in nz_face[].  Arrays sized from cutcell_sizes. */
typedef struct {
  int64_t* col_ptr;     /* [n_phi + 1]                                                  */
  int32_t* nz;          /* [nnz]                                                        */
  int32_t* nz_face;     /* [nnz]                                                        */
} cutcell_transpose;

/* Gradients with respect to one geometry's inputs, same layouts as cutcell_geom. */
typedef struct {
  double* vol_mom;      /* [ncell][M]                                                   */
  double* face_mom[3];  /* [nface_d][Mf] for d < D                                      */
  double* eb_mom;       /* [n_eb][M]     (may be NULL when n_eb = 0)                    */
  double* eb_nmom;      /* [n_eb][D][M1] (may be NULL when n_eb = 0)                    */
} cutcell_geom_grad;

/* Bytes of workspace cutcell_build_transpose needs (0 if nnz >= 2^31: unsupported). */
size_t cutcell_transpose_workspace_bytes(const cutcell_sizes* sizes);

/* Builds the transpose of the stencils in `st` (output of cutcell_build_stencils) into
 * *out by a stable sort of the CSR positions by column.  Asynchronous on `stream`. */
int cutcell_build_transpose(const cutcell_sizes* sizes, const cutcell_stencils* st, cutcell_transpose* out,
                            void* workspace, size_t workspace_bytes, cutcell_stream_t stream);

/* Adjoint of cutcell_apply (the transpose of the linear map Phi -> L(Phi) of Sec. 2.2,
 * eq. 'laplacian over V', and its derivatives in the stencil values and the volume scales).
 * Given lphi_bar = dl/dL [n_vol]:
 *   flux_bar[f] = sum over the volumes v of f of sigma_vf vol_scale[v] lphi_bar[v]   (out, required)
 *   phi_bar[k]  = sum_{j: col[j] = k} val[j] flux_bar[face(j)]                       (out, required)
 *   val_bar[j]  = flux_bar[face(j)] phi[col[j]]             (out, optional; needs phi)
 *   scale_bar[v]= lphi_bar[v] sum_f sigma_vf flux[f]        (out, optional; needs the
 *                 forward's flux output)  -- dl/d vol_scale, which
 *                 cutcell_stencils_backward turns into a kappa gradient.
 * Asynchronous on `stream`. */
int cutcell_apply_adjoint(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                          const cutcell_transpose* tr, const double* phi, const double* flux,
                          const double* lphi_bar, double* phi_bar, double* val_bar, double* scale_bar,
                          double* flux_bar, cutcell_stream_t stream);

/* Bytes of workspace cutcell_stencils_backward needs (it includes the build's). */
size_t cutcell_backward_workspace_bytes(const cutcell_opts* opts, const cutcell_sizes* sizes);

/* Adjoint of cutcell_build_stencils (Dirichlet EB conditions only: CUTCELL_E_UNSUPPORTED
 * for Neumann) (the derivative of s = W (A^T W)^+ F of Sec. 2.2.1
 * with the rows, centring and weights of Sec. 2.4): given val_bar = dl/dval [nnz] and,
 * optionally, scale_bar = dl/dvol_scale [n_vol] (from cutcell_apply_adjoint), writes
 * dl/d(inputs) into grads[g] for every geometry (overwritten, not accumulated; zero where
 * an input has no influence, and zero for faces with a nonzero status, whose stencil is
 * zero).  The EB face's x0 (the cut volume's centroid) makes the volume's moments 0..D
 * enter every row of that face; that dependence is included.  weight_bar (optional,
 * [nnz]) receives dl/dW_i of every row with the other inputs fixed.  `st` and `tr` must be
 * the outputs of cutcell_build_stencils / cutcell_build_transpose for the same inputs.
 * Synchronises `stream`. */
int cutcell_stencils_backward(const cutcell_geom* geoms, int32_t n_geom, const cutcell_opts* opts,
                              const cutcell_sizes* sizes, const cutcell_stencils* st,
                              const cutcell_transpose* tr, const double* val_bar, const double* scale_bar,
                              const cutcell_geom_grad* grads, double* weight_bar, void* workspace,
                              size_t workspace_bytes, cutcell_stream_t stream);

/* The operator as one sparse matrix over volumes (Sec. 2.2, eq. 'laplacian over V'):
 *   lphi[v] = sum_{k in row v} val[k] phi[col[k]]  =  L_v of cutcell_apply,
 * row v the sigma-signed, vol_scale-weighted merge of the stencil rows of v's faces
 * (columns ascending and distinct; explicit zeros kept).  Device arrays owned by the
 * caller: row_ptr [n_vol + 1], col and val [nnz] from cutcell_laplacian_count. */
typedef struct {
  int64_t* row_ptr;
  int32_t* col;
  double* val;
} cutcell_laplacian;

/* Bytes of workspace cutcell_laplacian_count needs. */
size_t cutcell_laplacian_workspace_bytes(const cutcell_sizes* sizes);

/* Row lengths and offsets of the volume matrix of the stencils `st`: writes row_ptr
 * [n_vol + 1] (device) and the number of entries to *nnz (host).  Synchronises `stream`. */
int cutcell_laplacian_count(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st, int64_t* row_ptr,
                            int64_t* nnz, void* workspace, size_t workspace_bytes, cutcell_stream_t stream);

/* Fills col and val of `lap` (row_ptr from cutcell_laplacian_count on the same stencils).
 * Deterministic: equal columns of different faces are summed in face-slot order (low,
 * high per direction, then the EB face).  Asynchronous on `stream`. */
int cutcell_laplacian_fill(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                           const cutcell_laplacian* lap, cutcell_stream_t stream);

/* lphi [n_vol] = lap phi (phi [n_phi]).  Agrees with cutcell_apply up to the order of
 * the additions.  Asynchronous on `stream`. */
int cutcell_apply_laplacian(const cutcell_sizes* sizes, int32_t dim, const cutcell_laplacian* lap, const double* phi,
                            double* lphi, cutcell_stream_t stream);

/* Bytes of workspace cutcell_solve needs for `restart` Krylov vectors (0 if restart is
 * outside [1, 1024]).  About (restart + 8) n_vol + 2 n_phi + n_face doubles. */
size_t cutcell_solve_workspace_bytes(const cutcell_sizes* sizes, int32_t restart);

/* Solves the discrete Poisson problem L(Phi) = rhs for the volume values of Phi
 * (Sec. 3.2; Sec. 2.2, eq. 'laplacian over V'), the EB and box entries of Phi held fixed
 * at the Dirichlet data given in phi_bc.  L is affine in the volume values x, L = A x +
 * L([0 | bc]); restarted GMRES(restart) with right Jacobi preconditioning (D = diag A,
 * computed from the stencils) solves A x = rhs - L([0 | bc]).  The paper uses GMRES with
 * an algebraic multigrid preconditioner (Sec. 3.2); this solver keeps the Krylov part
 * and replaces the preconditioner by the diagonal.
 *   phi_bc  [n_phi]  Phi with the boundary values; its volume entries are ignored
 *   rhs     [n_vol]  the right-hand side per volume (the volume average of the source,
 *                    in the units of L)
 *   x       [n_vol]  in: the initial guess; out: the volume values of the solution
 *   restart          Krylov vectors per cycle, 1..1024
 *   max_iters        limit on matrix-vector products of the Arnoldi steps
 *   rtol             stop when ||rhs - L([x | bc])||_2 <= rtol ||rhs - L([0 | bc])||_2,
 *                    tested on the true residual
 *   iters, relres    (host, may be NULL) iterations taken and the final relative residual
 *   lap              (may be NULL) the volume matrix of the same stencils: the products
 *                    then take one gather per volume (cutcell_apply_laplacian) instead of
 *                    the face fluxes and their divergence
 * Returns CUTCELL_OK, CUTCELL_W_NOT_CONVERGED, or an error.  Inner products are summed in
 * a fixed order (512 partials per product), so the result does not vary between runs.
 * Synchronises `stream` (every Arnoldi step reads its inner products back). */
int cutcell_solve(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st,
                  const cutcell_laplacian* lap, const double* phi_bc, const double* rhs, double* x,
                  int32_t restart, int32_t max_iters, double rtol, void* workspace, size_t workspace_bytes,
                  int32_t* iters, double* relres, cutcell_stream_t stream);

/* Eigenvalues of an n x n upper Hessenberg matrix H (host arrays, row-major with leading
 * dimension ld; entries below the subdiagonal are ignored) into re[n], im[n]: shifted QR
 * iterations in complex arithmetic (Wilkinson shifts, deflation from the bottom).  Host
 * only, no device work.  Returns CUTCELL_OK, or CUTCELL_E_BREAKDOWN if it fails to
 * converge. */
int cutcell_hessenberg_eigs(int32_t n, const double* H, int32_t ld, double* re, double* im);

/* Bytes of workspace cutcell_ritz needs (mode 1 includes the inner solves'). */
size_t cutcell_ritz_workspace_bytes(const cutcell_sizes* sizes, int32_t steps, int32_t mode, int32_t inner_restart);

/* Ritz values of the volume operator A (L restricted to the volume values, every boundary
 * entry of Phi zero; the spectra of Sec. 3.4 and 3.5) from `steps` Arnoldi steps on the
 * GPU with a fixed pseudo-random start vector and classical Gram-Schmidt twice:
 *   mode 0: on A -- the eigenvalues of largest magnitude converge first (lambda_min, and
 *           any large positive eigenvalue of an unstable operator);
 *   mode 1: on A^-1 (each step a cutcell_solve with inner_rtol, inner_restart,
 *           inner_max_iters), values inverted -- the eigenvalues nearest 0 (lambda_max of
 *           a stable operator).
 * lap (may be NULL): the volume matrix for the products.  ritz_re/ritz_im [steps] (host)
 * receive *n_ritz values (fewer than steps if an invariant subspace is found); ritz_res
 * (host, may be NULL) their relative residuals |A u - theta u| / |theta| (of A^-1 in mode
 * 1; -1 when steps > 256): only values with small residuals are eigenvalues -- for a
 * strongly non-normal operator the others can lie far outside the spectrum.  Returns
 * CUTCELL_W_NOT_CONVERGED if an inner solve did not converge.  Synchronises `stream`. */
int cutcell_ritz(const cutcell_sizes* sizes, int32_t dim, const cutcell_stencils* st, const cutcell_laplacian* lap,
                 int32_t mode, int32_t steps, double inner_rtol, int32_t inner_restart, int32_t inner_max_iters,
                 double* ritz_re, double* ritz_im, double* ritz_res, int32_t* n_ritz, void* workspace,
                 size_t workspace_bytes, cutcell_stream_t stream);

/* Observability: when enabled (per calling thread), cutcell_build_stencils records HIP
 * events on its stream between its phases, and cutcell_last_profile copies the last
 * build's phase durations in milliseconds into ms[0 .. n-1]: enumeration, row counts and
 * their scan, neighbour fill, binning, stencil solves, volume tables (-1 where a phase did
 * not run).  Returns the number of phases (6), or CUTCELL_E_INVALID_ARG. */
void cutcell_set_profiling(int enable);
int cutcell_last_profile(double* ms, int32_t n);

/* Faces whose stencil the last build on the calling thread copied from a template
 * (cutcell_opts.reuse_templates), 0 without reuse. */
int64_t cutcell_last_reused_faces(void);

/* Faces of each row-count bin (cutcell_tuning) in the last build on the calling thread
 * (solved there, not copied from templates) into counts[0 .. n-1]: which bins a tuning
 * for this workload needs.  Returns the number of bins (8), or CUTCELL_E_INVALID_ARG. */
int cutcell_last_bin_faces(int64_t* counts, int32_t n);

/* Faces of the last build on the calling thread that the Householder QR path solved
 * (all of them under CUTCELL_FACTOR_QR). */
int64_t cutcell_last_qr_faces(void);

/* Message of the last error on the calling thread ("" if none). */
const char* cutcell_last_error(void);

/* CUTCELL_ABI_VERSION of the loaded library. */
int cutcell_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CUTCELL_H */
