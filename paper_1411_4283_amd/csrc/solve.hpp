// The Poisson solve with the operator (Sec. 3.2).
#pragma once

#include "kernels.hpp"

namespace cutcell {

// Poisson solve with the operator (Sec. 3.2): restarted, right-Jacobi-preconditioned GMRES
struct SolveOp {
  int D;
  long long n_vol, n_phi, n_face;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  const int32_t* vol_face;
  const double* vol_scale;
  hipStream_t st;
  // optional volume matrix (then the products are one gather per volume)
  const int64_t* lap_ptr = nullptr;
  const int32_t* lap_col = nullptr;
  const double* lap_val = nullptr;
};
// the volume matrix of the operator (laplacian.hip)
size_t laplacian_temp_bytes(long long n_vol);
int laplacian_count(int D, long long n_vol, const int64_t* row_ptr, const int32_t* col, const double* val,
                    const int32_t* vol_face, const double* vol_scale, int64_t* lap_ptr, int64_t* nnz, char* ws,
                    size_t ws_bytes, hipStream_t st);
int laplacian_fill(int D, long long n_vol, const int64_t* row_ptr, const int32_t* col, const double* val,
                   const int32_t* vol_face, const double* vol_scale, const int64_t* lap_ptr, int32_t* lap_col,
                   double* lap_val, hipStream_t st);
int apply_laplacian(int D, long long n_vol, const int64_t* lap_ptr, const int32_t* lap_col, const double* lap_val,
                    const double* phi, double* lphi, hipStream_t st);
size_t solve_workspace_bytes(long long n_vol, long long n_phi, long long n_face, int m);
int solve_poisson(const SolveOp& op, int G, const int64_t* phi_off, const int64_t* vol_off, const double* phi_bc,
                  const double* f, double* x, int m, int max_iters, double rtol, char* ws, size_t ws_bytes,
                  int* iters_out, double* relres_out);

// extreme eigenvalues by Arnoldi's method (mode 0: A, mode 1: shift-invert about 0)
int hessenberg_eigs(int n, const double* H, int ld, double* re, double* im);
size_t ritz_workspace_bytes(long long n_vol, long long n_phi, long long n_face, int k, int inner_m);
int ritz_values(const SolveOp& op, int G, const int64_t* phi_off, const int64_t* vol_off, int mode, int k,
                double inner_rtol, int inner_m, int inner_max, double* ritz_re, double* ritz_im, double* ritz_res,
                double* hess, int* n_out, char* ws, size_t ws_bytes);

}  // namespace cutcell
