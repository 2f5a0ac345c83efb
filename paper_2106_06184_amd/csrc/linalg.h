// Dense products, sparse glue and Krylov kernels (interface shared by the host driver).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace bem {

// One dense product y (+)= alpha A x [+ alpha2 A2 x2], A and A2 row-major complex with the same
// shape and storage (float64 or float32).
struct GemvDesc {
  const void* A;      // double2* (fp64) or float2* (fp32) rows x cols, leading dimension lda
  const void* A2;     // optional second matrix (same shape, lda2), or nullptr
  int64_t lda, lda2;
  int64_t rows, cols;
  const double2* x;   // cols, float64 complex
  const double2* x2;
  double2* y;         // rows, float64 complex
  double2 alpha, alpha2;
  int accumulate;     // 0: y = ... ; 1: y += ...
  int fp32;           // storage of A (and A2): 0 float64; 1 float32 (float32 arithmetic);
                      // 2 float32 entries in float64 arithmetic
  int64_t tile0;      // first row tile of this descriptor (filled by the launcher)
  int64_t ldx, ldx2, ldy;  // column strides of x, x2, y for multi-column products
};
// Device-side copy of a descriptor (what the kernel reads), passed by value in a pack that
// stays under 1 KiB of kernel arguments.
struct GemvDev {
  const void* A;
  const void* A2;
  int64_t lda, lda2;
  int64_t rows, cols;
  const double2* x;
  const double2* x2;
  double2* y;
  double ar, ai, a2r, a2i;  // alpha, alpha2 (8-byte aligned: keeps the pack dense)
  int accumulate;
  int fp32;
  int64_t tile0;
};
constexpr int kMaxGroup = 8;
struct GemvPack {
  int n;
  GemvDev d[kMaxGroup];
};
static_assert(sizeof(GemvPack) <= 1024, "grouped GEMV arguments must stay under 1 KiB");

// Runs all descriptors (any number; kMaxGroup per launch) with their rows spread over the grid.
// Descriptors travel as kernel arguments; the call is asynchronous on `st`.
void launch_gemv_grouped(const GemvDesc* host_descs, int n, hipStream_t st);

// Multi-RHS dense product Y (+)= alpha A X on float32 matrix cores (complex 4M split) or
// float64 (plain VALU): X column-major cols x nrhs (ldx), Y column-major rows x nrhs (ldy).
struct GemmDesc {
  const void* A;
  int64_t lda, rows, cols;
  const double2* X;
  int64_t ldx;
  double2* Y;
  int64_t ldy;
  int64_t nrhs;
  double2 alpha;
  int accumulate;
  int fp32;
};
void launch_gemm(const GemmDesc& d, void* ws, size_t ws_bytes, hipStream_t st);
// Runs the descriptors for R columns: R = 1 -> one grouped GEMV launch; R > 1 -> one matrix-core
// GEMM per descriptor (float32 or float64 storage), using ws (gemm_workspace_bytes) for the
// real-embedded right-hand sides.
void launch_products(const std::vector<GemvDesc>& ds, int R, void* ws, size_t ws_bytes, hipStream_t st);

// ---- batched Krylov kernels: R independent Krylov spaces that share their products.  Basis
// vector i of column c at V + (i R + c) ldv (each step's R vectors form one n x R column-major
// block); per-column small arrays at base + c * stride.  Reductions are deterministic (fixed
// chunking and summation order).  `part` needs R (j1 max) bkry_chunks(n) complex entries.
int bkry_chunks(int64_t n);
// h[c hstride + i] = V_i,c^H w_c for i < j1
void launch_bmdot(const double2* V, int64_t ldv, int R, int j1, const double2* W, int64_t ldw, int64_t n,
                  double2* part, double2* h, int64_t hstride, hipStream_t st);
// w_c += sign sum_{i < j_c} V_i,c h[c hstride + i], j_c = jr ? jr[c] : j1
// Step j >= 1 of Gram-Schmidt with delayed reorthogonalisation (see k_bdcgs2_coef): one pass
// over V_0..V_j for both projections (into part1 / part2, R (j + 1) bkry_chunks(n) entries each),
// the per-column coefficients (H columns j - 1 corrected and j written; coef: 2 (j + 1) entries
// per column at c cstride; rinv: R), and, with update, one pass for v_j <- (V_j - V a) / r and
// Y <- (Y - V cf) / r.  Without update only the column j - 1 correction is wanted (the last step
// of a cycle; Y unused).
void launch_bdcgs2(double2* V, int64_t ldv, int R, int j, double2* Y, int64_t ldy, int64_t n, double2* part1,
                   double2* part2, double2* H, int64_t hs, int64_t ldh, double2* coef, int64_t cstride, double* rinv,
                   const int* frozen, bool update, hipStream_t st);
void launch_bmupdate(const double2* V, int64_t ldv, int R, int j1, const int* jr, const double2* h, int64_t hstride,
                     double sign, double2* W, int64_t ldw, int64_t n, hipStream_t st);
// out[c ostride] = (||w_c||_2, 0)
void launch_bnorm(const double2* W, int64_t ldw, int R, int64_t n, double2* part, double2* out, int64_t ostride,
                  hipStream_t st);
// w_c = w_c / nrm[c nstride] (0 when the norm is 0 or frozen[c] is set; frozen may be null)
void launch_bscale_inv(double2* W, int64_t ldw, int R, int64_t n, const double2* nrm, int64_t nstride,
                       const int* frozen, hipStream_t st);
// Givens step j of every column: Hessenberg column j of column c at H + c hs + j ldh, rotated
// into the same place of HR (HR = H: in place); cs, sn, y with stride m+1, g and h2 with stride
// m+2; res[c] = |g_c[j+1]|.
void launch_bgivens(const double2* H, double2* HR, int64_t hs, int64_t ldh, int j, double2* cs, double2* sn,
                    double2* g, double* res, const double2* h2, int m, int R, hipStream_t st);
// y_c = R_c^{-1} g_c over the leading jr[c] x jr[c] block
void launch_bbacksolve(const double2* H, int64_t hs, int64_t ldh, const int* jr, const double2* g, double2* y, int m,
                       int R, hipStream_t st);
// g_c = (beta[c bstride], 0, ..., 0)
void launch_binit_g(double2* g, int m, const double2* beta, int64_t bstride, int R, hipStream_t st);
// U[:, c] = X[:, idx[c]]
void launch_gather_cols(const double2* X, int64_t ldx, double2* U, int64_t ldu, const int* idx, int64_t n, int R,
                        hipStream_t st);
// X[:, idx[c]] (+)= U[:, c]
void launch_scatter_cols(const double2* U, int64_t ldu, double2* X, int64_t ldx, const int* idx, int64_t n, int R,
                         int accumulate, hipStream_t st);

// ---- sparse glue (float64 complex vectors).  Every launcher processes R columns (grid.y),
// column r of an argument starting at pointer + r * ld (ld unused when R = 1).
// Charges: full[t] (per triangle) from reduced w (kept triangles); the last triangle of each
// object gets minus the sum of the object's other charges.
void launch_expand_charge(const double2* w, double2* full, const int64_t* obj_tri, int64_t nobj,
                          double2 scale, hipStream_t st, int R = 1, int64_t ldw = 0, int64_t ldf = 0);
// y[n] (+)= s * sedge[n] * (z[T+(n)] - z[T-(n)])      (D^T z; sedge may be null)
void launch_DT(const double2* z, const int32_t* tp, const int32_t* tm, int64_t ne, double2 s, const double2* sedge,
               double2* y, int accumulate, hipStream_t st, int R = 1, int64_t ldz = 0, int64_t ldy = 0);
// Reduced continuity rows: y[q] = s1 * (D u)[t(q)] + s2 * w[q] for kept triangles q (F D u + s2 w)
void launch_FD(const double2* u, const int32_t* tri_edge, const int8_t* tri_sign, const int32_t* kept_tri,
               int64_t nq, double2 s1, const double2* w, double2 s2, double2* y, hipStream_t st, int R = 1,
               int64_t ldu = 0, int64_t ldw = 0, int64_t ldy = 0);
// y (+)= s * S x for a CSR real sparse matrix S
void launch_spmv(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, const double2* x,
                 double2 s, double2* y, int accumulate, hipStream_t st, int R = 1, int64_t ldx = 0, int64_t ldy = 0);
// y1 (+)= s1 A x and y2 (+)= s2 A x (acc1, acc2: accumulate) in one pass, R columns.
void launch_spmv2(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, const double2* x,
                  int64_t ldx, double2 s1, double2* y1, int64_t ldy1, int acc1, double2 s2, double2* y2, int64_t ldy2,
                  int acc2, hipStream_t st, int R);
// z = a*x + b*y (elementwise, n; x or y may be null)
void launch_axpby(int64_t n, double2 a, const double2* x, double2 b, const double2* y, double2* z,
                  hipStream_t st, int R = 1, int64_t ldx = 0, int64_t ldy = 0, int64_t ldz = 0);
// Workspace bytes of launch_gemm for products of blocks with at most n rows and n complex
// columns and nrhs right-hand sides (either storage precision).
size_t gemm_workspace_bytes(int64_t n, int64_t nrhs);
// out[i] = A[i][i], i < n (row-major, leading dimension ld)
void launch_diag(const double2* A, int64_t ld, int64_t n, double2* out, hipStream_t st);
void launch_cast_f32(const double2* src, int64_t rows, int64_t cols, int64_t lds, float2* dst, int64_t ldd,
                     hipStream_t st);
// dst[r][c] = src[r][c] widened to float64, r < rows, c < cols
void launch_cast_f64(const float2* src, int64_t rows, int64_t cols, int64_t lds, double2* dst, int64_t ldd,
                     hipStream_t st);

// ---- Krylov (float64 complex, deterministic reductions)
struct KrylovScratch {
  double2* partial;       // nblk * (mmax + 1)
  unsigned int* counter;  // 1 (zero-initialised once; every kernel leaves it at zero)
  int nblk;
};
// h[i] = sum_n conj(V[i][n]) w[n], i < j   (V rows of length ldv)
void launch_mdot(const double2* V, int64_t ldv, int j, const double2* w, int64_t n, double2* h,
                 const KrylovScratch& ks, hipStream_t st);
// w -= sum_i V[i] h[i] (sign = -1) or x += sum_i V[i] h[i] (sign = +1)
void launch_mupdate(const double2* V, int64_t ldv, int j, const double2* h, double sign, double2* w, int64_t n,
                    hipStream_t st);
// out = ||w||_2 (as the real part of a double2)
void launch_norm(const double2* w, int64_t n, double2* out, const KrylovScratch& ks, hipStream_t st);
// v = w / nrm
void launch_scale_inv(const double2* w, int64_t n, const double2* nrm, double2* v, hipStream_t st);
// Givens step on Hessenberg column j (column stored contiguously at Hcol, j+2 entries; the
// second Gram-Schmidt pass h2[0..j] is added first), rotations cs/sn (mmax), right-hand side g
// (mmax+1); writes |g[j+1]| into res.
void launch_givens(double2* Hcol, int j, double2* cs, double2* sn, double2* g, double* res, const double2* h2,
                   hipStream_t st);
// Back substitution y = R^{-1} g for the leading j x j block (H column-major, ldh), y in place of g.
void launch_backsolve(const double2* H, int64_t ldh, int j, double2* g, double2* y, hipStream_t st);
// g = (beta, 0, ..., 0) with beta = ||r|| read from device
void launch_init_g(double2* g, int mmax, const double2* beta, hipStream_t st);

}  // namespace bem
