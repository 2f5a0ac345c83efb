// Dense inversion, dense-matrix builders and block-preconditioner kernels (interface).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bem {

struct DenseScratch {
  double2* P;        // 64 x 64
  double2* R;        // 256 x n (four row panels)
  double2* C;        // n x 256 (four column panels side by side)
  double2* probe_y;  // n
  double* probe_d;   // n
  double* health;    // 2: smallest pivot ratio, probe error
};

// Device workspace of dense_invert for matrices up to n rows, in elements of double2
// (P, R, C, probe_y, then probe_d and health reinterpreted as doubles).
constexpr size_t dense_scratch_elems(int64_t n) { return size_t(64 * 64) + size_t(513) * size_t(n) + size_t(n) + 2; }
inline DenseScratch dense_scratch_at(double2* base, int64_t n) {
  DenseScratch ws;
  ws.P = base;
  ws.R = ws.P + 64 * 64;
  ws.C = ws.R + size_t(256) * n;
  ws.probe_y = ws.C + size_t(256) * n;
  ws.probe_d = reinterpret_cast<double*>(ws.probe_y + n);
  ws.health = ws.probe_d + n;
  return ws;
}

// In-place inverse of the n x n complex matrix A (row-major, leading dimension ld) by blocked
// Gauss-Jordan elimination without pivoting.  Asynchronous on st.  Breakdown is watched, not
// avoided: the smallest pivot relative to its diagonal block and the relative error
// |A^-1 (A x) - x| / |x| of a fixed probe vector x end in ws.health (read by dense_health).
void dense_invert(double2* A, int64_t n, int64_t ld, DenseScratch& ws, hipStream_t st);

// Health of the last dense_invert with this workspace (synchronises st).  An inversion is
// accepted when every pivot is at least kMinPivotRatio times the largest entry of its diagonal
// block and the probe error is at most kMaxProbeError (NaN fails both): below that the
// elimination without pivoting has broken down, and its inverse is not used.
struct DenseHealth {
  double min_pivot_ratio;
  double probe_error;
};
constexpr double kMinPivotRatio = 1e-12;
constexpr double kMaxProbeError = 1e-6;
DenseHealth dense_health(const DenseScratch& ws, hipStream_t st);
bool dense_health_ok(const DenseHealth& h);

// Inversion without allocation: the same elimination on a workspace that is a fixed device array
// (one per GPU, for matrices of up to kNoAllocMaxN rows, about 17 MB).  noalloc_scratch_init takes
// the array's device address once per device, with that device current (at context creation);
// dense_invert_noalloc then allocates nothing.  Calls that overlap on one GPU share the array and
// race.
constexpr int64_t kNoAllocMaxN = 2048;
constexpr int kMaxDevices = 64;
void noalloc_scratch_init(int device);
void dense_invert_noalloc(int device, double2* A, int64_t n, int64_t ld, DenseHealth* health, hipStream_t st);

// A[i][j] *= rs[i] cs[j] for i < nr, j < nc (device scale vectors, real).
void scale_rows_cols(double2* A, int64_t ld, int64_t nr, int64_t nc, const double* rs, const double* cs,
                     hipStream_t st);
// out[j] = max over rows [r0, r1) of |A[i][c0 + j]|, j < nc; and out[i] = max over columns
// [0, nc) of |A[r0 + i][j]|, i < nr (device outputs).
void col_maxabs(const double2* A, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t nc, double* out,
                hipStream_t st);
void row_maxabs(const double2* A, int64_t ld, int64_t r0, int64_t nr, int64_t nc, double* out, hipStream_t st);
// Equilibration vectors on the device: v[i] = val (i < n); v[i] = |A_ii|^-1/2 for i in [i0, i1)
// (1 where that is not finite); out1[i] = out2[i] = 1 / in[i] (1 where not finite), i < n.
void fill_vec(double* v, int64_t n, double val, hipStream_t st);
void jacobi_vec(const double2* A, int64_t ld, int64_t i0, int64_t i1, double* v, hipStream_t st);
void recip_vec(const double* in, int64_t n, double* out1, double* out2, hipStream_t st);

// Dense M_eq of one object (eq. AEFIEeqvdis) from its diagonal blocks of L^A_l and L^phi_l;
// tp/tm are the object's edges' triangles (device), toff its first triangle; mu = mu_l,
// meps = -1/eps_l, k02 = k0^2.
void build_meq(const double2* LA, int64_t lda, const double2* Lp, int64_t ldp, const int32_t* tp, const int32_t* tm,
               int32_t toff, int64_t ne, int64_t nt, double2 mu, double2 meps, double k02, double2* M, int64_t ldm,
               hipStream_t st);

// Charge-eliminated M_eq of one object: S = mu L^A_l + c D^T L^phi_l D (ne x ne), with
// c = -1/(eps_l k0^2).  Since the charges of D u sum to zero per object, M_eq [u; w] = [r; 0]
// is equivalent to S u = r, w = k0^-2 F D u.
void build_s(const double2* LA, int64_t lda, const double2* Lp, int64_t ldp, const int32_t* tp, const int32_t* tm,
             int32_t toff, int64_t ne, double2 mu, double2 c, double2* S, int64_t lds, hipStream_t st);

// Dense S (nq x nq) = diag * I + G B for a sparse G (CSR over the nq kept charges, columns =
// object-local triangles, the last one being the eliminated charge): (G B)[q][c] = G[q][c] -
// G[q][last].
void build_schur(const int64_t* ptr, const int32_t* idx, const double2* val, int64_t nq, int64_t last, double2 diag,
                 double2* S, int64_t lds, hipStream_t st);

// Block preconditioner of the final system (eq. pcext), per edge n with W = [[w11, w12],
// [w21, w22]] the inverse of its 2x2 diagonal block:
//   stage 1: t[n] = w11 r1[n] + w12 r2[n]
//   stage 2: s_b = e_b[n] (lb[T+] v[T+] - lb[T-] v[T-]), s_i likewise with li and e_i,
//            x1 = w11 (r1 - s_b) + w12 (r2 - s_i),  x2 = w21 (r1 - s_b) + w22 (r2 - s_i)
// (R columns: r-vectors r1, r2, x1, x2 with column stride ldr, temporaries t, v with ldt.)
void launch_pc_stage1(const double2* W, const double2* r1, const double2* r2, int64_t ne, double2* t, hipStream_t st,
                      int R = 1, int64_t ldr = 0, int64_t ldt = 0);
void launch_pc_stage2(const double2* W, const double2* r1, const double2* r2, const double2* v, const double2* lb,
                      const double2* li, double2 e_b, const double2* e_i, const int32_t* tp, const int32_t* tm,
                      int64_t ne, double2* x1, double2* x2, hipStream_t st, int R = 1, int64_t ldr = 0,
                      int64_t ldt = 0);
// Equivalent-configuration preconditioner: t = d r1 ; x1 = t + d e (lb[T+] v[T+] - lb[T-] v[T-])
void launch_peq_stage1(const double2* d, const double2* r1, int64_t ne, double2* t, hipStream_t st, int R = 1,
                       int64_t ldr = 0, int64_t ldt = 0);
void launch_peq_stage2(const double2* d, const double2* t, const double2* v, const double2* lb, double2 e,
                       const int32_t* tp, const int32_t* tm, int64_t ne, double2* x1, hipStream_t st, int R = 1,
                       int64_t ldr = 0, int64_t ldt = 0);

}  // namespace bem
