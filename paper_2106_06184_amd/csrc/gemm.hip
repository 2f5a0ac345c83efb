// Multi-excitation complex products on matrix cores: Y (+)= alpha A X with A complex float32 or
// float64 (interleaved re/im rows, the storage of the dense blocks), X and Y complex float64
// column-major with R columns.
//
// 4M real embedding: reading each complex row of A as 2K real numbers (re, im, re, im, ...),
//   Re(A x) = sum_k' A'[k'] x_re'[k'],  x_re' = (Re x_0, -Im x_0, Re x_1, -Im x_1, ...)
//   Im(A x) = sum_k' A'[k'] x_im'[k'],  x_im' = (Im x_0,  Re x_0, Im x_1,  Re x_1, ...)
// so one real GEMM C (M x 2R) = A' (M x 2K) B (2K x 2R) with B's column 2r = x_re' and column
// 2r+1 = x_im' of excitation r gives Re and Im of Y in adjacent columns.  8 real flops per
// complex multiply-add, as the 4M method.
//
// float64 arithmetic above 8 columns instead takes three real products per complex one (3M,
// k_gemm3m_f64 below): 6 real flops per complex multiply-add.  The float32 path keeps the
// embedding (in float32 a 3M form would round the operand sums, which float64 holds exactly).
//
// Kernels: 256-thread workgroups of four waves; float32 MFMA 32x32x2 (wave tile 64 x 32 JN) or
// float64 MFMA 4x4x4 four-block (wave tile 32 x 16 JN), K step 16, double-buffered LDS (A stored
// k-major so that MFMA operand reads are conflict-free).  The N tile is the smallest of the
// path's tiles that holds the R columns, so a few excitations do not pay for a wide tile of
// zero columns, and the waves not needed along N go along M.  Where the row and
// column tiles give fewer than four waves of the workgroups the device holds at once (tall
// matrices with few columns), K is split S ways (split_waves): split s of every tile writes its
// partial product to a workspace and a second kernel sums the S partials in a fixed order
// (deterministic), applies alpha and accumulates into Y.  With S a power of two, split s runs on
// XCDs s mod 8 (workgroups are dealt round-robin), so the slice of the right-hand sides it reads
// stays in those XCDs' L2; with S = 1 the column tiles of one row tile are given to the same XCD
// and share its L2 copy of the A rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "linalg.h"
#include "prof.h"
#include "tune.h"

namespace bem {
namespace dev {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BK = 16, PADA = 4, PADB = 4;

__global__ void k_build_B(const double2* __restrict__ X, int64_t ldx, int64_t nc, int64_t R, float* __restrict__ Bm,
                          int64_t ldb, int64_t K16) {
  const int64_t col = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // 0 .. ldb-1
  if (col >= ldb) return;
  for (int64_t kp = blockIdx.y; kp < K16; kp += gridDim.y) {            // 0 .. K16-1
    float v = 0.f;
    const int64_t k = kp >> 1, r = col >> 1;
    if (k < nc && r < R) {
      const double2 x = X[r * ldx + k];
      const bool re_row = (kp & 1) == 0, re_col = (col & 1) == 0;
      if (re_col) v = re_row ? float(x.x) : float(-x.y);
      else v = re_row ? float(x.y) : float(x.x);
    }
    Bm[kp * ldb + col] = v;
  }
}

// Tile decode shared by both kernels: blockIdx.x -> (row tile, column tile, K split).  xcd = 1
// deals consecutive tiles to one XCD (workgroups go round-robin over the 8 XCDs), xcd = 0 keeps
// the launch order; either way every tile is computed the same.
struct TileIdx {
  int64_t tm, tn, ks;
};
__device__ __forceinline__ TileIdx tile_of(int64_t ntn, int64_t S, int xcd) {
  const int64_t nwg = int64_t(gridDim.x), p = blockIdx.x;
  TileIdx t;
  if (S > 1) {
    t.ks = p % S;
    const int64_t tile = p / S;
    t.tm = tile / ntn;
    t.tn = tile % ntn;
    return t;
  }
  int64_t logical = p;
  if (xcd && nwg % 8 == 0) logical = (p % 8) * (nwg / 8) + p / 8;
  t.tm = logical / ntn;
  t.tn = logical % ntn;
  t.ks = 0;
  return t;
}

// One output element of the real embedding: with S = 1 the even lane of a (Re, Im) column pair
// writes alpha (re + j im) (+ Y) to Y; with S > 1 every lane writes its real partial.
__device__ __forceinline__ void emit(double mine, double other, int lane, int64_t row, int64_t col, int64_t M,
                                     int64_t R, int64_t ldb, int64_t S, int64_t ks, double* __restrict__ P,
                                     double2* __restrict__ Y, int64_t ldy, double2 alpha, int accumulate) {
  if (row >= M) return;
  if (S > 1) {
    if (col < ldb) P[(size_t(ks) * M + row) * ldb + col] = mine;
    return;
  }
  if ((lane & 1) == 0 && (col >> 1) < R) {
    double yr = alpha.x * mine - alpha.y * other, yi = alpha.x * other + alpha.y * mine;
    double2* y = Y + (col >> 1) * ldy + row;
    if (accumulate) {
      yr += y->x;
      yi += y->y;
    }
    *y = make_double2(yr, yi);
  }
}

// Y[r][row] = alpha sum_s (P[s][row][2r] + j P[s][row][2r+1]) (+ Y), s in order.
__global__ void k_splitk_reduce(const double* __restrict__ P, int64_t M, int64_t ldb, int64_t S, int64_t R,
                                double2* __restrict__ Y, int64_t ldy, double2 alpha, int accumulate) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= M * R) return;
  const int64_t row = e / R, r = e % R;
  double re = 0.0, im = 0.0;
  for (int64_t s = 0; s < S; ++s) {
    const double* p = P + (size_t(s) * M + row) * ldb + 2 * r;
    re += p[0];
    im += p[1];
  }
  double yr = alpha.x * re - alpha.y * im, yi = alpha.x * im + alpha.y * re;
  double2* y = Y + r * ldy + row;
  if (accumulate) {
    yr += y->x;
    yi += y->y;
  }
  *y = make_double2(yr, yi);
}

// float32 storage: WN waves along N, JN 32-column MFMA blocks per wave, 2 x 32 rows per wave;
// tile (4 / WN) 64 x WN JN 32.  Split s covers K [s kc, (s + 1) kc).
template <bool ALIGNED, int WN, int JN>
__global__ void __launch_bounds__(256) k_gemm_f32(const float* __restrict__ A, int64_t lda, const float* __restrict__ Bm,
                                                  int64_t ldb, int64_t M, int64_t K, int64_t K16, int64_t kc,
                                                  int64_t ntn, int64_t S, double* __restrict__ P,
                                                  double2* __restrict__ Y, int64_t ldy, int64_t R, double2 alpha,
                                                  int accumulate, int xcd) {
  constexpr int WM = 4 / WN, TM = WM * 64, TN = WN * JN * 32;
  constexpr int EA = TM * BK / 256, EB = TN * BK / 256;  // A and B values per thread per K step
  __shared__ float As[2][BK][TM + PADA];
  __shared__ float Bs[2][BK][TN + PADB];
  const TileIdx ti = tile_of(ntn, S, xcd);
  const int64_t m0 = ti.tm * TM, n0 = ti.tn * TN;
  const int64_t kbeg = ti.ks * kc, kend = min(K16, kbeg + kc);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;

  const int a_row = tid / (BK / EA), a_k = (tid % (BK / EA)) * EA;
  const int b_k = tid >> 4, b_col = (tid & 15) * EB;
  const int64_t gm = m0 + a_row;

  floatx16 acc[2][JN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float ra[EA], rb[EB];
  auto load_tile = [&](int64_t k0) {
    const int64_t kk = k0 + a_k;
    if (gm < M) {
      const float* src = A + gm * lda + kk;
      if (ALIGNED && kk + EA <= K) {
#pragma unroll
        for (int e = 0; e < EA; e += 4) {
          const float4 u = *reinterpret_cast<const float4*>(src + e);
          ra[e] = u.x; ra[e + 1] = u.y; ra[e + 2] = u.z; ra[e + 3] = u.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < EA; ++e) ra[e] = (kk + e < K) ? src[e] : 0.f;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) ra[e] = 0.f;
    }
    const float* bsrc = Bm + (k0 + b_k) * ldb + n0 + b_col;
#pragma unroll
    for (int e = 0; e < EB; e += 2) {
      const float2 u = *reinterpret_cast<const float2*>(bsrc + e);
      rb[e] = u.x;
      rb[e + 1] = u.y;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_k + e][a_row] = ra[e];
#pragma unroll
    for (int e = 0; e < EB; ++e) Bs[buf][b_k][b_col + e] = rb[e];
  };

  const int64_t nk = (kend - kbeg) / BK;
  if (nk > 0) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = int(kt & 1);
    if (kt + 1 < nk) load_tile(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int kr = 2 * s + (lane >> 5);
      float af[2], bf[JN];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[buf][kr][wm * 64 + i * 32 + (lane & 31)];
#pragma unroll
      for (int j = 0; j < JN; ++j) bf[j] = Bs[buf][kr][wn * JN * 32 + j * 32 + (lane & 31)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

  // item v of lane l: row (v / 4) 8 + (l / 32) 4 + v % 4, column l % 32 of the 32 x 32 block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const double mine = acc[i][j][v];
        const double other = __shfl_xor(mine, 1, 64);
        const int64_t row = m0 + wm * 64 + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int64_t col = n0 + wn * JN * 32 + j * 32 + (lane & 31);
        emit(mine, other, lane, row, col, M, R, ldb, S, ti.ks, P, Y, ldy, alpha, accumulate);
      }
}

// ---- float64: the same real embedding on the float64 4x4x4 four-block matrix instruction.
constexpr int DK = 16, DPAD = 2;

__global__ void k_build_B64(const double2* __restrict__ X, int64_t ldx, int64_t nc, int64_t R,
                            double* __restrict__ Bm, int64_t ldb, int64_t K16) {
  const int64_t col = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= ldb) return;
  for (int64_t kp = blockIdx.y; kp < K16; kp += gridDim.y) {
    double v = 0.0;
    const int64_t k = kp >> 1, r = col >> 1;
    if (k < nc && r < R) {
      const double2 x = X[r * ldx + k];
      const bool re_row = (kp & 1) == 0, re_col = (col & 1) == 0;
      if (re_col) v = re_row ? x.x : -x.y;
      else v = re_row ? x.y : x.x;
    }
    Bm[kp * ldb + col] = v;
  }
}

// Lane l of an instruction supplies A_q[l % 4][l / 16] and B_q[l / 16][l % 4] of block
// q = (l % 16) / 4; all four blocks share the rows, so per 4 k a wave issues 8 x JN instructions
// for its 32 x 16 JN tile, and the result of instruction (i, j) on lane l is row 4 i + l / 16,
// column 16 j + l % 16 (even columns real, odd imaginary parts).  WN waves along N: tile
// (4 / WN) 32 x WN JN 16.
// TA = float: float32 entries widened as they are staged (float64 arithmetic on a float32-only
// operator, for the refinement's residuals).
template <typename TA, bool ALIGNED, int WN, int JN>
__global__ void __launch_bounds__(256) k_gemm_f64(const TA* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ Bm, int64_t ldb, int64_t M, int64_t K,
                                                  int64_t K16, int64_t kc, int64_t ntn, int64_t S,
                                                  double* __restrict__ P, double2* __restrict__ Y, int64_t ldy,
                                                  int64_t R, double2 alpha, int accumulate, int xcd) {
  constexpr int WM = 4 / WN, TM = WM * 32, TN = WN * JN * 16;
  constexpr int EA = TM * DK / 256, EB = TN * DK / 256;
  __shared__ double As[2][DK][TM + DPAD];
  __shared__ double Bs[2][DK][TN + DPAD];
  const TileIdx ti = tile_of(ntn, S, xcd);
  const int64_t m0 = ti.tm * TM, n0 = ti.tn * TN;
  const int64_t kbeg = ti.ks * kc, kend = min(K16, kbeg + kc);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;

  const int a_row = tid / (DK / EA), a_k = (tid % (DK / EA)) * EA;
  const int b_k = tid >> 4, b_col = (tid & 15) * EB;
  const int64_t gm = m0 + a_row;

  double acc4[8][JN];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) acc4[i][j] = 0.0;

  double ra[EA], rb[EB];
  auto load_tile = [&](int64_t k0) {
    const int64_t kk = k0 + a_k;
    if (gm < M) {
      const TA* src = A + gm * lda + kk;
      if (ALIGNED && kk + EA <= K) {
#pragma unroll
        for (int e = 0; e < EA; e += 2) {
          if constexpr (sizeof(TA) == 8) {
            const double2 u = *reinterpret_cast<const double2*>(src + e);
            ra[e] = u.x;
            ra[e + 1] = u.y;
          } else {
            const float2 u = *reinterpret_cast<const float2*>(src + e);
            ra[e] = double(u.x);
            ra[e + 1] = double(u.y);
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < EA; ++e) ra[e] = (kk + e < K) ? double(src[e]) : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) ra[e] = 0.0;
    }
    const double* bsrc = Bm + (k0 + b_k) * ldb + n0 + b_col;
    if constexpr (EB % 2 == 0) {
#pragma unroll
      for (int e = 0; e < EB; e += 2) {
        const double2 u = *reinterpret_cast<const double2*>(bsrc + e);
        rb[e] = u.x;
        rb[e + 1] = u.y;
      }
    } else {
      // odd counts (16- and 48-column tiles) start at odd columns: single loads
#pragma unroll
      for (int e = 0; e < EB; ++e) rb[e] = bsrc[e];
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_k + e][a_row] = ra[e];
#pragma unroll
    for (int e = 0; e < EB; ++e) Bs[buf][b_k][b_col + e] = rb[e];
  };

  const int64_t nk = (kend - kbeg) / DK;
  if (nk > 0) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = int(kt & 1);
    if (kt + 1 < nk) load_tile(kbeg + (kt + 1) * DK);
#pragma unroll
    for (int s = 0; s < DK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double av[8], bv[JN];
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = As[buf][kr][wm * 32 + 4 * i + (lane & 3)];
#pragma unroll
      for (int j = 0; j < JN; ++j) bv[j] = Bs[buf][kr][wn * JN * 16 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) acc4[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc4[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const double mine = acc4[i][j];
      const double other = __shfl_xor(mine, 1, 64);
      const int64_t row = m0 + wm * 32 + 4 * i + (lane >> 4);
      const int64_t col = n0 + wn * JN * 16 + j * 16 + (lane & 15);
      emit(mine, other, lane, row, col, M, R, ldb, S, ti.ks, P, Y, ldy, alpha, accumulate);
    }
}

// ---- float64, three real products per complex product (3M, Gauss's trick): for a = ar + j ai
// and x = xr + j xi,
//   P1 = ar xr,  P2 = ai xi,  P3 = (ar + ai)(xr + xi);   Re(a x) = P1 - P2,  Im(a x) = P3 - P1 - P2,
// summed over k as three real products on the 4x4x4 four-block instruction: 6 real flops per
// complex multiply-add instead of the embedding's 8.  The operands stay complex: A tiles and the
// right-hand sides are staged as (re, im) pairs straight from their complex storage (no
// embedded copy of X), and the sums ar + ai, xr + xi are formed as the operands are read.
// Lane l of an instruction supplies A_q[l % 4][l / 16] and B_q[l / 16][l % 4] of block
// q = (l % 16) / 4 and receives D_q[l / 16][l % 4].  Two operand layouts:
//   BSH = false: the four blocks share 4 rows and take 16 consecutive columns; a wave holds NI
//     row groups of 4 and NJ column groups of 16 (result: row 4 i + l / 16, column 16 j + l % 16);
//   BSH = true: the four blocks share 4 columns and take 16 consecutive rows; NI row groups of 16
//     and NJ column groups of 4 (result: row 16 i + 4 ((l % 16) / 4) + l / 16, column 4 j + l % 4),
//     for column tiles in steps of 4.
// Each lane holds P1, P2 and P3 of whole complex outputs, so every lane completes its own.  WN
// waves along N.  Split s covers complex K [s kc, (s + 1) kc); partials are written as (Re, Im)
// pairs in the embedding's layout, so the split-K sum is shared.
constexpr int CK = 8, CPAD = 1;  // complex k per K step; LDS row padding (complex entries)

template <typename TA, bool ALIGNED, int WN, int NI, int NJ, bool BSH>
__global__ void __launch_bounds__(256, 2) k_gemm3m_f64(const TA* __restrict__ A, int64_t lda,
                                                       const double2* __restrict__ X, int64_t ldx, int64_t M,
                                                       int64_t K, int64_t kc, int64_t ntn, int64_t S,
                                                       double* __restrict__ P, int64_t ldb, double2* __restrict__ Y,
                                                       int64_t ldy, int64_t R, double2 alpha, int accumulate,
                                                       int xcd) {
  constexpr int RS = BSH ? 16 : 4, CS = BSH ? 4 : 16;  // row / column group sizes of an instruction
  constexpr int WTM = NI * RS, WTN = NJ * CS;           // wave tile (rows, complex columns)
  constexpr int WM = 4 / WN, TM = WM * WTM, TN = WN * WTN;
  constexpr int EA = TM * CK / 256;                      // complex A entries per thread
  constexpr int NB = (TN * CK + 255) / 256;              // complex X entries per thread
  static_assert(EA >= 1 && CK % EA == 0, "row tile");
  __shared__ double2 As[2][CK][TM + CPAD];
  __shared__ double2 Bs[2][CK][TN + CPAD];
  const TileIdx ti = tile_of(ntn, S, xcd);
  const int64_t m0 = ti.tm * TM, n0 = ti.tn * TN;
  const int64_t kbeg = ti.ks * kc, kend = min(K, kbeg + kc);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;
  const int a_lane = BSH ? (lane & 15) : (lane & 3), b_lane = BSH ? (lane & 3) : (lane & 15);

  const int a_row = tid / (CK / EA), a_k = (tid % (CK / EA)) * EA;
  const int64_t gm = m0 + a_row;

  double p1[NI][NJ], p2[NI][NJ], p3[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) p1[i][j] = p2[i][j] = p3[i][j] = 0.0;

  double2 ra[EA], rb[NB];
  auto load_tile = [&](int64_t k0) {
    const int64_t kk = k0 + a_k;
    if (gm < M) {
      const TA* src = A + (gm * lda + kk) * 2;
      if (ALIGNED && kk + EA <= K) {
        if constexpr (sizeof(TA) == 8) {
#pragma unroll
          for (int e = 0; e < EA; ++e) ra[e] = *reinterpret_cast<const double2*>(src + 2 * e);
        } else if constexpr (EA % 2 == 0) {
#pragma unroll
          for (int e = 0; e < EA; e += 2) {
            const float4 u = *reinterpret_cast<const float4*>(src + 2 * e);
            ra[e] = make_double2(double(u.x), double(u.y));
            ra[e + 1] = make_double2(double(u.z), double(u.w));
          }
        } else {
#pragma unroll
          for (int e = 0; e < EA; ++e) {
            const float2 u = *reinterpret_cast<const float2*>(src + 2 * e);
            ra[e] = make_double2(double(u.x), double(u.y));
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < EA; ++e)
          ra[e] = (kk + e < K) ? make_double2(double(src[2 * e]), double(src[2 * e + 1])) : make_double2(0.0, 0.0);
      }
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) ra[e] = make_double2(0.0, 0.0);
    }
    // X entries: consecutive threads take consecutive k of one column (coalesced along k)
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int v = tid + 256 * e, bk = v % CK, bc = v / CK;
      const int64_t k = k0 + bk, c = n0 + bc;
      rb[e] = (v < TN * CK && k < K && c < R) ? X[c * ldx + k] : make_double2(0.0, 0.0);
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_k + e][a_row] = ra[e];
#pragma unroll
    for (int e = 0; e < NB; ++e) {
      const int v = tid + 256 * e;
      if (v < TN * CK) Bs[buf][v % CK][v / CK] = rb[e];
    }
  };

  const int64_t nk = (kend - kbeg + CK - 1) / CK;
  if (nk > 0) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = int(kt & 1);
    if (kt + 1 < nk) load_tile(kbeg + (kt + 1) * CK);
#pragma unroll
    for (int s = 0; s < CK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double ar[NI], ai[NI], br[NJ], bi[NJ];
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        const double2 u = As[buf][kr][wm * WTM + RS * i + a_lane];
        ar[i] = u.x;
        ai[i] = u.y;
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const double2 u = Bs[buf][kr][wn * WTN + CS * j + b_lane];
        br[j] = u.x;
        bi[j] = u.y;
      }
#pragma unroll
      for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[i], br[j], p1[i][j], 0, 0, 0);
          p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(ai[i], bi[j], p2[i][j], 0, 0, 0);
          p3[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[i] + ai[i], br[j] + bi[j], p3[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

  const int o_row = BSH ? 4 * ((lane & 15) >> 2) + (lane >> 4) : (lane >> 4);
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int64_t row = m0 + wm * WTM + RS * i + o_row;
      const int64_t col = n0 + wn * WTN + CS * j + b_lane;
      if (row >= M) continue;
      const double re = p1[i][j] - p2[i][j], im = (p3[i][j] - p1[i][j]) - p2[i][j];
      if (S > 1) {
        *reinterpret_cast<double2*>(P + (size_t(ti.ks) * M + row) * ldb + 2 * col) = make_double2(re, im);
      } else if (col < R) {
        double yr = alpha.x * re - alpha.y * im, yi = alpha.x * im + alpha.y * re;
        double2* y = Y + col * ldy + row;
        if (accumulate) {
          yr += y->x;
          yi += y->y;
        }
        *y = make_double2(yr, yi);
      }
    }
}

}  // namespace dev

namespace {
// Work decomposition of one product.  The embedding's N tile (real columns) is the smallest one
// of the path that holds the 2R columns (float32: 32, 64, 96, 128; float64, 3-8 columns: 16).
// Each N tile has one or more variants (waves along N x MFMA blocks per wave, so different row
// tiles; for 3M also the operand layout); the first is canonical and its row tile alone sets
// the K split, so all variants sum the same partial products in the same order and agree
// bitwise.
constexpr int64_t kTargetWorkgroups = 2048;
constexpr int64_t kMaxSplit = 16;
int ntile_f64(int64_t nrhs) {
  (void)nrhs;  // 3-8 columns (more take the 3M path)
  return 16;
}
int ntile_f32(int64_t nrhs) {
  const int64_t c = 2 * nrhs;
  for (int t : {32, 64, 96})
    if (c <= t) return t;
  return 128;
}
int64_t ldb_of(int64_t nrhs, int tn) { return (2 * nrhs + tn - 1) / tn * tn; }
// the larger leading dimension of the two paths (workspace sizing)
int64_t ldb_for(int64_t nrhs) { return ldb_of(nrhs, ntile_f32(nrhs)); }
struct Var {
  int wn, jn;
};
// variants per N tile, canonical first
std::vector<Var> vars_f64(int tn) {
  (void)tn;
  return {{1, 1}};
}
std::vector<Var> vars_f32(int tn) {
  switch (tn) {
    case 32: return {{1, 1}};
    case 64: return {{1, 2}, {2, 1}};
    case 96: return {{1, 3}};
    default: return {{2, 2}, {1, 4}};
  }
}

// 3M path (float64 arithmetic, 9 columns and more): complex column tiles in steps of 4 up to 32
// columns and of 8 up to 64 (at most 3 or 7 padding columns).  Up to 8 columns the embedding's
// 16-real-column tile pads less (and those products are bound by the matrix read).
constexpr int kMin3M = 9;
int ntile_3m(int64_t nrhs) {
  for (int t : {12, 16, 20, 24, 28, 32, 40, 48, 56})
    if (nrhs <= t) return t;
  // above 56 columns: the tile of 64, 48 or 32 that pads least (ties to the wider)
  int best = 64;
  for (int t : {48, 32})
    if ((nrhs + t - 1) / t * t < (nrhs + best - 1) / best * best) best = t;
  return best;
}
struct Var3 {
  int wn, ni, nj;
  bool bsh;
};
// variants per tile, canonical first (its row tile sets the K split)
std::vector<Var3> vars_3m(int tn) {
  switch (tn) {
    case 12: return {{1, 2, 3, true}, {1, 4, 3, true}};
    case 16: return {{1, 8, 1, false}, {1, 2, 4, true}};
    case 20: return {{1, 2, 5, true}, {1, 4, 5, true}};
    case 24: return {{1, 2, 6, true}, {2, 4, 3, true}};
    case 28: return {{1, 2, 7, true}};
    case 32: return {{1, 8, 2, false}, {2, 8, 1, false}, {1, 2, 8, true}};
    case 40: return {{1, 2, 10, true}, {2, 2, 5, true}};
    case 48: return {{1, 8, 3, false}, {2, 4, 6, true}};
    case 56: return {{2, 2, 7, true}};
    default: return {{2, 8, 2, false}, {4, 8, 1, false}, {2, 2, 8, true}, {4, 4, 4, true}};
  }
}
int64_t tm_3m(const Var3& v) { return (4 / v.wn) * v.ni * (v.bsh ? 16 : 4); }

struct GemmLaunch {
  dim3 g;
  int64_t lda, ldb, K, K16, kc, ntn, S;
  double* P;
  int xcd;
};

// The embedding's float64 kernel serves 3-8 columns only (one 16-real-column tile, one variant).
template <typename TA, bool AL>
void launch_f64_variant(const GemmLaunch& l, const GemmDesc& d, const double* Bm, hipStream_t st) {
  const TA* A = static_cast<const TA*>(d.A);
  hipLaunchKernelGGL((dev::k_gemm_f64<TA, AL, 1, 1>), l.g, dim3(256), 0, st, A, l.lda, Bm, l.ldb, d.rows, l.K, l.K16,
                     l.kc, l.ntn, l.S, l.P, d.Y, d.ldy, d.nrhs, d.alpha, d.accumulate, l.xcd);
}

constexpr int code3m(int wn, int ni, int nj, bool bsh) { return ((wn * 16 + ni) * 32 + nj) * 2 + (bsh ? 1 : 0); }

template <typename TA, bool AL>
void launch_3m_variant(const Var3& v, const GemmLaunch& l, const GemmDesc& d, hipStream_t st) {
  const TA* A = static_cast<const TA*>(d.A);
#define BEM_G3M(WN, NI, NJ, BS)                                                                                \
  hipLaunchKernelGGL((dev::k_gemm3m_f64<TA, AL, WN, NI, NJ, BS>), l.g, dim3(256), 0, st, A, d.lda, d.X, d.ldx, \
                     d.rows, d.cols, l.kc, l.ntn, l.S, l.P, l.ldb, d.Y, d.ldy, d.nrhs, d.alpha, d.accumulate, l.xcd)
  const int code = code3m(v.wn, v.ni, v.nj, v.bsh);
  if constexpr (AL) {
    switch (code) {
      case code3m(1, 2, 3, true): BEM_G3M(1, 2, 3, true); break;
      case code3m(1, 4, 3, true): BEM_G3M(1, 4, 3, true); break;
      case code3m(1, 8, 1, false): BEM_G3M(1, 8, 1, false); break;
      case code3m(1, 2, 4, true): BEM_G3M(1, 2, 4, true); break;
      case code3m(1, 2, 5, true): BEM_G3M(1, 2, 5, true); break;
      case code3m(1, 4, 5, true): BEM_G3M(1, 4, 5, true); break;
      case code3m(1, 2, 6, true): BEM_G3M(1, 2, 6, true); break;
      case code3m(2, 4, 3, true): BEM_G3M(2, 4, 3, true); break;
      case code3m(1, 2, 7, true): BEM_G3M(1, 2, 7, true); break;
      case code3m(1, 8, 2, false): BEM_G3M(1, 8, 2, false); break;
      case code3m(2, 8, 1, false): BEM_G3M(2, 8, 1, false); break;
      case code3m(1, 2, 8, true): BEM_G3M(1, 2, 8, true); break;
      case code3m(1, 2, 10, true): BEM_G3M(1, 2, 10, true); break;
      case code3m(2, 2, 5, true): BEM_G3M(2, 2, 5, true); break;
      case code3m(1, 8, 3, false): BEM_G3M(1, 8, 3, false); break;
      case code3m(2, 4, 6, true): BEM_G3M(2, 4, 6, true); break;
      case code3m(2, 2, 7, true): BEM_G3M(2, 2, 7, true); break;
      case code3m(2, 8, 2, false): BEM_G3M(2, 8, 2, false); break;
      case code3m(4, 8, 1, false): BEM_G3M(4, 8, 1, false); break;
      case code3m(2, 2, 8, true): BEM_G3M(2, 2, 8, true); break;
      case code3m(4, 4, 4, true): BEM_G3M(4, 4, 4, true); break;
      default: throw Error(BEM_E_INVALID, "no such 3M GEMM variant");
    }
  } else {
    switch (code) {  // unaligned operands: canonical variants only
      case code3m(1, 2, 3, true): BEM_G3M(1, 2, 3, true); break;
      case code3m(1, 8, 1, false): BEM_G3M(1, 8, 1, false); break;
      case code3m(1, 2, 5, true): BEM_G3M(1, 2, 5, true); break;
      case code3m(1, 2, 6, true): BEM_G3M(1, 2, 6, true); break;
      case code3m(1, 2, 7, true): BEM_G3M(1, 2, 7, true); break;
      case code3m(1, 8, 2, false): BEM_G3M(1, 8, 2, false); break;
      case code3m(1, 2, 10, true): BEM_G3M(1, 2, 10, true); break;
      case code3m(1, 8, 3, false): BEM_G3M(1, 8, 3, false); break;
      case code3m(2, 2, 7, true): BEM_G3M(2, 2, 7, true); break;
      case code3m(2, 8, 2, false): BEM_G3M(2, 8, 2, false); break;
      default: throw Error(BEM_E_INVALID, "no such 3M GEMM variant");
    }
  }
#undef BEM_G3M
}

// Workgroups of the canonical variant of tile tn that fit on the device at once (compute units
// x workgroups per unit), queried once per device, entry type, alignment and tile.
template <typename TA, bool AL>
const void* canonical_3m(int tn) {
  switch (tn) {
    case 12: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 2, 3, true>);
    case 16: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 8, 1, false>);
    case 20: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 2, 5, true>);
    case 24: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 2, 6, true>);
    case 28: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 2, 7, true>);
    case 32: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 8, 2, false>);
    case 40: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 2, 10, true>);
    case 48: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 1, 8, 3, false>);
    case 56: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 2, 2, 7, true>);
    default: return reinterpret_cast<const void*>(&dev::k_gemm3m_f64<TA, AL, 2, 8, 2, false>);
  }
}
// Workgroups of 256 threads of kernel fn that fit on the current device at once.
int64_t resident_of(const void* fn) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int64_t> cache;
  int dev = 0;
  BEM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({dev, fn});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  BEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0));
  BEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t r = std::max<int64_t>(1, int64_t(per_cu) * cus);
  cache[{dev, fn}] = r;
  return r;
}
int64_t resident_3m(int tn, bool f32e, bool aligned) {
  return resident_of(f32e ? (aligned ? canonical_3m<float, true>(tn) : canonical_3m<float, false>(tn))
                          : (aligned ? canonical_3m<double, true>(tn) : canonical_3m<double, false>(tn)));
}
// K split of a product.  The workgroups run in waves of `resident`; a last wave that is
// nearly empty leaves most of the device idle for a whole workgroup's time.  The smallest split
// that gives at least four waves is taken (its last wave is then at most a fifth of the time);
// where no split reaches four waves, the split whose last wave is fullest (ties to the larger
// split).  Where the right-hand sides exceed 8 MiB only powers of two are taken: workgroups go
// round-robin over the 8 XCDs, so split s then stays on XCDs s mod 8 and each XCD's L2 holds
// only its splits' slices (other splits scatter every slice over every XCD).  S <= 16 and at
// most `top` (at least 64 complex K per split, the partials within the workspace).  It depends
// only on the shape and the device, so results stay bitwise reproducible.
int64_t split_waves(int64_t tiles, int64_t top, double rhs_bytes, int64_t resident) {
  top = std::max<int64_t>(1, std::min(top, kMaxSplit));
  const bool pow2 = rhs_bytes > double(8 << 20);
  auto allowed = [&](int64_t S) { return !pow2 || (S & (S - 1)) == 0; };
  for (int64_t S = 1; S <= top; ++S)
    if (allowed(S) && tiles * S >= 4 * resident) return S;
  int64_t best = 1;
  double best_f = 0;
  for (int64_t S = 1; S <= top; ++S) {
    if (!allowed(S)) continue;
    const int64_t W = tiles * S, waves = (W + resident - 1) / resident;
    const double f = double(W) / double(waves * resident);
    if (f >= best_f - 1e-9) {
      best = S;
      best_f = f;
    }
  }
  return best;
}

// Canonical variant of an embedding tile: float32 MFMA (tn real columns) or, up to 8 columns,
// the float64 kernel's 16-column tile.
const void* canonical_4m(int tn, bool mfma32, bool f32e, bool aligned) {
  if (mfma32) {
    switch (tn) {
      case 32: return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f32<true, 1, 1>)
                              : reinterpret_cast<const void*>(&dev::k_gemm_f32<false, 1, 1>);
      case 64: return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f32<true, 1, 2>)
                              : reinterpret_cast<const void*>(&dev::k_gemm_f32<false, 1, 2>);
      case 96: return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f32<true, 1, 3>)
                              : reinterpret_cast<const void*>(&dev::k_gemm_f32<false, 1, 3>);
      default: return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f32<true, 2, 2>)
                              : reinterpret_cast<const void*>(&dev::k_gemm_f32<false, 2, 2>);
    }
  }
  if (f32e)
    return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f64<float, true, 1, 1>)
                   : reinterpret_cast<const void*>(&dev::k_gemm_f64<float, false, 1, 1>);
  return aligned ? reinterpret_cast<const void*>(&dev::k_gemm_f64<double, true, 1, 1>)
                 : reinterpret_cast<const void*>(&dev::k_gemm_f64<double, false, 1, 1>);
}

// The float64-arithmetic product on the 3M kernel (d.fp32 = 0: float64 entries, 2: float32).
void launch_gemm3m(const GemmDesc& d, void* ws, size_t ws_bytes, hipStream_t st) {
  const int tn = ntile_3m(d.nrhs);
  const bool f32e = d.fp32 != 0;
  GemmLaunch l;
  l.ldb = 2 * ((d.nrhs + tn - 1) / tn * tn);  // real leading dimension of the partials
  l.ntn = l.ldb / (2 * tn);
  l.K = d.cols;
  l.K16 = (2 * d.cols + dev::BK - 1) / dev::BK * dev::BK;
  l.lda = d.lda;
  const uintptr_t ab = reinterpret_cast<uintptr_t>(d.A);
  const bool aligned = f32e ? ((ab & 15) == 0 && (d.lda & 1) == 0) : (ab & 15) == 0;
  std::vector<Var3> vars = vars_3m(tn);
  if (!aligned) vars.resize(1);
  const int64_t ntm0 = (d.rows + tm_3m(vars[0]) - 1) / tm_3m(vars[0]);
  const int64_t smax = std::max<int64_t>(1, int64_t(ws_bytes / (sizeof(double) * size_t(d.rows) * l.ldb)));
  l.S = split_waves(ntm0 * l.ntn, std::min<int64_t>(smax, d.cols / 64), 16.0 * double(d.cols) * double(d.nrhs),
                    resident_3m(tn, f32e, aligned));
  l.kc = ((d.cols + l.S - 1) / l.S + dev::CK - 1) / dev::CK * dev::CK;
  const size_t need = l.S > 1 ? size_t(l.S) * d.rows * l.ldb * sizeof(double) : 0;
  if (need > ws_bytes) throw Error(BEM_E_INVALID, "GEMM workspace too small");
  l.P = static_cast<double*>(ws);
  const int nx = l.S == 1 ? 2 : 1;
  const int ncand = int(vars.size()) * nx;
  const uint64_t key = tune_key(f32e ? 5 : 4, {tn, l.S, aligned ? 1 : 0, log2_bucket(d.rows), log2_bucket(l.K16)});
  ProfScope ps(st, KC_GEMM_F64, double(d.rows) * d.cols * (f32e ? 8.0 : 16.0), 8.0 * double(d.rows) * d.cols * d.nrhs);
  {
    TuneScope ts(key, ncand, st);
    const int cand = ts.variant();
    const Var3& v = vars[cand / nx];
    l.xcd = (cand % nx) == 0 ? 1 : 0;
    l.g = dim3(unsigned(((d.rows + tm_3m(v) - 1) / tm_3m(v)) * l.ntn * l.S));
    if (f32e) {
      if (aligned) launch_3m_variant<float, true>(v, l, d, st);
      else launch_3m_variant<float, false>(v, l, d, st);
    } else {
      if (aligned) launch_3m_variant<double, true>(v, l, d, st);
      else launch_3m_variant<double, false>(v, l, d, st);
    }
    BEM_HIP(hipGetLastError());
  }
  if (l.S > 1) {
    const int64_t n = d.rows * d.nrhs;
    hipLaunchKernelGGL(dev::k_splitk_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, l.P, d.rows, l.ldb,
                       l.S, d.nrhs, d.Y, d.ldy, d.alpha, d.accumulate);
    BEM_HIP(hipGetLastError());
  }
}

template <bool AL>
void launch_f32_variant(const Var& v, const GemmLaunch& l, const GemmDesc& d, const float* Bm, hipStream_t st) {
  const float* A = static_cast<const float*>(d.A);
#define BEM_G32(WN, JN)                                                                                        \
  hipLaunchKernelGGL((dev::k_gemm_f32<AL, WN, JN>), l.g, dim3(256), 0, st, A, l.lda, Bm, l.ldb, d.rows, l.K, \
                     l.K16, l.kc, l.ntn, l.S, l.P, d.Y, d.ldy, d.nrhs, d.alpha, d.accumulate, l.xcd)
  const int code = v.wn * 10 + v.jn;
  if constexpr (AL) {
    switch (code) {
      case 11: BEM_G32(1, 1); break;
      case 12: BEM_G32(1, 2); break;
      case 21: BEM_G32(2, 1); break;
      case 13: BEM_G32(1, 3); break;
      case 22: BEM_G32(2, 2); break;
      case 14: BEM_G32(1, 4); break;
      default: throw Error(BEM_E_INVALID, "no such float32 GEMM variant");
    }
  } else {
    switch (code) {
      case 11: BEM_G32(1, 1); break;
      case 12: BEM_G32(1, 2); break;
      case 13: BEM_G32(1, 3); break;
      case 22: BEM_G32(2, 2); break;
      default: throw Error(BEM_E_INVALID, "no such float32 GEMM variant");
    }
  }
#undef BEM_G32
}
}  // namespace

size_t gemm_workspace_bytes(int64_t n, int64_t nrhs) {
  // the float64 embedding of the right-hand sides (K16 x ldb doubles, the larger of the two),
  // then the split-K partials: S M ldb doubles for blocks of up to n rows (the split is capped
  // by the space given here)
  const int64_t K16 = (2 * n + dev::BK - 1) / dev::BK * dev::BK;
  const int64_t ldb = ldb_for(nrhs);
  const int64_t partial = std::min<int64_t>(kMaxSplit * n * ldb, 2 * kTargetWorkgroups * 256 * 128 + n * ldb);
  return (size_t(K16) * ldb + size_t(partial)) * sizeof(double) + 256;
}

void launch_gemm(const GemmDesc& d, void* ws, size_t ws_bytes, hipStream_t st) {
  if (d.rows <= 0 || d.nrhs <= 0) return;
  // fp32 == 2: float32 entries on the float64 kernel (float64 arithmetic)
  const bool mfma32 = d.fp32 == 1;
  if (!mfma32 && d.nrhs >= kMin3M) {
    launch_gemm3m(d, ws, ws_bytes, st);
    return;
  }
  const int tn = mfma32 ? ntile_f32(d.nrhs) : ntile_f64(d.nrhs);
  GemmLaunch l;
  l.K = 2 * d.cols;
  l.K16 = (l.K + dev::BK - 1) / dev::BK * dev::BK;
  l.ldb = ldb_of(d.nrhs, tn);
  l.ntn = l.ldb / tn;
  l.lda = 2 * d.lda;  // real leading dimension
  const size_t esz = mfma32 ? sizeof(float) : (d.fp32 ? sizeof(float) : sizeof(double));
  const bool aligned = mfma32 ? ((reinterpret_cast<uintptr_t>(d.A) | uintptr_t(l.lda * 4)) & 15) == 0
                              : ((reinterpret_cast<uintptr_t>(d.A) | uintptr_t(l.lda * esz)) & (2 * esz - 1)) == 0;
  std::vector<Var> vars = mfma32 ? vars_f32(tn) : vars_f64(tn);
  if (!aligned) vars.resize(1);
  auto tm_of = [&](const Var& v) -> int64_t { return (4 / v.wn) * (mfma32 ? 64 : 32); };
  const int64_t ntm0 = (d.rows + tm_of(vars[0]) - 1) / tm_of(vars[0]);
  const size_t bbytes = size_t(l.K16) * l.ldb * (mfma32 ? sizeof(float) : sizeof(double));
  const size_t poff = (bbytes + 255) / 256 * 256;
  {
    const void* fn = canonical_4m(tn, mfma32, d.fp32 != 0, aligned);
    const int64_t smax =
        ws_bytes > poff ? int64_t((ws_bytes - poff) / (sizeof(double) * size_t(d.rows) * size_t(l.ldb))) : 1;
    l.S = split_waves(ntm0 * l.ntn, std::min<int64_t>(smax, l.K16 / 128), double(bbytes), resident_of(fn));
  }
  l.kc = ((l.K16 + l.S - 1) / l.S + dev::BK - 1) / dev::BK * dev::BK;
  const size_t need = poff + (l.S > 1 ? size_t(l.S) * d.rows * l.ldb * sizeof(double) : 0);
  if (need > ws_bytes) throw Error(BEM_E_INVALID, "GEMM workspace too small");
  l.P = reinterpret_cast<double*>(static_cast<char*>(ws) + poff);
  // candidates: the variants, and with S = 1 the tile-to-XCD mapping on and off
  const int nx = l.S == 1 ? 2 : 1;
  const int ncand = int(vars.size()) * nx;
  const uint64_t key = tune_key(mfma32 ? 1 : (d.fp32 ? 2 : 3),
                                {tn, l.S, aligned ? 1 : 0, log2_bucket(d.rows), log2_bucket(l.K16)});
  // the split-K sum belongs to the product (inside its timing scope)
  auto reduce = [&]() {
    if (l.S <= 1) return;
    const int64_t n = d.rows * d.nrhs;
    hipLaunchKernelGGL(dev::k_splitk_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, l.P, d.rows, l.ldb,
                       l.S, d.nrhs, d.Y, d.ldy, d.alpha, d.accumulate);
    BEM_HIP(hipGetLastError());
  };
  auto shape = [&](int cand) {
    const Var& v = vars[cand / nx];
    l.xcd = (cand % nx) == 0 ? 1 : 0;
    const int64_t ntm = (d.rows + tm_of(v) - 1) / tm_of(v);
    l.g = dim3(unsigned(ntm * l.ntn * l.S));
    return v;
  };
  if (!mfma32) {
    double* Bm = static_cast<double*>(ws);
    hipLaunchKernelGGL(dev::k_build_B64, dim3(unsigned((l.ldb + 255) / 256), unsigned(std::min<int64_t>(l.K16, 32768))),
                       dim3(256), 0, st, d.X, d.ldx, d.cols, d.nrhs, Bm, l.ldb, l.K16);
    BEM_HIP(hipGetLastError());
    ProfScope ps(st, KC_GEMM_F64, double(d.rows) * d.cols * (d.fp32 ? 8.0 : 16.0),
                 8.0 * double(d.rows) * d.cols * d.nrhs);
    {
      TuneScope ts(key, ncand, st);
      const Var v = shape(ts.variant());
      (void)v;
      if (!d.fp32) {
        if (aligned) launch_f64_variant<double, true>(l, d, Bm, st);
        else launch_f64_variant<double, false>(l, d, Bm, st);
      } else {
        if (aligned) launch_f64_variant<float, true>(l, d, Bm, st);
        else launch_f64_variant<float, false>(l, d, Bm, st);
      }
      BEM_HIP(hipGetLastError());
    }
    reduce();
  } else {
    float* Bm = static_cast<float*>(ws);
    hipLaunchKernelGGL(dev::k_build_B, dim3(unsigned((l.ldb + 255) / 256), unsigned(std::min<int64_t>(l.K16, 32768))),
                       dim3(256), 0, st, d.X, d.ldx, d.cols, d.nrhs, Bm, l.ldb, l.K16);
    BEM_HIP(hipGetLastError());
    ProfScope ps(st, KC_GEMM_F32, double(d.rows) * d.cols * 8.0, 8.0 * double(d.rows) * d.cols * d.nrhs);
    {
      TuneScope ts(key, ncand, st);
      const Var v = shape(ts.variant());
      if (aligned) launch_f32_variant<true>(v, l, d, Bm, st);
      else launch_f32_variant<false>(v, l, d, Bm, st);
      BEM_HIP(hipGetLastError());
    }
    reduce();
  }
}

// Columns at or below this count run as repeated grouped GEMVs (the float32 tile of 64 real
// columns would be mostly padding); above it, one GEMM per descriptor.
constexpr int kGemmMinCols = 3;

void launch_products(const std::vector<GemvDesc>& ds, int R, void* ws, size_t ws_bytes, hipStream_t st) {
  if (ds.empty() || R <= 0) return;
  if (R == 1) {
    launch_gemv_grouped(ds.data(), int(ds.size()), st);
    return;
  }
  if (R < kGemmMinCols) {
    std::vector<GemvDesc> all;
    all.reserve(ds.size() * R);
    for (int r = 0; r < R; ++r)
      for (const GemvDesc& d : ds) {
        GemvDesc c = d;
        c.x = d.x + r * d.ldx;
        if (d.x2) c.x2 = d.x2 + r * d.ldx2;
        c.y = d.y + r * d.ldy;
        all.push_back(c);
      }
    launch_gemv_grouped(all.data(), int(all.size()), st);
    return;
  }
  for (const GemvDesc& d : ds) {
    GemmDesc g{d.A, d.lda, d.rows, d.cols, d.x, d.ldx, d.y, d.ldy, R, d.alpha, d.accumulate, d.fp32};
    launch_gemm(g, ws, ws_bytes, st);
    if (d.A2) {
      GemmDesc g2{d.A2, d.lda2, d.rows, d.cols, d.x2, d.ldx2, d.y, d.ldy, R, d.alpha2, 1, d.fp32};
      launch_gemm(g2, ws, ws_bytes, st);
    }
  }
}

}  // namespace bem
