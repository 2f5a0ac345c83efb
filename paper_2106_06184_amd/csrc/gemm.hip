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
// Kernel: 128 x 128 output tile per 256-thread workgroup (2 x 2 waves of 64 x 64), K step 16,
// double-buffered LDS (A stored k-major so that MFMA operand reads are conflict-free), float32
// MFMA 32x32x2 with float32 accumulation.  Workgroup ids are remapped so that the column tiles
// of one row tile run on the same XCD and share its L2 copy of the A rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "linalg.h"
#include "prof.h"

namespace bem {
namespace dev {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 16, PADA = 4, PADB = 4;

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

template <bool ALIGNED>
__global__ void __launch_bounds__(256) k_gemm_f32(const float* __restrict__ A, int64_t lda, const float* __restrict__ Bm,
                                                  int64_t ldb, int64_t M, int64_t K, int64_t K16, int64_t ntn,
                                                  double2* __restrict__ Y, int64_t ldy, int64_t R, double2 alpha,
                                                  int accumulate) {
  __shared__ float As[2][BK][BM + PADA];
  __shared__ float Bs[2][BK][BN + PADB];
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs; consecutive
  // logical tiles (the column tiles of one row tile) are given to the same XCD.
  const int64_t nwg = int64_t(gridDim.x);
  const int64_t p = blockIdx.x;
  int64_t logical = p;
  if (nwg % 8 == 0) logical = (p % 8) * (nwg / 8) + p / 8;
  const int64_t tm = logical / ntn, tn = logical % ntn;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;

  // global-load coordinates
  const int a_row = tid >> 1, a_k = (tid & 1) * 8;     // A: 128 rows x 16 k
  const int b_k = tid >> 4, b_col = (tid & 15) * 8;    // B: 16 k x 128 cols
  const int64_t gm = m0 + a_row;

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  float ra[8], rb[8];
  auto load_tile = [&](int64_t k0) {
    const int64_t kk = k0 + a_k;
    if (gm < M) {
      const float* src = A + gm * lda + kk;
      if (ALIGNED && kk + 8 <= K) {
        const float4 u = *reinterpret_cast<const float4*>(src);
        const float4 w = *reinterpret_cast<const float4*>(src + 4);
        ra[0] = u.x; ra[1] = u.y; ra[2] = u.z; ra[3] = u.w;
        ra[4] = w.x; ra[5] = w.y; ra[6] = w.z; ra[7] = w.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[e] = (kk + e < K) ? src[e] : 0.f;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = 0.f;
    }
    const float* bsrc = Bm + (k0 + b_k) * ldb + n0 + b_col;
    const float4 u = *reinterpret_cast<const float4*>(bsrc);
    const float4 w = *reinterpret_cast<const float4*>(bsrc + 4);
    rb[0] = u.x; rb[1] = u.y; rb[2] = u.z; rb[3] = u.w;
    rb[4] = w.x; rb[5] = w.y; rb[6] = w.z; rb[7] = w.w;
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[buf][a_k + e][a_row] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) Bs[buf][b_k][b_col + e] = rb[e];
  };

  const int64_t nk = K16 / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = int(kt & 1);
    if (kt + 1 < nk) load_tile((kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 2; ++s) {
      const int kr = 2 * s + (lane >> 5);
      float af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) af[i] = As[buf][kr][wm * 64 + i * 32 + (lane & 31)];
#pragma unroll
      for (int j = 0; j < 2; ++j) bf[j] = Bs[buf][kr][wn * 64 + j * 32 + (lane & 31)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      store_tile(buf ^ 1);
    }
    __syncthreads();
  }

  // epilogue: output column c = 2r (Re) or 2r+1 (Im); even lanes own the pair of an excitation
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float mine = acc[i][j][v];
        const float other = __shfl_xor(mine, 1, 64);
        const int64_t row = m0 + wm * 64 + i * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        const int64_t col = n0 + wn * 64 + j * 32 + (lane & 31);
        if ((lane & 1) == 0 && row < M && (col >> 1) < R) {
          const double re = mine, im = other;
          double yr = alpha.x * re - alpha.y * im, yi = alpha.x * im + alpha.y * re;
          double2* y = Y + (col >> 1) * ldy + row;
          if (accumulate) {
            yr += y->x;
            yi += y->y;
          }
          *y = make_double2(yr, yi);
        }
      }
}

// ---- float64: the same real embedding on the float64 4x4x4 four-block matrix instruction.  Tile
// 64 x 128 per 256-thread workgroup (2 x 2 waves of 32 x 64 reals), K step 16.
constexpr int DM = 64, DN = 128, DK = 16, DPAD = 2;

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
// q = (l % 16) / 4; all four blocks share the rows, so per 4 k a wave issues 8 x 4 instructions
// for its 32 x 64 tile, and the result of instruction (i, j) on lane l is row 4 i + l / 16,
// column 16 j + l % 16 (even columns real, odd imaginary parts).
template <bool ALIGNED>
__global__ void __launch_bounds__(256) k_gemm_f64(const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ Bm, int64_t ldb, int64_t M, int64_t K,
                                                  int64_t K16, int64_t ntn, double2* __restrict__ Y, int64_t ldy,
                                                  int64_t R, double2 alpha, int accumulate) {
  __shared__ double As[2][DK][DM + DPAD];
  __shared__ double Bs[2][DK][DN + DPAD];
  const int64_t nwg = int64_t(gridDim.x);
  const int64_t p = blockIdx.x;
  int64_t logical = p;
  if (nwg % 8 == 0) logical = (p % 8) * (nwg / 8) + p / 8;
  const int64_t tm = logical / ntn, tn = logical % ntn;
  const int64_t m0 = tm * DM, n0 = tn * DN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;

  const int a_row = tid >> 2, a_k = (tid & 3) * 4;   // A: 64 rows x 16 k, 4 per thread
  const int b_k = tid >> 4, b_col = (tid & 15) * 8;  // B: 16 k x 128 columns, 8 per thread
  const int64_t gm = m0 + a_row;

  double acc4[8][4];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc4[i][j] = 0.0;

  double ra[4], rb[8];
  auto load_tile = [&](int64_t k0) {
    const int64_t kk = k0 + a_k;
    if (gm < M) {
      const double* src = A + gm * lda + kk;
      if (ALIGNED && kk + 4 <= K) {
        const double2 u = *reinterpret_cast<const double2*>(src);
        const double2 w = *reinterpret_cast<const double2*>(src + 2);
        ra[0] = u.x; ra[1] = u.y; ra[2] = w.x; ra[3] = w.y;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[e] = (kk + e < K) ? src[e] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[e] = 0.0;
    }
    const double* bsrc = Bm + (k0 + b_k) * ldb + n0 + b_col;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const double2 u = *reinterpret_cast<const double2*>(bsrc + e);
      rb[e] = u.x;
      rb[e + 1] = u.y;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) As[buf][a_k + e][a_row] = ra[e];
#pragma unroll
    for (int e = 0; e < 8; ++e) Bs[buf][b_k][b_col + e] = rb[e];
  };

  const int64_t nk = K16 / DK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = int(kt & 1);
    if (kt + 1 < nk) load_tile((kt + 1) * DK);
#pragma unroll
    for (int s = 0; s < DK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      double av[8], bv[4];
#pragma unroll
      for (int i = 0; i < 8; ++i) av[i] = As[buf][kr][wm * 32 + 4 * i + (lane & 3)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[buf][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc4[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc4[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_tile(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double mine = acc4[i][j];
      const double other = __shfl_xor(mine, 1, 64);
      const int64_t row = m0 + wm * 32 + 4 * i + (lane >> 4);
      const int64_t col = n0 + wn * 64 + j * 16 + (lane & 15);
      if ((lane & 1) == 0 && row < M && (col >> 1) < R) {
        double yr = alpha.x * mine - alpha.y * other, yi = alpha.x * other + alpha.y * mine;
        double2* y = Y + (col >> 1) * ldy + row;
        if (accumulate) {
          yr += y->x;
          yi += y->y;
        }
        *y = make_double2(yr, yi);
      }
    }
}

}  // namespace dev

size_t gemm_workspace_bytes(int64_t cols, int64_t nrhs) {
  // float64 embedding (the larger of the two): K16 x ldb doubles
  const int64_t K16 = (2 * cols + dev::BK - 1) / dev::BK * dev::BK;
  const int64_t ldb = (2 * nrhs + dev::BN - 1) / dev::BN * dev::BN;
  return size_t(K16) * ldb * sizeof(double);
}

void launch_gemm(const GemmDesc& d, void* ws, size_t ws_bytes, hipStream_t st) {
  if (d.rows <= 0 || d.nrhs <= 0) return;
  const int64_t K = 2 * d.cols;
  const int64_t K16 = (K + dev::BK - 1) / dev::BK * dev::BK;
  const int64_t ldb = (2 * d.nrhs + dev::BN - 1) / dev::BN * dev::BN;
  const int64_t lda = 2 * d.lda;  // real leading dimension
  if (!d.fp32) {
    if (size_t(K16) * ldb * sizeof(double) > ws_bytes) throw Error(BEM_E_INVALID, "GEMM workspace too small");
    double* Bm = static_cast<double*>(ws);
    hipLaunchKernelGGL(dev::k_build_B64, dim3(unsigned((ldb + 255) / 256), unsigned(std::min<int64_t>(K16, 32768))), dim3(256), 0, st, d.X,
                       d.ldx, d.cols, d.nrhs, Bm, ldb, K16);
    BEM_HIP(hipGetLastError());
    const int64_t ntm = (d.rows + dev::DM - 1) / dev::DM, ntn = ldb / dev::DN;
    const double* A = static_cast<const double*>(d.A);
    const bool aligned = ((reinterpret_cast<uintptr_t>(A) | uintptr_t(lda * 8)) & 15) == 0;
    ProfScope ps(st, KC_GEMM_F64, double(d.rows) * d.cols * 16.0, 8.0 * double(d.rows) * d.cols * d.nrhs);
    const dim3 g(unsigned(ntm * ntn));
    if (aligned)
      hipLaunchKernelGGL((dev::k_gemm_f64<true>), g, dim3(256), 0, st, A, lda, Bm, ldb, d.rows, K, K16, ntn, d.Y,
                         d.ldy, d.nrhs, d.alpha, d.accumulate);
    else
      hipLaunchKernelGGL((dev::k_gemm_f64<false>), g, dim3(256), 0, st, A, lda, Bm, ldb, d.rows, K, K16, ntn, d.Y,
                         d.ldy, d.nrhs, d.alpha, d.accumulate);
    BEM_HIP(hipGetLastError());
    return;
  }
  if (size_t(K16) * ldb * sizeof(float) > ws_bytes) throw Error(BEM_E_INVALID, "GEMM workspace too small");
  float* Bm = static_cast<float*>(ws);
  hipLaunchKernelGGL(dev::k_build_B, dim3(unsigned((ldb + 255) / 256), unsigned(std::min<int64_t>(K16, 32768))), dim3(256), 0, st, d.X, d.ldx,
                     d.cols, d.nrhs, Bm, ldb, K16);
  BEM_HIP(hipGetLastError());
  const int64_t ntm = (d.rows + dev::BM - 1) / dev::BM, ntn = ldb / dev::BN;
  const float* A = static_cast<const float*>(d.A);
  const bool aligned = ((reinterpret_cast<uintptr_t>(A) | uintptr_t(lda * 4)) & 15) == 0;
  ProfScope ps(st, KC_GEMM_F32, double(d.rows) * d.cols * 8.0, 8.0 * double(d.rows) * d.cols * d.nrhs);
  if (aligned)
    hipLaunchKernelGGL(dev::k_gemm_f32<true>, dim3(unsigned(ntm * ntn)), dim3(256), 0, st, A, lda, Bm, ldb, d.rows, K,
                       K16, ntn, d.Y, d.ldy, d.nrhs, d.alpha, d.accumulate);
  else
    hipLaunchKernelGGL(dev::k_gemm_f32<false>, dim3(unsigned(ntm * ntn)), dim3(256), 0, st, A, lda, Bm, ldb, d.rows,
                       K, K16, ntn, d.Y, d.ldy, d.nrhs, d.alpha, d.accumulate);
  BEM_HIP(hipGetLastError());
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
