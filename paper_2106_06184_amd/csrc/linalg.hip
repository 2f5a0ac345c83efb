// Dense complex products, sparse glue and Krylov kernels (gfx950).
//
// The single-excitation products are HBM-bound (one complex MAC per matrix element read):
// every block owns 8 rows of one dense block and its 4 waves split the columns, the 64 lanes of
// a wave streaming the rows with 16-byte loads (one float64 complex, or two float32 complex per
// load); each x chunk is loaded once per wave and reused for the 8 rows, row sums are reduced
// with cross-lane shuffles and then across the waves in a fixed order.  Several independent
// products (different matrices and vectors) share one launch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "linalg.h"
#include "prof.h"
#include "tune.h"

namespace bem {
namespace dev {

constexpr int kWave = 64;
// A block of the grouped GEMV owns RPB rows of one matrix (4, 8 or 16, chosen per problem class
// by the launch tuner: every row is summed the same way whatever RPB is); its kWavesPerBlock
// waves split the columns (every wave reads all the rows over a quarter of the columns), so that
// the grid has enough waves for the HBM latency and x is read once per block from L2.
constexpr int kWavesPerBlock = 4;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

typedef double dx2 __attribute__((ext_vector_type(2)));

// Row sums of one matrix for RPW consecutive rows, float64 storage, float64 accumulation (the
// matrix is streamed once per product: non-temporal loads keep x resident in L2).
template <int RPW>
__device__ __forceinline__ void rows_f64(const double2* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                                         const double2* __restrict__ x, int64_t row0, int lane, int wv,
                                         double2 alpha, double* yr, double* yi) {
  double ar[RPW], ai[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) ar[r] = ai[r] = 0.0;
  const double2* rowp[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) rowp[r] = A + min(row0 + r, rows - 1) * lda;
  // chunks of 2 kWave columns, dealt round-robin to the waves of the block
  for (int64_t cs = int64_t(wv) * 2 * kWave; cs < cols; cs += int64_t(kWavesPerBlock) * 2 * kWave) {
    const int64_t c = cs + lane;
    if (cs + 2 * kWave <= cols) {
      const double2 x0 = x[c], x1 = x[c + kWave];
      double2 a0[RPW], a1[RPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const dx2 u = __builtin_nontemporal_load(reinterpret_cast<const dx2*>(rowp[r] + c));
        const dx2 w = __builtin_nontemporal_load(reinterpret_cast<const dx2*>(rowp[r] + c + kWave));
        a0[r] = make_double2(u[0], u[1]);
        a1[r] = make_double2(w[0], w[1]);
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        ar[r] += a0[r].x * x0.x - a0[r].y * x0.y + a1[r].x * x1.x - a1[r].y * x1.y;
        ai[r] += a0[r].x * x0.y + a0[r].y * x0.x + a1[r].x * x1.y + a1[r].y * x1.x;
      }
    } else {
      for (int h = 0; h < 2; ++h) {
        const int64_t cc = c + h * kWave;
        if (cc < cols) {
          const double2 x0 = x[cc];
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            const double2 a0 = rowp[r][cc];
            ar[r] += a0.x * x0.x - a0.y * x0.y;
            ai[r] += a0.x * x0.y + a0.y * x0.x;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const double sr = wave_sum(ar[r]), si = wave_sum(ai[r]);
    yr[r] += alpha.x * sr - alpha.y * si;
    yi[r] += alpha.x * si + alpha.y * sr;
  }
}

// float32 storage, float64 arithmetic (the float64 residuals of a float32-only operator): the
// loop of rows_f64 with each entry widened as it is loaded.
template <int RPW>
__device__ __forceinline__ void rows_f32w(const float2* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                                          const double2* __restrict__ x, int64_t row0, int lane, int wv,
                                          double2 alpha, double* yr, double* yi) {
  double ar[RPW], ai[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) ar[r] = ai[r] = 0.0;
  const float2* rowp[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) rowp[r] = A + min(row0 + r, rows - 1) * lda;
  for (int64_t cs = int64_t(wv) * 2 * kWave; cs < cols; cs += int64_t(kWavesPerBlock) * 2 * kWave) {
    const int64_t c = cs + lane;
    for (int h = 0; h < 2; ++h) {
      const int64_t cc = c + h * kWave;
      if (cc < cols) {
        const double2 x0 = x[cc];
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const float2 f = rowp[r][cc];
          const double a0x = double(f.x), a0y = double(f.y);
          ar[r] += a0x * x0.x - a0y * x0.y;
          ai[r] += a0x * x0.y + a0y * x0.x;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const double sr = wave_sum(ar[r]), si = wave_sum(ai[r]);
    yr[r] += alpha.x * sr - alpha.y * si;
    yi[r] += alpha.x * si + alpha.y * sr;
  }
}

typedef float fx4 __attribute__((ext_vector_type(4)));

// float32 storage and accumulation; each lane reads two consecutive complex entries per
// 16-byte non-temporal load (two 8-byte loads when the rows are not 16-byte aligned); chunks of
// 4 kWave columns are dealt round-robin to the waves of the block.
template <int RPW, bool ALIGNED>
__device__ __forceinline__ void rows_f32(const float2* __restrict__ A, int64_t lda, int64_t rows, int64_t cols,
                                         const double2* __restrict__ x, int64_t row0, int lane, int wv,
                                         double2 alpha, double* yr, double* yi) {
  float ar[RPW], ai[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) ar[r] = ai[r] = 0.0f;
  const float2* rowp[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) rowp[r] = A + min(row0 + r, rows - 1) * lda;
  for (int64_t cs = int64_t(wv) * 4 * kWave; cs < cols; cs += int64_t(kWavesPerBlock) * 4 * kWave) {
    const int64_t c = cs + 2 * lane;
    if (cs + 4 * kWave <= cols) {
      const double2 xa = x[c], xb = x[c + 1], xc = x[c + 2 * kWave], xd = x[c + 2 * kWave + 1];
      const float x0r = float(xa.x), x0i = float(xa.y), x1r = float(xb.x), x1i = float(xb.y);
      const float x2r = float(xc.x), x2i = float(xc.y), x3r = float(xd.x), x3i = float(xd.y);
      float4 a0[RPW], a1[RPW];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        if (ALIGNED) {
          const fx4 u = __builtin_nontemporal_load(reinterpret_cast<const fx4*>(rowp[r] + c));
          const fx4 w = __builtin_nontemporal_load(reinterpret_cast<const fx4*>(rowp[r] + c + 2 * kWave));
          a0[r] = make_float4(u[0], u[1], u[2], u[3]);
          a1[r] = make_float4(w[0], w[1], w[2], w[3]);
        } else {
          const float2 p0 = rowp[r][c], p1 = rowp[r][c + 1];
          const float2 p2 = rowp[r][c + 2 * kWave], p3 = rowp[r][c + 2 * kWave + 1];
          a0[r] = make_float4(p0.x, p0.y, p1.x, p1.y);
          a1[r] = make_float4(p2.x, p2.y, p3.x, p3.y);
        }
      }
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        ar[r] += a0[r].x * x0r - a0[r].y * x0i + a0[r].z * x1r - a0[r].w * x1i;
        ai[r] += a0[r].x * x0i + a0[r].y * x0r + a0[r].z * x1i + a0[r].w * x1r;
        ar[r] += a1[r].x * x2r - a1[r].y * x2i + a1[r].z * x3r - a1[r].w * x3i;
        ai[r] += a1[r].x * x2i + a1[r].y * x2r + a1[r].z * x3i + a1[r].w * x3r;
      }
    } else {
      for (int h = 0; h < 4; ++h) {
        const int64_t cc = c + (h & 1) + (h >> 1) * 2 * kWave;
        if (cc < cols) {
          const double2 xv = x[cc];
          const float xr = float(xv.x), xi = float(xv.y);
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            const float2 a0 = rowp[r][cc];
            ar[r] += a0.x * xr - a0.y * xi;
            ai[r] += a0.x * xi + a0.y * xr;
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const double sr = double(wave_sum(ar[r])), si = double(wave_sum(ai[r]));
    yr[r] += alpha.x * sr - alpha.y * si;
    yi[r] += alpha.x * si + alpha.y * sr;
  }
}


template <int RPB>
__global__ void __launch_bounds__(256) k_gemv_grouped(GemvPack pack) {
  const int64_t b = blockIdx.x;
  int di = 0;
  while (di + 1 < pack.n && pack.d[di + 1].tile0 <= b) ++di;
  const GemvDev& d = pack.d[di];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t row0 = (b - d.tile0) * RPB;
  constexpr int R = RPB;
  double yr[R], yi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) yr[r] = yi[r] = 0.0;
  if (d.fp32 == 2) {
    rows_f32w<R>(static_cast<const float2*>(d.A), d.lda, d.rows, d.cols, d.x, row0, lane, wave,
                 make_double2(d.ar, d.ai), yr, yi);
    if (d.A2)
      rows_f32w<R>(static_cast<const float2*>(d.A2), d.lda2, d.rows, d.cols, d.x2, row0, lane, wave,
                   make_double2(d.a2r, d.a2i), yr, yi);
  } else if (d.fp32) {
    const bool al1 = ((reinterpret_cast<uintptr_t>(d.A) | uintptr_t(d.lda * 8)) & 15) == 0;
    if (al1)
      rows_f32<R, true>(static_cast<const float2*>(d.A), d.lda, d.rows, d.cols, d.x, row0, lane, wave,
                        make_double2(d.ar, d.ai), yr, yi);
    else
      rows_f32<R, false>(static_cast<const float2*>(d.A), d.lda, d.rows, d.cols, d.x, row0, lane, wave,
                         make_double2(d.ar, d.ai), yr, yi);
    if (d.A2) {
      const bool al2 = ((reinterpret_cast<uintptr_t>(d.A2) | uintptr_t(d.lda2 * 8)) & 15) == 0;
      if (al2)
        rows_f32<R, true>(static_cast<const float2*>(d.A2), d.lda2, d.rows, d.cols, d.x2, row0, lane, wave,
                          make_double2(d.a2r, d.a2i), yr, yi);
      else
        rows_f32<R, false>(static_cast<const float2*>(d.A2), d.lda2, d.rows, d.cols, d.x2, row0, lane, wave,
                           make_double2(d.a2r, d.a2i), yr, yi);
    }
  } else {
    rows_f64<R>(static_cast<const double2*>(d.A), d.lda, d.rows, d.cols, d.x, row0, lane, wave,
                make_double2(d.ar, d.ai), yr, yi);
    if (d.A2)
      rows_f64<R>(static_cast<const double2*>(d.A2), d.lda2, d.rows, d.cols, d.x2, row0, lane, wave,
                  make_double2(d.a2r, d.a2i), yr, yi);
  }
  // the waves' partial row sums, added in wave order
  __shared__ double red[kWavesPerBlock][R][2];
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      red[wave][r][0] = yr[r];
      red[wave][r][1] = yi[r];
    }
  }
  __syncthreads();
  if (wave == 0 && lane < R && row0 + lane < d.rows) {
    double vr = 0, vi = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
      vr += red[w][lane][0];
      vi += red[w][lane][1];
    }
    double2* y = d.y + row0 + lane;
    if (d.accumulate) { vr += y->x; vi += y->y; }
    *y = make_double2(vr, vi);
  }
}

// ----------------------------------------------------------------- glue

__global__ void k_expand_charge(const double2* __restrict__ w, double2* __restrict__ full,
                                const int64_t* __restrict__ obj_tri, double2 scale, int64_t ldw, int64_t ldf) {
  const int64_t o = blockIdx.x;
  w += int64_t(blockIdx.y) * ldw;
  full += int64_t(blockIdx.y) * ldf;
  const int64_t t0 = obj_tri[o], t1 = obj_tri[o + 1];
  // kept charges of object o are w[t0 - o .. t1 - o - 2]; the last triangle t1-1 is eliminated
  const int64_t q0 = t0 - o;
  const int64_t nk = t1 - t0 - 1;
  __shared__ double sr[256], si[256];
  double ar = 0, ai = 0;
  for (int64_t i = threadIdx.x; i < nk; i += blockDim.x) {
    const double2 v = w[q0 + i];
    ar += v.x;
    ai += v.y;
    full[t0 + i] = make_double2(scale.x * v.x - scale.y * v.y, scale.x * v.y + scale.y * v.x);
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = -sr[0], i = -si[0];
    full[t1 - 1] = make_double2(scale.x * r - scale.y * i, scale.x * i + scale.y * r);
  }
}

__global__ void k_DT(const double2* __restrict__ z, const int32_t* __restrict__ tp, const int32_t* __restrict__ tm,
                     int64_t ne, double2 s, const double2* __restrict__ sedge, double2* __restrict__ y, int acc,
                     int64_t ldz, int64_t ldy) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ne) return;
  z += int64_t(blockIdx.y) * ldz;
  y += int64_t(blockIdx.y) * ldy;
  const double2 a = z[tp[n]], b = z[tm[n]];
  const double dr = a.x - b.x, di = a.y - b.y;
  double2 sc = s;
  if (sedge) {
    const double2 q = sedge[n];
    sc = make_double2(s.x * q.x - s.y * q.y, s.x * q.y + s.y * q.x);
  }
  double yr = sc.x * dr - sc.y * di, yi = sc.x * di + sc.y * dr;
  if (acc) { yr += y[n].x; yi += y[n].y; }
  y[n] = make_double2(yr, yi);
}

__global__ void k_FD(const double2* __restrict__ u, const int32_t* __restrict__ tri_edge,
                     const int8_t* __restrict__ tri_sign, const int32_t* __restrict__ kept, int64_t nq, double2 s1,
                     const double2* __restrict__ w, double2 s2, double2* __restrict__ y, int64_t ldu, int64_t ldw,
                     int64_t ldy) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  u += int64_t(blockIdx.y) * ldu;
  if (w) w += int64_t(blockIdx.y) * ldw;
  y += int64_t(blockIdx.y) * ldy;
  const int64_t t = kept[q];
  double dr = 0, di = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 v = u[tri_edge[3 * t + i]];
    const double sg = double(tri_sign[3 * t + i]);
    dr += sg * v.x;
    di += sg * v.y;
  }
  double yr = s1.x * dr - s1.y * di, yi = s1.x * di + s1.y * dr;
  if (w) {
    const double2 v = w[q];
    yr += s2.x * v.x - s2.y * v.y;
    yi += s2.x * v.y + s2.y * v.x;
  }
  y[q] = make_double2(yr, yi);
}

__global__ void k_spmv(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, const double* __restrict__ val,
                       int64_t rows, const double2* __restrict__ x, double2 s, double2* __restrict__ y, int acc,
                       int64_t ldx, int64_t ldy) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  x += int64_t(blockIdx.y) * ldx;
  y += int64_t(blockIdx.y) * ldy;
  double ar = 0, ai = 0;
  for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) {
    const double2 v = x[idx[p]];
    ar += val[p] * v.x;
    ai += val[p] * v.y;
  }
  double yr = s.x * ar - s.y * ai, yi = s.x * ai + s.y * ar;
  if (acc) { yr += y[r].x; yi += y[r].y; }
  y[r] = make_double2(yr, yi);
}

// The same product added to two outputs with their own scales: y1 (+)= s1 A x, y2 (+)= s2 A x
// (one pass over A and x).
__global__ void k_spmv2(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                        const double* __restrict__ val, int64_t rows, const double2* __restrict__ x, int64_t ldx,
                        double2 s1, double2* __restrict__ y1, int64_t ldy1, int acc1, double2 s2,
                        double2* __restrict__ y2, int64_t ldy2, int acc2) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  x += int64_t(blockIdx.y) * ldx;
  y1 += int64_t(blockIdx.y) * ldy1;
  y2 += int64_t(blockIdx.y) * ldy2;
  double ar = 0, ai = 0;
  for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) {
    const double2 v = x[idx[p]];
    ar += val[p] * v.x;
    ai += val[p] * v.y;
  }
  double yr = s1.x * ar - s1.y * ai, yi = s1.x * ai + s1.y * ar;
  if (acc1) { yr += y1[r].x; yi += y1[r].y; }
  y1[r] = make_double2(yr, yi);
  yr = s2.x * ar - s2.y * ai;
  yi = s2.x * ai + s2.y * ar;
  if (acc2) { yr += y2[r].x; yi += y2[r].y; }
  y2[r] = make_double2(yr, yi);
}

__global__ void k_axpby(int64_t n, double2 a, const double2* __restrict__ x, double2 b, const double2* __restrict__ y,
                        double2* __restrict__ z, int64_t ldx, int64_t ldy, int64_t ldz) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (x) x += int64_t(blockIdx.y) * ldx;
  if (y) y += int64_t(blockIdx.y) * ldy;
  z += int64_t(blockIdx.y) * ldz;
  const double2 u = x ? x[i] : make_double2(0, 0), v = y ? y[i] : make_double2(0, 0);
  z[i] = make_double2(a.x * u.x - a.y * u.y + b.x * v.x - b.y * v.y, a.x * u.y + a.y * u.x + b.x * v.y + b.y * v.x);
}

__global__ void k_diag(const double2* __restrict__ A, int64_t ld, int64_t n, double2* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = A[i * ld + i];
}

__global__ void k_cast_f64(const float2* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                           double2* __restrict__ dst, int64_t ldd) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= cols) return;
  const float2 v = src[r * lds + c];
  dst[r * ldd + c] = make_double2(double(v.x), double(v.y));
}

__global__ void k_cast_f32(const double2* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                           float2* __restrict__ dst, int64_t ldd) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= ldd) return;
  if (c < cols) {
    const double2 v = src[r * lds + c];
    dst[r * ldd + c] = make_float2(float(v.x), float(v.y));
  } else {
    dst[r * ldd + c] = make_float2(0.f, 0.f);
  }
}

// ----------------------------------------------------------------- Krylov

// one block per basis vector: h[i] = sum_n conj(V_i[n]) w[n]
__global__ void __launch_bounds__(256) k_mdot(const double2* __restrict__ V, int64_t ldv,
                                              const double2* __restrict__ w, int64_t n, double2* __restrict__ h) {
  const int i = blockIdx.x;
  const double2* vi = V + int64_t(i) * ldv;
  double ar = 0, ai = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    const double2 a = vi[k], b = w[k];
    ar += a.x * b.x + a.y * b.y;
    ai += a.x * b.y - a.y * b.x;
  }
  __shared__ double sr[4], si[4];
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  const int wv = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) { sr[wv] = ar; si[wv] = ai; }
  __syncthreads();
  if (threadIdx.x == 0) h[i] = make_double2(sr[0] + sr[1] + sr[2] + sr[3], si[0] + si[1] + si[2] + si[3]);
}

__global__ void k_mupdate(const double2* __restrict__ V, int64_t ldv, int j, const double2* __restrict__ h, double sign,
                          double2* __restrict__ w, int64_t n) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double ar = w[k].x, ai = w[k].y;
  for (int i = 0; i < j; ++i) {
    const double2 a = V[int64_t(i) * ldv + k], c = h[i];
    ar += sign * (a.x * c.x - a.y * c.y);
    ai += sign * (a.x * c.y + a.y * c.x);
  }
  w[k] = make_double2(ar, ai);
}

constexpr int kNormBlocks = 128;

__global__ void __launch_bounds__(256) k_norm_partial(const double2* __restrict__ w, int64_t n, double* __restrict__ part) {
  double s = 0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x) {
    const double2 a = w[k];
    s += a.x * a.x + a.y * a.y;
  }
  s = wave_sum(s);
  __shared__ double sh[4];
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_norm_final(const double* __restrict__ part, int nb, double2* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *out = make_double2(sqrt(s), 0.0);
}

__global__ void k_scale_inv(const double2* __restrict__ w, int64_t n, const double2* __restrict__ nrm,
                            double2* __restrict__ v) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double s = nrm->x > 0 ? 1.0 / nrm->x : 0.0;
  v[k] = make_double2(w[k].x * s, w[k].y * s);
}

// Hcol: entries 0..j (projections) and j+1 (norm of the new vector, real).
// Column j of the Hessenberg matrix (h2, if given, is added to entries 0..j first) gets the j
// earlier rotations and then the new rotation that zeroes entry j+1; g is rotated with it and
// |g_{j+1}| is the residual norm.  Run by one wave: the rotations and the column are staged
// through LDS in chunks with coalesced loads, so the serial recurrence of lane 0 (the rotated
// entry carried in registers) reads only LDS.
__device__ void givens_step(const double2* Hcol, double2* Rcol, int j, const double2* __restrict__ cs_in,
                            const double2* __restrict__ sn_in, double2* __restrict__ cs, double2* __restrict__ sn,
                            double2* __restrict__ g, double* __restrict__ res, const double2* __restrict__ h2) {
  constexpr int CH = 256;
  __shared__ double2 sh[CH + 1], sc[CH], ss[CH];
  const int t = threadIdx.x, nth = blockDim.x;
  auto hload = [&](int i) {
    double2 v = Hcol[i];
    if (h2) v = make_double2(v.x + h2[i].x, v.y + h2[i].y);
    return v;
  };
  double2 a = make_double2(0, 0);  // lane 0: entry i0 of the column, rotations before i0 applied
  if (t == 0) a = hload(0);
  for (int i0 = 0; i0 < j; i0 += CH) {
    const int cnt = min(CH, j - i0);
    for (int e = t; e < cnt; e += nth) {
      sh[e + 1] = hload(i0 + e + 1);
      sc[e] = cs_in[i0 + e];
      ss[e] = sn_in[i0 + e];
    }
    __syncthreads();
    if (t == 0) {
      // [h_i; h_{i+1}] <- [c, s; -conj(s), c] [h_i; h_{i+1}]  (c real)
#pragma unroll 8
      for (int e = 0; e < cnt; ++e) {
        const double c = sc[e].x;
        const double2 sv = ss[e], b = sh[e + 1];
        sh[e] = make_double2(c * a.x + (sv.x * b.x - sv.y * b.y), c * a.y + (sv.x * b.y + sv.y * b.x));
        a = make_double2(-(sv.x * a.x + sv.y * a.y) + c * b.x, -(sv.x * a.y - sv.y * a.x) + c * b.y);
      }
    }
    __syncthreads();
    for (int e = t; e < cnt; e += nth) Rcol[i0 + e] = sh[e];
    __syncthreads();
  }
  if (t != 0) return;
  const double2 b = Hcol[j + 1];
  const double na = hypot(a.x, a.y), nb = hypot(b.x, b.y);
  double c;
  double2 s;
  if (nb == 0.0) {
    c = 1.0;
    s = make_double2(0, 0);
  } else if (na == 0.0) {
    c = 0.0;
    s = make_double2(b.x / nb, -b.y / nb);  // s = conj(b)/|b|
  } else {
    const double t2 = hypot(na, nb);
    c = na / t2;
    // s = (a/|a|) conj(b) / t
    const double2 ua = make_double2(a.x / na, a.y / na);
    s = make_double2((ua.x * b.x + ua.y * b.y) / t2, (ua.y * b.x - ua.x * b.y) / t2);
  }
  cs[j] = make_double2(c, 0);
  sn[j] = s;
  // rotated column: R[j] = c a + s b ; R[j+1] = 0
  Rcol[j] = make_double2(c * a.x + (s.x * b.x - s.y * b.y), c * a.y + (s.x * b.y + s.y * b.x));
  Rcol[j + 1] = make_double2(0, 0);
  const double2 gj = g[j];
  g[j] = make_double2(c * gj.x, c * gj.y);
  // g[j+1] = -conj(s) g_j
  g[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
  *res = hypot(g[j + 1].x, g[j + 1].y);
}

__global__ void __launch_bounds__(64) k_givens(double2* Hcol, int j, double2* cs, double2* sn, double2* g,
                                               double* res, const double2* h2) {
  givens_step(Hcol, Hcol, j, cs, sn, cs, sn, g, res, h2);
}

// y = R^{-1} g for the leading j x j upper-triangular block of H (column-major, ldh)
__device__ void backsolve(const double2* H, int64_t ldh, int j, const double2* g, double2* y) {
  for (int i = j - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int k = i + 1; k < j; ++k) {
      const double2 h = H[int64_t(k) * ldh + i], yk = y[k];
      s.x -= h.x * yk.x - h.y * yk.y;
      s.y -= h.x * yk.y + h.y * yk.x;
    }
    const double2 d = H[int64_t(i) * ldh + i];
    const double dd = d.x * d.x + d.y * d.y;
    y[i] = make_double2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
  }
}

__global__ void k_backsolve(const double2* H, int64_t ldh, int j, const double2* g, double2* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  backsolve(H, ldh, j, g, y);
}

__global__ void k_init_g(double2* g, int mmax, const double2* beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > mmax) return;
  g[i] = i == 0 ? make_double2(beta->x, 0) : make_double2(0, 0);
}

// ---- batched Krylov: R independent spaces, vector i of column c at V + (i R + c) ldv

constexpr int kChunk = 2048;  // vector elements per block of the batched reductions
constexpr int kPer = kChunk / 256;

// part[(c j1 + i) nch + ch] = sum over chunk ch of conj(V_i,c) w_c
__global__ void __launch_bounds__(256) k_bmdot_part(const double2* __restrict__ V, int64_t ldv, int R, int j1,
                                                    const double2* __restrict__ W, int64_t ldw, int64_t n, int nch,
                                                    double2* __restrict__ part) {
  const int ch = blockIdx.x, c = blockIdx.y;
  const int64_t k0 = int64_t(ch) * kChunk + threadIdx.x;
  const double2* w = W + int64_t(c) * ldw;
  double2 wl[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = k0 + 256 * s;
    wl[s] = k < n ? w[k] : make_double2(0, 0);
  }
  __shared__ double2 red[4];
  const int wv = threadIdx.x / kWave;
  for (int i = 0; i < j1; ++i) {
    const double2* v = V + (int64_t(i) * R + c) * ldv;
    double ar = 0, ai = 0;
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int64_t k = k0 + 256 * s;
      if (k < n) {
        const double2 a = v[k];
        ar += a.x * wl[s].x + a.y * wl[s].y;
        ai += a.x * wl[s].y - a.y * wl[s].x;
      }
    }
    ar = wave_sum(ar);
    ai = wave_sum(ai);
    if (threadIdx.x % kWave == 0) red[wv] = make_double2(ar, ai);
    __syncthreads();
    if (threadIdx.x == 0)
      part[(int64_t(c) * j1 + i) * nch + ch] =
          make_double2(red[0].x + red[1].x + red[2].x + red[3].x, red[0].y + red[1].y + red[2].y + red[3].y);
    __syncthreads();
  }
}

// Same partial sums with one block per (chunk, basis vector, column): for few columns, where
// the chunk-per-block form above leaves the GPU mostly idle.  Identical summation order.
__global__ void __launch_bounds__(256) k_bmdot_part3(const double2* __restrict__ V, int64_t ldv, int R, int j1,
                                                     const double2* __restrict__ W, int64_t ldw, int64_t n, int nch,
                                                     double2* __restrict__ part) {
  const int ch = blockIdx.x, i = blockIdx.y, c = blockIdx.z;
  const int64_t k0 = int64_t(ch) * kChunk + threadIdx.x;
  const double2* w = W + int64_t(c) * ldw;
  const double2* v = V + (int64_t(i) * R + c) * ldv;
  double ar = 0, ai = 0;
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = k0 + 256 * s;
    const double2 wl = k < n ? w[k] : make_double2(0, 0);
    if (k < n) {
      const double2 a = v[k];
      ar += a.x * wl.x + a.y * wl.y;
      ai += a.x * wl.y - a.y * wl.x;
    }
  }
  __shared__ double2 red[4];
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = make_double2(ar, ai);
  __syncthreads();
  if (threadIdx.x == 0)
    part[(int64_t(c) * j1 + i) * nch + ch] =
        make_double2(red[0].x + red[1].x + red[2].x + red[3].x, red[0].y + red[1].y + red[2].y + red[3].y);
}

__global__ void k_bmdot_final(const double2* __restrict__ part, int nch, int j1, double2* __restrict__ h,
                              int64_t hstride) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < j1; i += blockDim.x) {
    const double2* p = part + (int64_t(c) * j1 + i) * nch;
    double ar = 0, ai = 0;
    for (int ch = 0; ch < nch; ++ch) {
      ar += p[ch].x;
      ai += p[ch].y;
    }
    h[int64_t(c) * hstride + i] = make_double2(ar, ai);
  }
}

// w_c += sign sum_{i < j_c} V_i,c h_i,c.  A block owns 64 consecutive elements (one per lane);
// its four waves take the basis vectors i = wave, wave + 4, ... and their partial sums are
// added in LDS in a fixed order, then to w: one column alone still gives n / 64 blocks.
__global__ void __launch_bounds__(256) k_bmupdate(const double2* __restrict__ V, int64_t ldv, int R, int j1,
                                                  const int* __restrict__ jr, const double2* __restrict__ h,
                                                  int64_t hstride, double sign, double2* __restrict__ W,
                                                  int64_t ldw, int64_t n) {
  const int c = blockIdx.y, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t k = int64_t(blockIdx.x) * 64 + lane;
  const int jc = jr ? jr[c] : j1;
  const double2* hc = h + int64_t(c) * hstride;
  double ar = 0, ai = 0;
  if (k < n) {
#pragma unroll 4
    for (int i = wv; i < jc; i += 4) {
      const double2 a = V[(int64_t(i) * R + c) * ldv + k], q = hc[i];
      ar += a.x * q.x - a.y * q.y;
      ai += a.x * q.y + a.y * q.x;
    }
  }
  __shared__ double2 red[4][64];
  red[wv][lane] = make_double2(ar, ai);
  __syncthreads();
  if (wv == 0 && k < n) {
    const double sr = ((red[0][lane].x + red[1][lane].x) + red[2][lane].x) + red[3][lane].x;
    const double si = ((red[0][lane].y + red[1][lane].y) + red[2][lane].y) + red[3][lane].y;
    double2* w = W + int64_t(c) * ldw;
    w[k] = make_double2(w[k].x + sign * sr, w[k].y + sign * si);
  }
}

// ---- Gram-Schmidt with delayed reorthogonalisation (one read of the basis for the two
// projections of a step, one for the two updates).  Step j holds the basis V_0..V_{j-1}
// (final) and V_j, the previous step's vector after one projection (tentative), and the
// product Y = A V_j.

// part1 / part2[(c j1 + i) nch + ch] = chunk sums of conj(V_i,c) X_c and conj(V_i,c) Y_c
// (j1 = j + 1 basis vectors, X_c = V_j,c): each basis chunk is read once for both.  Block
// (ch, c, q) takes basis vectors [q G, (q + 1) G) with its chunk of X and Y held in registers.
__global__ void __launch_bounds__(256) k_bmdot2_part(const double2* __restrict__ V, int64_t ldv, int R, int j1,
                                                     int G, const double2* __restrict__ X,
                                                     const double2* __restrict__ Y, int64_t ldy, int64_t n, int nch,
                                                     double2* __restrict__ part1, double2* __restrict__ part2) {
  const int ch = blockIdx.x, c = blockIdx.y;
  const int ib = int(blockIdx.z) * G, ie = min(j1, ib + G);
  const int64_t k0 = int64_t(ch) * kChunk + threadIdx.x;
  const double2* x = X + int64_t(c) * ldv;
  const double2* y = Y + int64_t(c) * ldy;
  double2 xl[kPer], yl[kPer];
#pragma unroll
  for (int s = 0; s < kPer; ++s) {
    const int64_t k = k0 + 256 * s;
    xl[s] = k < n ? x[k] : make_double2(0, 0);
    yl[s] = k < n ? y[k] : make_double2(0, 0);
  }
  __shared__ double2 red[2][4];
  const int wv = threadIdx.x / kWave;
  for (int i = ib; i < ie; ++i) {
    const double2* v = V + (int64_t(i) * R + c) * ldv;
    double xr = 0, xi = 0, yr = 0, yi = 0;
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
      const int64_t k = k0 + 256 * s;
      if (k < n) {
        const double2 a = v[k];
        xr += a.x * xl[s].x + a.y * xl[s].y;
        xi += a.x * xl[s].y - a.y * xl[s].x;
        yr += a.x * yl[s].x + a.y * yl[s].y;
        yi += a.x * yl[s].y - a.y * yl[s].x;
      }
    }
    xr = wave_sum(xr);
    xi = wave_sum(xi);
    yr = wave_sum(yr);
    yi = wave_sum(yi);
    if (threadIdx.x % kWave == 0) {
      red[0][wv] = make_double2(xr, xi);
      red[1][wv] = make_double2(yr, yi);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
      const double2* q = red[threadIdx.x];
      double2* out = threadIdx.x == 0 ? part1 : part2;
      out[(int64_t(c) * j1 + i) * nch + ch] = make_double2(q[0].x + q[1].x + q[2].x + q[3].x, q[0].y + q[1].y + q[2].y + q[3].y);
    }
    __syncthreads();
  }
}

// Per column (one block): d1 = V^H V_j and d2 = V^H Y summed over the chunks (j1 = j + 1 entries
// each), then with a = d1[0..j), alpha = d1[j] the reorthogonalisation of V_j:
//   r = sqrt(alpha - |a|^2)     (the norm of V_j - V a, the basis before V_j orthonormal)
//   column j - 1 of H (tentative: its last entry is rho_j, the norm V_j was scaled by):
//     H[i][j-1] += rho_j a_i,  H[j][j-1] = rho_j r
//   the new column j: the final v_j = (V_j - V a) / r has the product (Y - V g) / r with
//     g = H a (A V = V H over the finished columns), so its projection is
//     H[i][j] = (d_i - g_i) / r,  d = (d2_0, .., d2_{j-1}, (d2_j - a^H d2) / r),
// and the update coefficients a (coef[0..j)), cf = d (coef[j+1 .. 2j+1], as V g lies in the
// span the projection removes, the new vector is (Y - V cf) / r) and 1/r.  Frozen columns get
// a = 0, cf = 0, 1/r = 1, column j zero and column j - 1 untouched.  Sums in a fixed order
// (deterministic).
constexpr int kCoefThreads = 256;
__global__ void __launch_bounds__(kCoefThreads) k_bdcgs2_coef(const double2* __restrict__ part1,
                                                              const double2* __restrict__ part2, int nch, int j,
                                                              double2* __restrict__ H, int64_t hs, int64_t ldh,
                                                              double2* __restrict__ coef, int64_t cstride,
                                                              double* __restrict__ rinv,
                                                              const int* __restrict__ frozen) {
  constexpr int NT = kCoefThreads;
  const int c = blockIdx.x, t = threadIdx.x, j1 = j + 1;
  double2* cc = coef + int64_t(c) * cstride;
  double2* d2 = cc + j1;  // the summed d2 (coef[j1 .. 2 j1)), then the update coefficients
  double2* Hc = H + int64_t(c) * hs;
  const bool fz = frozen && frozen[c];
  // chunk sums: d1 into coef[0..j1), d2 into coef[j1..2 j1)
  for (int i = t; i < j1; i += NT) {
    double ar = 0, ai = 0, br = 0, bi = 0;
    const double2* p = part1 + (int64_t(c) * j1 + i) * nch;
    const double2* q = part2 + (int64_t(c) * j1 + i) * nch;
    for (int ch = 0; ch < nch; ++ch) {
      ar += p[ch].x;
      ai += p[ch].y;
      br += q[ch].x;
      bi += q[ch].y;
    }
    cc[i] = make_double2(ar, ai);
    d2[i] = make_double2(br, bi);
  }
  __syncthreads();
  // |a|^2 and a^H d2 over i < j: strided partials, a fixed butterfly per wave, the four waves in
  // order
  double na = 0, pr = 0, pi = 0;
  for (int i = t; i < j; i += NT) {
    const double2 a = cc[i], z = d2[i];
    na += a.x * a.x + a.y * a.y;
    pr += a.x * z.x + a.y * z.y;
    pi += a.x * z.y - a.y * z.x;
  }
  na = wave_sum(na);
  pr = wave_sum(pr);
  pi = wave_sum(pi);
  __shared__ double red[3][NT / kWave];
  if (t % kWave == 0) {
    red[0][t / kWave] = na;
    red[1][t / kWave] = pr;
    red[2][t / kWave] = pi;
  }
  __syncthreads();
  na = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
  pr = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
  pi = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
  const double alpha = cc[j].x;
  const double r2 = alpha - na;
  const bool ok = !fz && j > 0 && r2 > 0.0;
  const double r = ok ? sqrt(r2) : 1.0;
  const double ir = 1.0 / r;
  if (!fz && j > 0) {
    double2* Hp = Hc + int64_t(j - 1) * ldh;
    const double rho = Hp[j].x;
    for (int i = t; i < j; i += NT) Hp[i] = make_double2(Hp[i].x + rho * cc[i].x, Hp[i].y + rho * cc[i].y);
    if (t == 0) Hp[j] = make_double2(rho * r, 0.0);
  }
  __syncthreads();
  double2* Hj = Hc + int64_t(j) * ldh;
  const double2 zj = d2[j];
  const double2 last = make_double2((zj.x - pr) * ir * ir, (zj.y - pi) * ir * ir);
  // H[k][j] = (d_k - g_k) / r with d = (d2_0 .. d2_{j-1}, r last) and g = H a over the finished
  // columns 0..j-1 (rows k <= j; column i holds rows 0..i+1), each row summed in column order
  for (int k = t; k <= j; k += NT) {
    double gr = 0, gi = 0;
    if (!fz)
      for (int i = k > 0 ? k - 1 : 0; i < j; ++i) {
        const double2 h = Hc[int64_t(i) * ldh + k], av = cc[i];
        gr += h.x * av.x - h.y * av.y;
        gi += h.x * av.y + h.y * av.x;
      }
    const double2 d = k < j ? d2[k] : make_double2(last.x * r, last.y * r);
    Hj[k] = fz ? make_double2(0, 0) : make_double2((d.x - gr) * ir, (d.y - gi) * ir);
  }
  __syncthreads();
  // update coefficients: cf = d (cf_i = d2_i for i < j, cf_j = r last); a and cf zeroed when
  // frozen
  for (int i = t; i < j; i += NT) {
    if (fz || j == 0) {
      cc[i] = make_double2(0, 0);
      d2[i] = make_double2(0, 0);
    }
  }
  if (t == 0) {
    d2[j] = fz ? make_double2(0, 0) : make_double2(last.x * r, last.y * r);
    rinv[c] = ir;
  }
}

// v_j <- (V_j - sum_{i<j} V_i a_i) / r;  Y <- (Y - sum_{i<j} V_i cf_i - v_j cf_j) / r, in place
// (V_j is slot j of V; Y the product).  A block owns 64 consecutive elements; its four waves
// take the basis vectors i = wave, wave + 4, ... and their partial sums are added in LDS in a
// fixed order.
__global__ void __launch_bounds__(256) k_bdcgs2_update(double2* __restrict__ V, int64_t ldv, int R, int j,
                                                       const double2* __restrict__ coef, int64_t cstride,
                                                       const double* __restrict__ rinv, double2* __restrict__ Y,
                                                       int64_t ldy, int64_t n) {
  const int c = blockIdx.y, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t k = int64_t(blockIdx.x) * 64 + lane;
  const double2* a = coef + int64_t(c) * cstride;
  const double2* cf = a + (j + 1);
  double sa_r = 0, sa_i = 0, sc_r = 0, sc_i = 0;
  if (k < n) {
#pragma unroll 4
    for (int i = wv; i < j; i += 4) {
      const double2 v = V[(int64_t(i) * R + c) * ldv + k], p = a[i], q = cf[i];
      sa_r += v.x * p.x - v.y * p.y;
      sa_i += v.x * p.y + v.y * p.x;
      sc_r += v.x * q.x - v.y * q.y;
      sc_i += v.x * q.y + v.y * q.x;
    }
  }
  __shared__ double2 red[2][4][64];
  red[0][wv][lane] = make_double2(sa_r, sa_i);
  red[1][wv][lane] = make_double2(sc_r, sc_i);
  __syncthreads();
  if (wv == 0 && k < n) {
    const double ar = ((red[0][0][lane].x + red[0][1][lane].x) + red[0][2][lane].x) + red[0][3][lane].x;
    const double ai = ((red[0][0][lane].y + red[0][1][lane].y) + red[0][2][lane].y) + red[0][3][lane].y;
    const double cr = ((red[1][0][lane].x + red[1][1][lane].x) + red[1][2][lane].x) + red[1][3][lane].x;
    const double ci = ((red[1][0][lane].y + red[1][1][lane].y) + red[1][2][lane].y) + red[1][3][lane].y;
    const double ir = rinv[c];
    double2* vj = V + (int64_t(j) * R + c) * ldv + k;
    const double2 vf = make_double2((vj->x - ar) * ir, (vj->y - ai) * ir);
    const double2 q = cf[j];
    double2* y = Y + int64_t(c) * ldy + k;
    const double yr = y->x - cr - (vf.x * q.x - vf.y * q.y), yi = y->y - ci - (vf.x * q.y + vf.y * q.x);
    *y = make_double2(yr * ir, yi * ir);
    *vj = vf;
  }
}

__global__ void __launch_bounds__(256) k_bnorm_part(const double2* __restrict__ W, int64_t ldw, int64_t n, int nch,
                                                    double* __restrict__ part) {
  const int ch = blockIdx.x, c = blockIdx.y;
  const double2* w = W + int64_t(c) * ldw;
  double s = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int64_t k = int64_t(ch) * kChunk + threadIdx.x + 256 * q;
    if (k < n) {
      const double2 a = w[k];
      s += a.x * a.x + a.y * a.y;
    }
  }
  s = wave_sum(s);
  __shared__ double sh[4];
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[int64_t(c) * nch + ch] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_bnorm_final(const double* __restrict__ part, int nch, int R, double2* __restrict__ out,
                              int64_t ostride) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= R) return;
  double s = 0;
  for (int ch = 0; ch < nch; ++ch) s += part[int64_t(c) * nch + ch];
  out[int64_t(c) * ostride] = make_double2(sqrt(s), 0.0);
}

__global__ void k_bscale_inv(double2* __restrict__ W, int64_t ldw, int64_t n, const double2* __restrict__ nrm,
                             int64_t nstride, const int* __restrict__ frozen) {
  const int c = blockIdx.y;
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double v = nrm[int64_t(c) * nstride].x;
  const double s = (frozen && frozen[c]) ? 0.0 : (v > 0 ? 1.0 / v : 0.0);
  double2* w = W + int64_t(c) * ldw;
  w[k] = make_double2(w[k].x * s, w[k].y * s);
}

// one wave per column c: the raw Hessenberg column j of H rotated into column j of HR (HR = H:
// in place)
__global__ void __launch_bounds__(64) k_bgivens(const double2* H, double2* HR, int64_t hs, int64_t ldh, int j,
                                                double2* cs, double2* sn, double2* g, double* res, const double2* h2,
                                                int m, int R) {
  const int c = blockIdx.x;
  double2* csc = cs + int64_t(c) * (m + 1);
  double2* snc = sn + int64_t(c) * (m + 1);
  const int64_t off = int64_t(c) * hs + int64_t(j) * ldh;
  givens_step(H + off, HR + off, j, csc, snc, csc, snc, g + int64_t(c) * (m + 2), res + c,
              h2 ? h2 + int64_t(c) * (m + 2) : nullptr);
}

__global__ void k_bbacksolve(const double2* H, int64_t hs, int64_t ldh, const int* jr, const double2* g, double2* y,
                             int m, int R) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= R) return;
  backsolve(H + int64_t(c) * hs, ldh, jr[c], g + int64_t(c) * (m + 2), y + int64_t(c) * (m + 1));
}

__global__ void k_binit_g(double2* g, int m, const double2* beta, int64_t bstride) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < m + 2; i += blockDim.x)
    g[int64_t(c) * (m + 2) + i] = i == 0 ? make_double2(beta[int64_t(c) * bstride].x, 0) : make_double2(0, 0);
}

__global__ void k_gather_cols(const double2* __restrict__ X, int64_t ldx, double2* __restrict__ U, int64_t ldu,
                              const int* __restrict__ idx, int64_t n) {
  const int c = blockIdx.y;
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  U[int64_t(c) * ldu + k] = X[int64_t(idx[c]) * ldx + k];
}

__global__ void k_scatter_cols(const double2* __restrict__ U, int64_t ldu, double2* __restrict__ X, int64_t ldx,
                               const int* __restrict__ idx, int64_t n, int accumulate) {
  const int c = blockIdx.y;
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double2* x = X + int64_t(idx[c]) * ldx + k;
  const double2 u = U[int64_t(c) * ldu + k];
  *x = accumulate ? make_double2(x->x + u.x, x->y + u.y) : u;
}

}  // namespace dev

// ----------------------------------------------------------------- launchers

void launch_gemv_grouped(const GemvDesc* host_descs, int n, hipStream_t st) {
  static const int kRpb[3] = {8, 4, 16};  // candidates, canonical first
  for (int base = 0; base < n; base += kMaxGroup) {
    GemvPack pack{};
    pack.n = std::min(kMaxGroup, n - base);
    int64_t rows = 0, cols = 0;
    for (int i = 0; i < pack.n; ++i) {
      const GemvDesc& h = host_descs[base + i];
      pack.d[i] = GemvDev{h.A,       h.A2,      h.lda,      h.lda2,     h.rows,       h.cols, h.x, h.x2, h.y,
                          h.alpha.x, h.alpha.y, h.alpha2.x, h.alpha2.y, h.accumulate, h.fp32, 0};
      rows += h.rows;
      cols = std::max(cols, h.cols);
    }
    if (rows == 0) continue;
    double bytes = 0;
    for (int i = 0; i < pack.n; ++i)
      bytes += double(pack.d[i].rows) * pack.d[i].cols * (pack.d[i].fp32 ? 8.0 : 16.0) * (pack.d[i].A2 ? 2 : 1);
    ProfScope ps(st, pack.d[0].fp32 ? KC_GEMV_F32 : KC_GEMV_F64, bytes, bytes / (pack.d[0].fp32 ? 8.0 : 16.0));
    TuneScope ts(tune_key(8, {pack.d[0].fp32, pack.n, log2_bucket(rows), log2_bucket(cols)}), 3, st);
    const int rpb = kRpb[ts.variant()];
    int64_t tiles = 0;
    for (int i = 0; i < pack.n; ++i) {
      pack.d[i].tile0 = tiles;
      tiles += (pack.d[i].rows + rpb - 1) / rpb;
    }
    if (rpb == 4) hipLaunchKernelGGL(dev::k_gemv_grouped<4>, dim3(unsigned(tiles)), dim3(256), 0, st, pack);
    else if (rpb == 16) hipLaunchKernelGGL(dev::k_gemv_grouped<16>, dim3(unsigned(tiles)), dim3(256), 0, st, pack);
    else hipLaunchKernelGGL(dev::k_gemv_grouped<8>, dim3(unsigned(tiles)), dim3(256), 0, st, pack);
    BEM_HIP(hipGetLastError());
  }
}

void launch_expand_charge(const double2* w, double2* full, const int64_t* obj_tri, int64_t nobj, double2 scale,
                          hipStream_t st, int R, int64_t ldw, int64_t ldf) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_expand_charge, dim3(unsigned(nobj), unsigned(R)), dim3(256), 0, st, w, full, obj_tri,
                     scale, ldw, ldf);
  BEM_HIP(hipGetLastError());
}

void launch_DT(const double2* z, const int32_t* tp, const int32_t* tm, int64_t ne, double2 s, const double2* sedge,
               double2* y, int accumulate, hipStream_t st, int R, int64_t ldz, int64_t ldy) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_DT, dim3(unsigned((ne + 255) / 256), unsigned(R)), dim3(256), 0, st, z, tp, tm, ne, s,
                     sedge, y, accumulate, ldz, ldy);
  BEM_HIP(hipGetLastError());
}

void launch_FD(const double2* u, const int32_t* tri_edge, const int8_t* tri_sign, const int32_t* kept, int64_t nq,
               double2 s1, const double2* w, double2 s2, double2* y, hipStream_t st, int R, int64_t ldu, int64_t ldw,
               int64_t ldy) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_FD, dim3(unsigned((nq + 255) / 256), unsigned(R)), dim3(256), 0, st, u, tri_edge,
                     tri_sign, kept, nq, s1, w, s2, y, ldu, ldw, ldy);
  BEM_HIP(hipGetLastError());
}

void launch_spmv(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, const double2* x,
                 double2 s, double2* y, int accumulate, hipStream_t st, int R, int64_t ldx, int64_t ldy) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_spmv, dim3(unsigned((rows + 255) / 256), unsigned(R)), dim3(256), 0, st, ptr, idx, val,
                     rows, x, s, y, accumulate, ldx, ldy);
  BEM_HIP(hipGetLastError());
}

void launch_spmv2(const int64_t* ptr, const int32_t* idx, const double* val, int64_t rows, const double2* x,
                  int64_t ldx, double2 s1, double2* y1, int64_t ldy1, int acc1, double2 s2, double2* y2, int64_t ldy2,
                  int acc2, hipStream_t st, int R) {
  if (R <= 0 || rows <= 0) return;
  hipLaunchKernelGGL(dev::k_spmv2, dim3(unsigned((rows + 255) / 256), unsigned(R)), dim3(256), 0, st, ptr, idx, val,
                     rows, x, ldx, s1, y1, ldy1, acc1, s2, y2, ldy2, acc2);
  BEM_HIP(hipGetLastError());
}

void launch_axpby(int64_t n, double2 a, const double2* x, double2 b, const double2* y, double2* z, hipStream_t st,
                  int R, int64_t ldx, int64_t ldy, int64_t ldz) {
  if (R <= 0 || n <= 0) return;
  hipLaunchKernelGGL(dev::k_axpby, dim3(unsigned((n + 255) / 256), unsigned(R)), dim3(256), 0, st, n, a, x, b, y, z,
                     ldx, ldy, ldz);
  BEM_HIP(hipGetLastError());
}

void launch_diag(const double2* A, int64_t ld, int64_t n, double2* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_diag, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, A, ld, n, out);
  BEM_HIP(hipGetLastError());
}

void launch_cast_f32(const double2* src, int64_t rows, int64_t cols, int64_t lds, float2* dst, int64_t ldd,
                     hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(dev::k_cast_f32, dim3(unsigned((ldd + 255) / 256), unsigned(rows)), dim3(256), 0, st, src, rows,
                     cols, lds, dst, ldd);
  BEM_HIP(hipGetLastError());
}

void launch_cast_f64(const float2* src, int64_t rows, int64_t cols, int64_t lds, double2* dst, int64_t ldd,
                     hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
    const int64_t nr = std::min<int64_t>(65535, rows - r0);
    hipLaunchKernelGGL(dev::k_cast_f64, dim3(unsigned((cols + 255) / 256), unsigned(nr)), dim3(256), 0, st,
                       src + r0 * lds, nr, cols, lds, dst + r0 * ldd, ldd);
    BEM_HIP(hipGetLastError());
  }
}

void launch_mdot(const double2* V, int64_t ldv, int j, const double2* w, int64_t n, double2* h,
                 const KrylovScratch&, hipStream_t st) {
  if (j <= 0) return;
  hipLaunchKernelGGL(dev::k_mdot, dim3(unsigned(j)), dim3(256), 0, st, V, ldv, w, n, h);
  BEM_HIP(hipGetLastError());
}

void launch_mupdate(const double2* V, int64_t ldv, int j, const double2* h, double sign, double2* w, int64_t n,
                    hipStream_t st) {
  if (j <= 0) return;
  hipLaunchKernelGGL(dev::k_mupdate, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, V, ldv, j, h, sign, w, n);
  BEM_HIP(hipGetLastError());
}

void launch_norm(const double2* w, int64_t n, double2* out, const KrylovScratch& ks, hipStream_t st) {
  double* part = reinterpret_cast<double*>(ks.partial);
  hipLaunchKernelGGL(dev::k_norm_partial, dim3(dev::kNormBlocks), dim3(256), 0, st, w, n, part);
  BEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(dev::k_norm_final, dim3(1), dim3(64), 0, st, part, dev::kNormBlocks, out);
  BEM_HIP(hipGetLastError());
}

void launch_scale_inv(const double2* w, int64_t n, const double2* nrm, double2* v, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_scale_inv, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, w, n, nrm, v);
  BEM_HIP(hipGetLastError());
}

void launch_givens(double2* Hcol, int j, double2* cs, double2* sn, double2* g, double* res, const double2* h2,
                   hipStream_t st) {
  hipLaunchKernelGGL(dev::k_givens, dim3(1), dim3(64), 0, st, Hcol, j, cs, sn, g, res, h2);
  BEM_HIP(hipGetLastError());
}

void launch_backsolve(const double2* H, int64_t ldh, int j, double2* g, double2* y, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_backsolve, dim3(1), dim3(64), 0, st, H, ldh, j, g, y);
  BEM_HIP(hipGetLastError());
}

void launch_init_g(double2* g, int mmax, const double2* beta, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_init_g, dim3(unsigned((mmax + 1 + 255) / 256)), dim3(256), 0, st, g, mmax, beta);
  BEM_HIP(hipGetLastError());
}

// ---- batched Krylov launchers

int bkry_chunks(int64_t n) { return int((std::max<int64_t>(n, 1) + dev::kChunk - 1) / dev::kChunk); }

void launch_bmdot(const double2* V, int64_t ldv, int R, int j1, const double2* W, int64_t ldw, int64_t n,
                  double2* part, double2* h, int64_t hstride, hipStream_t st) {
  if (R <= 0 || j1 <= 0) return;
  const int nch = bkry_chunks(n);
  if (int64_t(nch) * R >= 1024)
    hipLaunchKernelGGL(dev::k_bmdot_part, dim3(unsigned(nch), unsigned(R)), dim3(256), 0, st, V, ldv, R, j1, W, ldw,
                       n, nch, part);
  else
    hipLaunchKernelGGL(dev::k_bmdot_part3, dim3(unsigned(nch), unsigned(j1), unsigned(R)), dim3(256), 0, st, V, ldv,
                       R, j1, W, ldw, n, nch, part);
  BEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(dev::k_bmdot_final, dim3(unsigned(R)), dim3(64), 0, st, part, nch, j1, h, hstride);
  BEM_HIP(hipGetLastError());
}

void launch_bdcgs2(double2* V, int64_t ldv, int R, int j, double2* Y, int64_t ldy, int64_t n, double2* part1,
                   double2* part2, double2* H, int64_t hs, int64_t ldh, double2* coef, int64_t cstride, double* rinv,
                   const int* frozen, bool update, hipStream_t st) {
  if (R <= 0 || n <= 0) return;
  const int nch = bkry_chunks(n), j1 = j + 1;
  const double2* X = V + int64_t(j) * R * ldv;
  // basis vectors per block: enough blocks (about 2048) to fill the device, few re-reads of X, Y
  const int64_t want = std::max<int64_t>(1, (2048 + int64_t(nch) * R - 1) / (int64_t(nch) * R));
  const int G = int((j1 + std::min<int64_t>(want, j1) - 1) / std::min<int64_t>(want, j1));
  const int ng = (j1 + G - 1) / G;
  hipLaunchKernelGGL(dev::k_bmdot2_part, dim3(unsigned(nch), unsigned(R), unsigned(ng)), dim3(256), 0, st, V, ldv, R,
                     j1, G, X, Y, ldy, n, nch, part1, part2);
  BEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(dev::k_bdcgs2_coef, dim3(unsigned(R)), dim3(dev::kCoefThreads), 0, st, part1, part2, nch, j, H,
                     hs, ldh, coef, cstride, rinv, frozen);
  BEM_HIP(hipGetLastError());
  if (!update) return;
  hipLaunchKernelGGL(dev::k_bdcgs2_update, dim3(unsigned((n + 63) / 64), unsigned(R)), dim3(256), 0, st, V, ldv, R, j,
                     coef, cstride, rinv, Y, ldy, n);
  BEM_HIP(hipGetLastError());
}

void launch_bmupdate(const double2* V, int64_t ldv, int R, int j1, const int* jr, const double2* h, int64_t hstride,
                     double sign, double2* W, int64_t ldw, int64_t n, hipStream_t st) {
  if (R <= 0 || n <= 0 || (j1 <= 0 && !jr)) return;
  hipLaunchKernelGGL(dev::k_bmupdate, dim3(unsigned((n + 63) / 64), unsigned(R)), dim3(256), 0, st, V, ldv, R, j1,
                     jr, h, hstride, sign, W, ldw, n);
  BEM_HIP(hipGetLastError());
}

void launch_bnorm(const double2* W, int64_t ldw, int R, int64_t n, double2* part, double2* out, int64_t ostride,
                  hipStream_t st) {
  if (R <= 0) return;
  const int nch = bkry_chunks(n);
  double* p = reinterpret_cast<double*>(part);
  hipLaunchKernelGGL(dev::k_bnorm_part, dim3(unsigned(nch), unsigned(R)), dim3(256), 0, st, W, ldw, n, nch, p);
  BEM_HIP(hipGetLastError());
  hipLaunchKernelGGL(dev::k_bnorm_final, dim3(unsigned((R + 63) / 64)), dim3(64), 0, st, p, nch, R, out, ostride);
  BEM_HIP(hipGetLastError());
}

void launch_bscale_inv(double2* W, int64_t ldw, int R, int64_t n, const double2* nrm, int64_t nstride,
                       const int* frozen, hipStream_t st) {
  if (R <= 0 || n <= 0) return;
  hipLaunchKernelGGL(dev::k_bscale_inv, dim3(unsigned((n + 255) / 256), unsigned(R)), dim3(256), 0, st, W, ldw, n,
                     nrm, nstride, frozen);
  BEM_HIP(hipGetLastError());
}

void launch_bgivens(const double2* H, double2* HR, int64_t hs, int64_t ldh, int j, double2* cs, double2* sn,
                    double2* g, double* res, const double2* h2, int m, int R, hipStream_t st) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_bgivens, dim3(unsigned(R)), dim3(64), 0, st, H, HR, hs, ldh, j, cs, sn, g, res, h2, m,
                     R);
  BEM_HIP(hipGetLastError());
}

void launch_bbacksolve(const double2* H, int64_t hs, int64_t ldh, const int* jr, const double2* g, double2* y, int m,
                       int R, hipStream_t st) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_bbacksolve, dim3(unsigned((R + 63) / 64)), dim3(64), 0, st, H, hs, ldh, jr, g, y, m, R);
  BEM_HIP(hipGetLastError());
}

void launch_binit_g(double2* g, int m, const double2* beta, int64_t bstride, int R, hipStream_t st) {
  if (R <= 0) return;
  hipLaunchKernelGGL(dev::k_binit_g, dim3(unsigned(R)), dim3(64), 0, st, g, m, beta, bstride);
  BEM_HIP(hipGetLastError());
}

void launch_gather_cols(const double2* X, int64_t ldx, double2* U, int64_t ldu, const int* idx, int64_t n, int R,
                        hipStream_t st) {
  if (R <= 0 || n <= 0) return;
  hipLaunchKernelGGL(dev::k_gather_cols, dim3(unsigned((n + 255) / 256), unsigned(R)), dim3(256), 0, st, X, ldx, U,
                     ldu, idx, n);
  BEM_HIP(hipGetLastError());
}

void launch_scatter_cols(const double2* U, int64_t ldu, double2* X, int64_t ldx, const int* idx, int64_t n, int R,
                         int accumulate, hipStream_t st) {
  if (R <= 0 || n <= 0) return;
  hipLaunchKernelGGL(dev::k_scatter_cols, dim3(unsigned((n + 255) / 256), unsigned(R)), dim3(256), 0, st, U, ldu, X,
                     ldx, idx, n, accumulate);
  BEM_HIP(hipGetLastError());
}

}  // namespace bem
