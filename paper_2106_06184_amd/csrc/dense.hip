// Dense complex float64 inversion on the device (blocked Gauss-Jordan without pivoting) and the
// builders of the dense matrices it is applied to: the equivalent-configuration matrix M_eq of
// eq. AEFIEeqvdis (direct inner solve, the paper's route for small objects) and the charge Schur
// complements of the block preconditioners (eq. pcext for the final system, and its
// equivalent-configuration counterpart for the nested iterative solve).
//
// Gauss-Jordan step on the diagonal block kb (width b <= 64):
//   P = A_kb,kb^-1 ;  R = P A_kb,j (j outside kb) ;  C = A_i,kb (i outside kb)
//   A_i,j -= C_i R_j ;  A_kb,j = R_j ;  A_i,kb = -C_i P ;  A_kb,kb = P
// The update is a rank-b complex product over the whole matrix (64 x 64 output tiles per
// workgroup, K staged through LDS in chunks of 16, three real products per complex one).  Without pivoting the elimination needs
// non-singular leading blocks; for the matrices it is used on (near-field dominated BEM blocks
// and their charge Schur complements) this holds and round-off growth stays small.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "dense.h"
#include "prof.h"

namespace bem {

namespace dev {

constexpr int NB = 64;
constexpr int GMAX = 4;         // most panels applied by one pass
constexpr int LDC = GMAX * NB;  // row stride of the column panels C (panels side by side)

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cinv(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// In-place inversion of the b x b diagonal block, copied to P (ld NB).  Thread t keeps the
// S x S sub-block (rows S (t / (NB/S)) + [0, S), columns S (t % (NB/S)) + [0, S)) of the block in
// registers; at pivot p the owners of row p and of column p publish them in LDS (double-buffered
// by the parity of p, so one barrier per pivot suffices) and every thread updates its entries:
//   M[p][p] <- 1/a,  M[p][c] <- M[p][c]/a,  M[r][p] <- -M[r][p]/a,
//   M[r][c] <- M[r][c] - M[r][p] M[p][c]/a      (a = M[p][p] before the step).
// Entries outside the b x b block are identity (so padded pivots are 1).  The pivots form a
// serial chain, so the sub-blocks are small (S = 2: 1024 threads) to keep each step short.
constexpr int kDiagS = 2;
constexpr int kDiagThreads = (NB / kDiagS) * (NB / kDiagS);
//
// Breakdown watch (no pivoting is done): the smallest |pivot| of the block relative to the
// largest |entry| of the block as it arrives is folded into health[0] (a running minimum over
// the launches of one inversion, NaN once any ratio is not finite).  Launches of one inversion
// run in stream order, so thread 0 updates it without atomics.
__global__ void __launch_bounds__(kDiagThreads) k_gj_diag(double2* __restrict__ A, int64_t ld, int64_t k0, int b,
                                                          double2* __restrict__ P, double* __restrict__ health) {
  constexpr int S = kDiagS, W = NB / S;
  __shared__ double2 rowp[2][NB], colp[2][NB];
  __shared__ double red[kDiagThreads / 64];
  const int t = threadIdx.x;
  const int r0 = S * (t / W), c0 = S * (t % W);
  double2 m[S][S];
  double amax = 0.0;
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int r = r0 + i, c = c0 + j;
      m[i][j] = (r < b && c < b) ? A[(k0 + r) * ld + k0 + c] : make_double2(r == c ? 1.0 : 0.0, 0.0);
      if (r < b && c < b) amax = fmax(amax, sqrt(m[i][j].x * m[i][j].x + m[i][j].y * m[i][j].y));
    }
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  if ((t & 63) == 0) red[t >> 6] = amax;
  __syncthreads();
  double bmax = red[0];
  for (int w = 1; w < kDiagThreads / 64; ++w) bmax = fmax(bmax, red[w]);
  double min_ratio = HUGE_VAL;
  bool bad = false;
  for (int p = 0; p < NB; ++p) {
    const int buf = p & 1;
    const int pl = p % S;
    // (register arrays are indexed with compile-time constants only, so they stay in VGPRs)
    if (p / S == r0 / S) {
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (i == pl) {
#pragma unroll
          for (int j = 0; j < S; ++j) rowp[buf][c0 + j] = m[i][j];
        }
    }
    if (p / S == c0 / S) {
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (j == pl) {
#pragma unroll
          for (int i = 0; i < S; ++i) colp[buf][r0 + i] = m[i][j];
        }
    }
    __syncthreads();
    if (t == 0 && p < b) {
      const double2 a = rowp[buf][p];
      const double ratio = sqrt(a.x * a.x + a.y * a.y) / bmax;
      if (!isfinite(ratio)) bad = true;
      else min_ratio = fmin(min_ratio, ratio);
    }
    const double2 inv = cinv(rowp[buf][p]);
    double2 g[S], cr[S];
#pragma unroll
    for (int j = 0; j < S; ++j) g[j] = cm(rowp[buf][c0 + j], inv);
#pragma unroll
    for (int i = 0; i < S; ++i) cr[i] = colp[buf][r0 + i];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        m[i][j].x -= cr[i].x * g[j].x - cr[i].y * g[j].y;
        m[i][j].y -= cr[i].x * g[j].y + cr[i].y * g[j].x;
      }
    // pivot row and column: M[p][c] = g[c], M[r][p] = -M[r][p] / a (old M[r][p] = colp), M[p][p] = 1/a
    if (p / S == c0 / S) {
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (j == pl) {
#pragma unroll
          for (int i = 0; i < S; ++i) {
            const double2 v = cm(cr[i], inv);
            m[i][j] = make_double2(-v.x, -v.y);
          }
        }
    }
    if (p / S == r0 / S) {
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (i == pl) {
#pragma unroll
          for (int j = 0; j < S; ++j) m[i][j] = (c0 + j == p) ? inv : g[j];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) P[(r0 + i) * NB + c0 + j] = m[i][j];
  if (t == 0) {
    const double h = health[0];
    health[0] = (bad || isnan(h)) ? __builtin_nan("") : fmin(h, min_ratio);
  }
}

// Probe of an inversion: x_j = (1 + (j mod 7) / 7) e^{0.7 j i} (a fixed, full vector).  Before the
// inversion y = A x; after it z = A^-1 y and d_i = |z_i - x_i|^2.  One wave per row, lanes along
// the row, a fixed-order butterfly.  health[0] is reset to +inf before the inversion.
__device__ __forceinline__ double2 probe_x(int64_t j) {
  double s, c;
  sincos(0.7 * double(j), &s, &c);
  const double a = 1.0 + double(j % 7) / 7.0;
  return make_double2(a * c, a * s);
}
__global__ void __launch_bounds__(256) k_probe_mv(const double2* __restrict__ A, int64_t ld, int64_t n,
                                                  double2* __restrict__ y, double* __restrict__ d, int after,
                                                  double* __restrict__ health) {
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i == 0 && threadIdx.x == 0 && !after) health[0] = HUGE_VAL;
  if (i >= n) return;
  const double2* row = A + i * ld;
  double sr = 0.0, si = 0.0;
  for (int64_t j = lane; j < n; j += 64) {
    const double2 a = row[j];
    const double2 v = after ? y[j] : probe_x(j);
    sr += a.x * v.x - a.y * v.y;
    si += a.x * v.y + a.y * v.x;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sr += __shfl_xor(sr, off);
    si += __shfl_xor(si, off);
  }
  if (lane != 0) return;
  if (!after) {
    y[i] = make_double2(sr, si);
  } else {
    const double2 x = probe_x(i);
    d[i] = (sr - x.x) * (sr - x.x) + (si - x.y) * (si - x.y);
  }
}
// health[1] = sqrt(sum d / sum |x|^2), one block, fixed order.  The probe's y is read by the
// rows of the second product while they write d, so d has its own storage.
__global__ void __launch_bounds__(256) k_probe_reduce(const double* __restrict__ d, int64_t n,
                                                      double* __restrict__ health) {
  __shared__ double num[256], den[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double2 x = probe_x(i);
    a += d[i];
    b += x.x * x.x + x.y * x.y;
  }
  num[threadIdx.x] = a;
  den[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      num[threadIdx.x] += num[threadIdx.x + h];
      den[threadIdx.x] += den[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) health[1] = sqrt(num[0] / den[0]);
}

// R[s][j] = sum_t P[s][t] A[k0+t][j] for all j (thread: one column, 8 values of s; 32 columns
// per block so that even n = 2048 gives 64 blocks); C[i][s] = A[i][k0+s] for all i (copied
// before the update overwrites them).
__global__ void __launch_bounds__(256) k_gj_panels(const double2* __restrict__ A, int64_t ld, int64_t n, int64_t k0,
                                                   int b, const double2* __restrict__ P, double2* __restrict__ R,
                                                   double2* __restrict__ Cp) {
  __shared__ double2 Ps[NB][NB + 1];
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) Ps[e / NB][e % NB] = P[e];
  __syncthreads();
  const int64_t j = int64_t(blockIdx.x) * 32 + (threadIdx.x & 31);
  const int sg = threadIdx.x >> 5;  // s in [8 sg, 8 sg + 8)
  if (j < n) {
    double2 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = make_double2(0, 0);
#pragma unroll 4
    for (int t = 0; t < b; ++t) {
      const double2 a = A[(k0 + t) * ld + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 p = Ps[8 * sg + u][t];
        acc[u].x += p.x * a.x - p.y * a.y;
        acc[u].y += p.x * a.y + p.y * a.x;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (8 * sg + u < b) R[(8 * sg + u) * n + j] = acc[u];
  }
  // column panel: rows i of the kb columns (coalesced along s)
  for (int64_t e = int64_t(blockIdx.x) * 32 * NB + threadIdx.x; e < (int64_t(blockIdx.x) + 1) * 32 * NB;
       e += blockDim.x) {
    const int64_t i = e / NB;
    const int s = int(e % NB);
    if (i < n && s < b) Cp[i * LDC + s] = A[i * ld + k0 + s];
  }
}

// The 64 x 64 tile (ti, tj) of an update launch.  Mode 0 covers the matrix, gridDim.y x
// gridDim.x tiles, in an XCD-aware order: the 8 XCDs take consecutive blocks round-robin; each
// XCD gets a band of nby/8 row tiles, cut into balanced sub-bands of at most 10 row tiles, and
// walks one sub-band after the other column tile by column tile (rows fastest), so the
// sub-band's rows of the column panels C (at most 10 x 64 rows x 4 panels x 1 KiB = 2.5 MB) and
// the few R columns in flight stay in its L2 (4 MB).  Mode 3 is the strip pair of tile fix: the
// column of tiles tj = fix and the row of tiles ti = fix (without the tile the column has).
__device__ __forceinline__ void update_tile(int mode, int fix, unsigned& ti, unsigned& tj) {
  if (mode == 3) {
    // both strips of tile row / column fix: blocks [0, nt) the column strip (every tile row),
    // blocks [nt, 2 nt - 1) the row strip (every tile column but fix); disjoint tiles
    const unsigned nt = (gridDim.x + 1) / 2;
    if (blockIdx.x < nt) {
      ti = blockIdx.x;
      tj = unsigned(fix);
    } else {
      const unsigned b = blockIdx.x - nt;
      ti = unsigned(fix);
      tj = b + (b >= unsigned(fix) ? 1u : 0u);
    }
    return;
  }
  const unsigned nbx = gridDim.x, nby = gridDim.y;
  const unsigned lin = blockIdx.y * nbx + blockIdx.x;
  ti = lin / nbx;
  tj = lin % nbx;
  if (nby % 8 == 0) {
    const unsigned band = nby / 8, l = lin / 8;
    const unsigned nsb = (band + 9) / 10, sb = (band + nsb - 1) / nsb;  // sub-bands, their height
    const unsigned sub = l / (sb * nbx);                                 // full sub-bands before
    const unsigned h = min(sb, band - sub * sb);                         // this sub-band's height
    const unsigned r = l - sub * sb * nbx;
    ti = (lin % 8) * band + sub * sb + r % h;
    tj = r / h;
  }
}

// A[i][j] -= sum_s C[i][s] R[s][j] over the tiles of the launch (C: ld LDC, R: ld n) on the
// float64 matrix cores.  Whole tiles are updated: rows and columns of the pivot blocks are
// overwritten afterwards, and where a tile holds an earlier pivot block's rows or columns, that
// panel's C rows and R columns there are zero.  3M form (Gauss's trick, three real products per
// complex product): with c = cr + j ci and r = rr + j ri,
//   P1 = cr rr,  P2 = ci ri,  P3 = (cr + ci)(rr + ri);   Re(c r) = P1 - P2,  Im(c r) = P3 - P1 - P2,
// each summed over the panel columns on the float64 4x4x4 four-block instruction (alone, on
// gfx950, about 1.45x the float64 16x16x4 one): 6 real flops per complex multiply-add where the
// real embedding of the complex product takes 8.  Tile 64 x 64 complex, four waves of 32 x 32
// complex; C and R staged through LDS as complex pairs, 16 panel columns at a time.  Lane l of
// instruction (bi, g) supplies C[4 bi + l % 4][l / 16] (the four blocks share the rows) and
// R[l / 16][16 g + l % 16] and receives row 4 bi + l / 16, column 16 g + l % 16 of the wave tile:
// each lane holds P1, P2 and P3 of whole complex outputs and updates them itself.  The tile's
// old values are read after the products (the registers go to the three accumulators).
__global__ void __launch_bounds__(256, 2) k_gj_update_3m(double2* __restrict__ A, int64_t ld, int64_t n, int mode,
                                                      int fix, int b, const double2* __restrict__ R,
                                                      const double2* __restrict__ Cp) {
  constexpr int KCC = 16;  // complex panel columns per stage
  __shared__ double2 Cs[KCC][64 + 1];
  __shared__ double2 Rs[KCC][64 + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  unsigned ti, tj;
  update_tile(mode, fix, ti, tj);
  const int64_t i0 = int64_t(ti) * 64, j0 = int64_t(tj) * 64;
  const int sr = tid & 63, sg = (tid >> 6) * 4;
  double2 pc[4], pr[4];
  auto fetch = [&](int s0) {
    const int64_t gi = i0 + sr, gj = j0 + sr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int sc = s0 + sg + e;
      pc[e] = (gi < n && sc < b) ? Cp[gi * LDC + sc] : make_double2(0, 0);
      pr[e] = (gj < n && sc < b) ? R[int64_t(sc) * n + gj] : make_double2(0, 0);
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Cs[sg + e][sr] = pc[e];
      Rs[sg + e][sr] = pr[e];
    }
  };
  fetch(0);
  double p1[8][2], p2[8][2], p3[8][2];
#pragma unroll
  for (int bi = 0; bi < 8; ++bi)
#pragma unroll
    for (int g = 0; g < 2; ++g) p1[bi][g] = p2[bi][g] = p3[bi][g] = 0.0;
  const int ar_ = lane & 3, ak = lane >> 4, bc = lane & 15;
  for (int k0 = 0; k0 < b; k0 += KCC) {
    stage();
    __syncthreads();
    if (k0 + KCC < b) fetch(k0 + KCC);  // next stage streams in during the MFMAs
#pragma unroll
    for (int kk = 0; kk < KCC; kk += 4) {
      double cr[8], ci[8], rr[2], ri[2];
#pragma unroll
      for (int bi = 0; bi < 8; ++bi) {
        const double2 u = Cs[kk + ak][wm * 32 + 4 * bi + ar_];
        cr[bi] = u.x;
        ci[bi] = u.y;
      }
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const double2 u = Rs[kk + ak][wn * 32 + 16 * g + bc];
        rr[g] = u.x;
        ri[g] = u.y;
      }
#pragma unroll
      for (int bi = 0; bi < 8; ++bi)
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          p1[bi][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(cr[bi], rr[g], p1[bi][g], 0, 0, 0);
          p2[bi][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ci[bi], ri[g], p2[bi][g], 0, 0, 0);
          p3[bi][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(cr[bi] + ci[bi], rr[g] + ri[g], p3[bi][g], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  double* Ad = reinterpret_cast<double*>(A);
#pragma unroll
  for (int bi = 0; bi < 8; ++bi)
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int64_t gi = i0 + wm * 32 + 4 * bi + (lane >> 4);
      const int64_t gj = j0 + wn * 32 + 16 * g + (lane & 15);
      if (gi < n && gj < n) {
        // (read once and written once per pass: non-temporal, so that the panels keep the L2)
        double* a = Ad + 2 * (gi * ld + gj);
        const double re = p1[bi][g] - p2[bi][g], im = (p3[bi][g] - p1[bi][g]) - p2[bi][g];
        const double ox = __builtin_nontemporal_load(a), oy = __builtin_nontemporal_load(a + 1);
        __builtin_nontemporal_store(ox - re, a);
        __builtin_nontemporal_store(oy - im, a + 1);
      }
    }
}

// A[k0+s][j] = R[s][j] (j outside kb); A[i][k0+s] = -sum_t C[i][t] P[t][s] (i outside kb);
// A[kb][kb] = P.  A block takes 16 consecutive indices r: rows i = r of the pivot columns (a wave
// per row, lanes along s, C rows staged in LDS) and columns j = r of the pivot rows (16
// consecutive j per s, so the row-block copy moves 256-byte segments).
// Panel m of the group: R and Cp are the group's panel bases (panel q at R + q NB n and
// Cp + q NB).  The entries of panels 0..m in the pivot block's own rows and columns (R[q][s][i],
// C[i][q][s], i inside kb: read by no thread of the launch) are zeroed, so that the group's
// pass, which applies all its panels at once, leaves the rows and columns just written as they
// are.
__global__ void __launch_bounds__(256) k_gj_write(double2* __restrict__ A, int64_t ld, int64_t n, int64_t k0, int b,
                                                  const double2* __restrict__ P, double2* __restrict__ R,
                                                  double2* __restrict__ Cp, int m) {
  __shared__ double2 Ps[NB][NB];
  __shared__ double2 Cs[16][NB];
  const int64_t r0 = int64_t(blockIdx.x) * 16;
  const double2* Rm = R + int64_t(m) * NB * n;
  const double2* Cm = Cp + m * NB;
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) Ps[e / NB][e % NB] = P[e];
  for (int e = threadIdx.x; e < 16 * NB; e += blockDim.x) {
    const int64_t i = r0 + e / NB;
    const int t = e % NB;
    const bool out = i < n && t < b && !(i >= k0 && i < k0 + b);
    Cs[e / NB][t] = out ? Cm[i * LDC + t] : make_double2(0, 0);
  }
  __syncthreads();
  const int s = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r = w; r < 16; r += 4) {
    const int64_t i = r0 + r;
    if (i >= n || s >= b) continue;
    if (i >= k0 && i < k0 + b) {
      A[i * ld + k0 + s] = Ps[i - k0][s];
      for (int q = 0; q <= m; ++q) {
        R[int64_t(q * NB + s) * n + i] = make_double2(0, 0);
        Cp[i * LDC + q * NB + s] = make_double2(0, 0);
      }
      continue;
    }
    double2 acc = make_double2(0, 0);
    for (int t = 0; t < b; ++t) {
      const double2 c = Cs[r][t], p = Ps[t][s];
      acc.x += c.x * p.x - c.y * p.y;
      acc.y += c.x * p.y + c.y * p.x;
    }
    A[i * ld + k0 + s] = make_double2(-acc.x, -acc.y);
  }
  for (int e = threadIdx.x; e < 16 * NB; e += blockDim.x) {
    const int64_t j = r0 + e % 16;
    const int ss = e / 16;
    if (j >= n || ss >= b || (j >= k0 && j < k0 + b)) continue;
    A[(k0 + ss) * ld + j] = Rm[int64_t(ss) * n + j];
  }
}

// ------------------------------------------------------------- builders

// M_eq of one object (local indices): rows/cols [0, ne) edges, [ne, ne+nq) kept charges.
//  M[m][n]      = mu_l L^A[m][n]
//  M[m][ne+q]   = -eps_l^-1 ((L^phi B)[T+m][q] - (L^phi B)[T-m][q]),  (L^phi B)[t][q] = Lp[t][q] - Lp[t][last]
//  M[ne+q][n]   = (F D)[q][n] = +1 if T+(n) = q, -1 if T-(n) = q
//  M[ne+q][ne+q'] = -k0^2 delta
__global__ void k_build_meq(const double2* __restrict__ LA, int64_t lda, const double2* __restrict__ Lp, int64_t ldp,
                            const int32_t* __restrict__ tp, const int32_t* __restrict__ tm, int32_t toff, int64_t ne,
                            int64_t nt, double2 mu, double2 meps, double k02, double2* __restrict__ M, int64_t ldm) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  const int64_t nq = nt - 1, N = ne + nq;
  if (c >= N) return;
  double2 v = make_double2(0, 0);
  if (r < ne) {
    if (c < ne) {
      v = cm(mu, LA[r * lda + c]);
    } else {
      const int64_t q = c - ne, last = nt - 1;
      const int64_t tpr = tp[r] - toff, tmr = tm[r] - toff;
      const double2 a = Lp[tpr * ldp + q], b = Lp[tpr * ldp + last];
      const double2 d = Lp[tmr * ldp + q], e = Lp[tmr * ldp + last];
      const double2 diff = make_double2((a.x - b.x) - (d.x - e.x), (a.y - b.y) - (d.y - e.y));
      v = cm(meps, diff);
    }
  } else {
    const int64_t q = r - ne;
    if (c < ne) {
      if (tp[c] - toff == q) v.x += 1.0;
      if (tm[c] - toff == q) v.x -= 1.0;
    } else if (c - ne == q) {
      v.x = -k02;
    }
  }
  M[r * ldm + c] = v;
}

// Charge-eliminated equivalent-configuration matrix (eq. AEFIEeqvdis with w = k0^-2 F D u
// substituted): S = mu L^A_l + c D^T L^phi_l D, c = -1/(eps_l k0^2), object-local T+/T-.
__global__ void k_build_s(const double2* __restrict__ LA, int64_t lda, const double2* __restrict__ Lp, int64_t ldp,
                          const int32_t* __restrict__ tp, const int32_t* __restrict__ tm, int32_t toff, int64_t ne,
                          double2 mu, double2 c, double2* __restrict__ S, int64_t lds) {
  const int64_t col = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= ne) return;
  const int64_t cp = tp[col] - toff, cm_ = tm[col] - toff;
  for (int64_t r = blockIdx.y; r < ne; r += gridDim.y) {
    const double2* rp = Lp + int64_t(tp[r] - toff) * ldp;
    const double2* rm = Lp + int64_t(tm[r] - toff) * ldp;
    const double2 pp = rp[cp], pm = rp[cm_], mp = rm[cp], mm = rm[cm_];
    const double2 d = make_double2((pp.x - pm.x) - (mp.x - mm.x), (pp.y - pm.y) - (mp.y - mm.y));
    const double2 a = cm(mu, LA[r * lda + col]), b = cm(c, d);
    S[r * lds + col] = make_double2(a.x + b.x, a.y + b.y);
  }
}

// Dense charge Schur complement S = k0^2 s0 I + G_kept - g_last 1^T from a sparse G (CSR over
// kept charges, columns = triangles of the object) - see dense.h.
__global__ void k_build_schur(const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                              const double2* __restrict__ val, int64_t nq, int64_t last, double2 diag,
                              double2* __restrict__ S, int64_t lds) {
  const int64_t q = blockIdx.x;
  if (q >= nq) return;
  double2 gl = make_double2(0, 0);
  for (int64_t p = ptr[q]; p < ptr[q + 1]; ++p)
    if (idx[p] == last) gl = val[p];
  for (int64_t c = threadIdx.x; c < nq; c += blockDim.x)
    S[q * lds + c] = make_double2((c == q ? diag.x : 0.0) - gl.x, (c == q ? diag.y : 0.0) - gl.y);
  __syncthreads();
  if (threadIdx.x == 0)
    for (int64_t p = ptr[q]; p < ptr[q + 1]; ++p)
      if (idx[p] != last) {
        double2* s = S + q * lds + idx[p];
        *s = make_double2(s->x + val[p].x, s->y + val[p].y);
      }
}

// ------------------------------------------------------------- preconditioners

// Column r of the R-column batch: r-vectors (r1, r2, x1, x2) start at + r * ldr, temporaries
// (t, v) at + r * ldt.
__global__ void k_pc_stage1(const double2* __restrict__ W, const double2* __restrict__ r1, const double2* __restrict__ r2,
                            int64_t ne, double2* __restrict__ t, int64_t ldr, int64_t ldt) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ne) return;
  const int64_t cr = int64_t(blockIdx.y) * ldr, ct = int64_t(blockIdx.y) * ldt;
  const double2 a = cm(W[4 * n], r1[cr + n]), b = cm(W[4 * n + 1], r2[cr + n]);
  t[ct + n] = make_double2(a.x + b.x, a.y + b.y);
}

__global__ void k_pc_stage2(const double2* __restrict__ W, const double2* __restrict__ r1, const double2* __restrict__ r2,
                            const double2* __restrict__ v, const double2* __restrict__ lb, const double2* __restrict__ li,
                            double2 e_b, const double2* __restrict__ e_i, const int32_t* __restrict__ tp,
                            const int32_t* __restrict__ tm, int64_t ne, double2* __restrict__ x1,
                            double2* __restrict__ x2, int64_t ldr, int64_t ldt) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ne) return;
  const int64_t cr = int64_t(blockIdx.y) * ldr, ct = int64_t(blockIdx.y) * ldt;
  const int32_t p = tp[n], m = tm[n];
  const double2 vp = v[ct + p], vm = v[ct + m];
  const double2 db = make_double2(cm(lb[p], vp).x - cm(lb[m], vm).x, cm(lb[p], vp).y - cm(lb[m], vm).y);
  const double2 di = make_double2(cm(li[p], vp).x - cm(li[m], vm).x, cm(li[p], vp).y - cm(li[m], vm).y);
  const double2 sb = cm(e_b, db), si = cm(e_i[n], di);
  const double2 a = make_double2(r1[cr + n].x - sb.x, r1[cr + n].y - sb.y);
  const double2 b = make_double2(r2[cr + n].x - si.x, r2[cr + n].y - si.y);
  const double2 u1 = cm(W[4 * n], a), u2 = cm(W[4 * n + 1], b), u3 = cm(W[4 * n + 2], a), u4 = cm(W[4 * n + 3], b);
  x1[cr + n] = make_double2(u1.x + u2.x, u1.y + u2.y);
  x2[cr + n] = make_double2(u3.x + u4.x, u3.y + u4.y);
}

__global__ void k_peq_stage1(const double2* __restrict__ d, const double2* __restrict__ r1, int64_t ne,
                             double2* __restrict__ t, int64_t ldr, int64_t ldt) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ne) return;
  t[int64_t(blockIdx.y) * ldt + n] = cm(d[n], r1[int64_t(blockIdx.y) * ldr + n]);
}

__global__ void k_peq_stage2(const double2* __restrict__ d, const double2* __restrict__ t, const double2* __restrict__ v,
                             const double2* __restrict__ lb, double2 e, const int32_t* __restrict__ tp,
                             const int32_t* __restrict__ tm, int64_t ne, double2* __restrict__ x1, int64_t ldr,
                             int64_t ldt) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ne) return;
  const int64_t cr = int64_t(blockIdx.y) * ldr, ct = int64_t(blockIdx.y) * ldt;
  const int32_t p = tp[n], m = tm[n];
  const double2 a = cm(lb[p], v[ct + p]), b = cm(lb[m], v[ct + m]);
  const double2 s = cm(cm(d[n], e), make_double2(a.x - b.x, a.y - b.y));
  x1[cr + n] = make_double2(t[ct + n].x + s.x, t[ct + n].y + s.y);
}

}  // namespace dev

void launch_pc_stage1(const double2* W, const double2* r1, const double2* r2, int64_t ne, double2* t, hipStream_t st,
                      int R, int64_t ldr, int64_t ldt) {
  hipLaunchKernelGGL(dev::k_pc_stage1, dim3(unsigned((ne + 255) / 256), unsigned(R)), dim3(256), 0, st, W, r1, r2, ne,
                     t, ldr, ldt);
  BEM_HIP(hipGetLastError());
}

void launch_pc_stage2(const double2* W, const double2* r1, const double2* r2, const double2* v, const double2* lb,
                      const double2* li, double2 e_b, const double2* e_i, const int32_t* tp, const int32_t* tm,
                      int64_t ne, double2* x1, double2* x2, hipStream_t st, int R, int64_t ldr, int64_t ldt) {
  hipLaunchKernelGGL(dev::k_pc_stage2, dim3(unsigned((ne + 255) / 256), unsigned(R)), dim3(256), 0, st, W, r1, r2, v,
                     lb, li, e_b, e_i, tp, tm, ne, x1, x2, ldr, ldt);
  BEM_HIP(hipGetLastError());
}

void launch_peq_stage1(const double2* d, const double2* r1, int64_t ne, double2* t, hipStream_t st, int R,
                       int64_t ldr, int64_t ldt) {
  hipLaunchKernelGGL(dev::k_peq_stage1, dim3(unsigned((ne + 255) / 256), unsigned(R)), dim3(256), 0, st, d, r1, ne, t,
                     ldr, ldt);
  BEM_HIP(hipGetLastError());
}

void launch_peq_stage2(const double2* d, const double2* t, const double2* v, const double2* lb, double2 e,
                       const int32_t* tp, const int32_t* tm, int64_t ne, double2* x1, hipStream_t st, int R,
                       int64_t ldr, int64_t ldt) {
  hipLaunchKernelGGL(dev::k_peq_stage2, dim3(unsigned((ne + 255) / 256), unsigned(R)), dim3(256), 0, st, d, t, v, lb, e,
                     tp, tm, ne, x1, ldr, ldt);
  BEM_HIP(hipGetLastError());
}

// One update launch over the tiles of `mode` (see update_tile) with b panel columns.
static void launch_update(double2* A, int64_t ld, int64_t n, int mode, int fix, int b, const double2* R,
                          const double2* C, hipStream_t st) {
  const unsigned nt = unsigned((n + 63) / 64);
  const dim3 g = mode == 0 ? dim3(nt, nt) : dim3(2 * nt - 1);
  if (g.x == 0) return;
  const double ntile = double(g.x) * g.y, elems = ntile * 64.0 * 64.0;
  const double alg = std::min(elems, mode == 0 ? double(n) * n : 2.0 * 64.0 * n);
  ProfScope ps(st, KC_DENSE_INV, 32.0 * alg, 8.0 * b * alg);
  hipLaunchKernelGGL(dev::k_gj_update_3m, g, dim3(256), 0, st, A, ld, n, mode, fix, b, R, C);
  BEM_HIP(hipGetLastError());  // before the profiler's scope ends (it clears event-query status)
}

// Blocked Gauss-Jordan, panels of NB, applied in groups of G panels so that one pass over the
// matrix applies a whole group (rank G NB: 1/G of the matrix traffic per flop).  Within a group,
// before panel m's pivot block and panels are taken, only the row and column strips of its
// block are brought up to date with panels 0..m-1; panels before the last write their pivot
// rows and columns at once (zeroing the group's panel entries there).  The pass then gives
// every tile A - sum_q C_q R_q, and the last panel's rows and columns are written over it.
// Entry for entry this is G single-panel steps.
void dense_invert(double2* A, int64_t n, int64_t ld, DenseScratch& ws, hipStream_t st) {
  if (n <= 0) return;
  constexpr int G = dev::GMAX;
  const unsigned gp = unsigned((n + 31) / 32), gw = unsigned((n + 15) / 16), gr = unsigned((n + 3) / 4);
  hipLaunchKernelGGL(dev::k_probe_mv, dim3(gr), dim3(256), 0, st, A, ld, n, ws.probe_y, ws.probe_d, 0, ws.health);
  for (int64_t k0 = 0; k0 < n;) {
    const int npan = int(std::min<int64_t>(G, (n - k0 + dev::NB - 1) / dev::NB));
    int blast = 0;
    for (int mp = 0; mp < npan; ++mp) {
      const int64_t km = k0 + int64_t(mp) * dev::NB;
      const int bm = int(std::min<int64_t>(dev::NB, n - km));
      if (mp > 0) launch_update(A, ld, n, 3, int(km / 64), mp * dev::NB, ws.R, ws.C, st);
      double2* Rm = ws.R + int64_t(mp) * dev::NB * n;
      double2* Cm = ws.C + mp * dev::NB;
      hipLaunchKernelGGL(dev::k_gj_diag, dim3(1), dim3(dev::kDiagThreads), 0, st, A, ld, km, bm, ws.P, ws.health);
      hipLaunchKernelGGL(dev::k_gj_panels, dim3(gp), dim3(256), 0, st, A, ld, n, km, bm, ws.P, Rm, Cm);
      if (mp + 1 < npan)
        hipLaunchKernelGGL(dev::k_gj_write, dim3(gw), dim3(256), 0, st, A, ld, n, km, bm, ws.P, ws.R, ws.C, mp);
      blast = bm;
    }
    launch_update(A, ld, n, 0, 0, (npan - 1) * dev::NB + blast, ws.R, ws.C, st);
    const int64_t kl = k0 + int64_t(npan - 1) * dev::NB;
    hipLaunchKernelGGL(dev::k_gj_write, dim3(gw), dim3(256), 0, st, A, ld, n, kl, blast, ws.P, ws.R, ws.C, npan - 1);
    k0 += int64_t(npan) * dev::NB;
  }
  hipLaunchKernelGGL(dev::k_probe_mv, dim3(gr), dim3(256), 0, st, A, ld, n, ws.probe_y, ws.probe_d, 1, ws.health);
  hipLaunchKernelGGL(dev::k_probe_reduce, dim3(1), dim3(256), 0, st, ws.probe_d, n, ws.health);
  BEM_HIP(hipGetLastError());
}

// ---- inversion without allocation (for callers that cannot allocate device memory)
// A fixed workspace for matrices of up to kNoAllocMaxN rows, one copy per GPU (it lives as long as
// the process).  Host code never uses the array's name as an address: its device address is taken
// once per device by noalloc_scratch_init and kept in g_noalloc_ptr.
namespace dev {
static __device__ __align__(256) double2 scratch[64 * 64 + 514 * kNoAllocMaxN + 2];
}  // namespace dev
static_assert(sizeof(dev::scratch) >= sizeof(double2) * dense_scratch_elems(kNoAllocMaxN), "workspace layout");
static std::mutex g_noalloc_mu;
static double2* g_noalloc_ptr[kMaxDevices] = {};

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(BEM_E_DEVICE, "device index beyond the workspace table");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return;
  int cur = -1;
  BEM_HIP(hipGetDevice(&cur));
  if (cur != device) throw Error(BEM_E_DEVICE, "workspace set-up needs its device current");
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(dev::scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error(BEM_E_DEVICE, std::string("address of the inversion workspace: ") + hipGetErrorString(e));
  }
  g_noalloc_ptr[device] = static_cast<double2*>(p);
}

void dense_invert_noalloc(int device, double2* A, int64_t n, int64_t ld, DenseHealth* health, hipStream_t st) {
  if (n > kNoAllocMaxN)
    throw Error(BEM_E_INVALID, "n = " + std::to_string(n) + " exceeds the " + std::to_string(kNoAllocMaxN) +
                                   "-row limit of the inversion without allocation");
  double2* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    base = (device >= 0 && device < kMaxDevices) ? g_noalloc_ptr[device] : nullptr;
  }
  if (!base) throw Error(BEM_E_DEVICE, "inversion workspace not set up on this device");
  DenseScratch ws = dense_scratch_at(base, n);
  dense_invert(A, n, ld, ws, st);
  *health = dense_health(ws, st);
}

DenseHealth dense_health(const DenseScratch& ws, hipStream_t st) {
  double h[2] = {0.0, 0.0};
  BEM_HIP(hipMemcpyAsync(h, ws.health, sizeof(h), hipMemcpyDeviceToHost, st));
  BEM_HIP(hipStreamSynchronize(st));
  return DenseHealth{h[0], h[1]};
}

bool dense_health_ok(const DenseHealth& h) {
  return h.min_pivot_ratio >= kMinPivotRatio && h.probe_error <= kMaxProbeError;
}

namespace dev {
__global__ void k_scale_rc(double2* __restrict__ A, int64_t ld, int64_t nr, int64_t nc, const double* __restrict__ rs,
                           const double* __restrict__ cs) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  const double c = cs[j];
  for (int64_t i = blockIdx.y; i < nr; i += gridDim.y) {
    const double s = rs[i] * c;
    double2 v = A[i * ld + j];
    A[i * ld + j] = make_double2(s * v.x, s * v.y);
  }
}
__global__ void k_col_maxabs(const double2* __restrict__ A, int64_t ld, int64_t r0, int64_t r1, int64_t c0,
                             int64_t nc, double* __restrict__ out) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  double m = 0;
  for (int64_t i = r0; i < r1; ++i) {
    const double2 v = A[i * ld + c0 + j];
    m = fmax(m, sqrt(v.x * v.x + v.y * v.y));
  }
  out[j] = m;
}
// one wave per row, fixed-order butterfly reduction
__global__ void __launch_bounds__(256) k_row_maxabs(const double2* __restrict__ A, int64_t ld, int64_t r0, int64_t nr,
                                                    int64_t nc, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nr) return;
  const double2* row = A + (r0 + i) * ld;
  double m = 0;
  for (int64_t j = lane; j < nc; j += 64) m = fmax(m, sqrt(row[j].x * row[j].x + row[j].y * row[j].y));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if (lane == 0) out[i] = m;
}
}  // namespace dev

namespace dev {
__global__ void k_fill_vec(double* v, int64_t n, double val) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = val;
}
__global__ void k_jacobi_vec(const double2* __restrict__ A, int64_t ld, int64_t i0, int64_t i1, double* v) {
  const int64_t i = i0 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= i1) return;
  const double2 d = A[i * ld + i];
  const double s = 1.0 / sqrt(sqrt(d.x * d.x + d.y * d.y));
  v[i] = isfinite(s) && s > 0 ? s : 1.0;
}
__global__ void k_recip_vec(const double* __restrict__ in, int64_t n, double* out1, double* out2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = 1.0 / in[i];
  const double r = isfinite(s) && s > 0 ? s : 1.0;
  out1[i] = r;
  out2[i] = r;
}
}  // namespace dev

void fill_vec(double* v, int64_t n, double val, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_fill_vec, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, v, n, val);
  BEM_HIP(hipGetLastError());
}

void jacobi_vec(const double2* A, int64_t ld, int64_t i0, int64_t i1, double* v, hipStream_t st) {
  if (i1 <= i0) return;
  hipLaunchKernelGGL(dev::k_jacobi_vec, dim3(unsigned((i1 - i0 + 255) / 256)), dim3(256), 0, st, A, ld, i0, i1, v);
  BEM_HIP(hipGetLastError());
}

void recip_vec(const double* in, int64_t n, double* out1, double* out2, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(dev::k_recip_vec, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, in, n, out1, out2);
  BEM_HIP(hipGetLastError());
}

void scale_rows_cols(double2* A, int64_t ld, int64_t nr, int64_t nc, const double* rs, const double* cs,
                     hipStream_t st) {
  if (nr <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(dev::k_scale_rc, dim3(unsigned((nc + 255) / 256), unsigned(std::min<int64_t>(nr, 32768))),
                     dim3(256), 0, st, A, ld, nr, nc, rs, cs);
  BEM_HIP(hipGetLastError());
}

void col_maxabs(const double2* A, int64_t ld, int64_t r0, int64_t r1, int64_t c0, int64_t nc, double* out,
                hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(dev::k_col_maxabs, dim3(unsigned((nc + 255) / 256)), dim3(256), 0, st, A, ld, r0, r1, c0, nc,
                     out);
  BEM_HIP(hipGetLastError());
}

void row_maxabs(const double2* A, int64_t ld, int64_t r0, int64_t nr, int64_t nc, double* out, hipStream_t st) {
  if (nr <= 0) return;
  hipLaunchKernelGGL(dev::k_row_maxabs, dim3(unsigned((nr + 3) / 4)), dim3(256), 0, st, A, ld, r0, nr, nc, out);
  BEM_HIP(hipGetLastError());
}

void build_meq(const double2* LA, int64_t lda, const double2* Lp, int64_t ldp, const int32_t* tp, const int32_t* tm,
               int32_t toff, int64_t ne, int64_t nt, double2 mu, double2 meps, double k02, double2* M, int64_t ldm,
               hipStream_t st) {
  const int64_t N = ne + nt - 1;
  hipLaunchKernelGGL(dev::k_build_meq, dim3(unsigned((N + 255) / 256), unsigned(N)), dim3(256), 0, st, LA, lda, Lp, ldp,
                     tp, tm, toff, ne, nt, mu, meps, k02, M, ldm);
  BEM_HIP(hipGetLastError());
}

void build_s(const double2* LA, int64_t lda, const double2* Lp, int64_t ldp, const int32_t* tp, const int32_t* tm,
             int32_t toff, int64_t ne, double2 mu, double2 c, double2* S, int64_t lds, hipStream_t st) {
  if (ne <= 0) return;
  hipLaunchKernelGGL(dev::k_build_s, dim3(unsigned((ne + 255) / 256), unsigned(std::min<int64_t>(ne, 32768))),
                     dim3(256), 0, st, LA, lda, Lp, ldp, tp, tm, toff, ne, mu, c, S, lds);
  BEM_HIP(hipGetLastError());
}

void build_schur(const int64_t* ptr, const int32_t* idx, const double2* val, int64_t nq, int64_t last, double2 diag,
                 double2* S, int64_t lds, hipStream_t st) {
  hipLaunchKernelGGL(dev::k_build_schur, dim3(unsigned(nq)), dim3(256), 0, st, ptr, idx, val, nq, last, diag, S, lds);
  BEM_HIP(hipGetLastError());
}

}  // namespace bem
