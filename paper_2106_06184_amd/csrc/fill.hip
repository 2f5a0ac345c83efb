// Galerkin fill kernels (gfx950, float64 VALU): L^(A), L^(phi) on RWG/pulse bases and K~ on BC
// sources over the barycentric refinement (eqs. opLAhgf, opLphihgf, opKhgf, hgf).
//
// Work decomposition
//  * L: one thread per source triangle T', a wave-uniform loop over test triangles T.  The
//    thread accumulates 8 complex moments of the Q7 x Q7 product rule with positions taken
//    relative to each triangle's centroid (no cancellation between far and near scales):
//      I0 = sum w w G,  Id = sum w w G d_k,  Id' = sum w w G d'_l,  Idd' = sum w w G d_k.d'_l
//    and writes the 3x3 block of half-RWG interactions
//      H_ij = 1/4 [Idd' - p'_j.Id - p_i.Id' + (p_i.p'_j) I0]     (p relative to the centroids)
//    plus L^phi = I0.  A gather kernel then adds the four half blocks of every edge pair.
//  * K~: one thread per dual cell C(v) (source), a wave-uniform loop over test triangles.  For
//    every sub-triangle t of the cell the thread forms the inner Q3 moments of g_k relative to
//    v, contracts them over the Q7 outer rule into 10 complex moments, and applies them to the
//    linear restriction (alpha r' - beta)/(2A_t) of each BC function of the cell.  The result,
//    per test half-RWG and (cell, BC) column, is gathered into K~ (two cells per BC function).
//  * Near pairs (shared vertex or close centroids) are recomputed by separate kernels with
//    singularity extraction: closed-form static parts plus Q7 (L) / Q3 (K~) on the bounded
//    remainders; they overwrite the far-rule values.  K~ is zero for coplanar near pairs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "devmath.h"
#include "fill.h"
#include "prof.h"

namespace bem {
namespace dev {

// Q7 (Radon, degree 5) and Q3 (degree 2) weights; the points live in the geometry tables.
__constant__ double cW7[7];
__constant__ double cB7[7][3];
__constant__ double cB3[3][3];

// Level of the source-rule subdivision (same test as the host's subdiv_level_host).
__device__ __forceinline__ int subdiv_level(double kr, double h) {
  const double x = fabs(kr) * h;
  int L = 0;
  while (L < kSubdivMax && x / double(1 << L) > kSubdivKh) ++L;
  return L;
}

// Barycentric corners of piece j of the level-L 4-to-1 split of a triangle (base-4 digits of
// j from the first split on; children: (c0, m01, m20), (m01, c1, m12), (m20, m12, c2),
// (m01, m12, m20)).  Row i = corner i.
__device__ __forceinline__ void subdiv_corners(int L, int j, double c[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int m = 0; m < 3; ++m) c[i][m] = i == m ? 1.0 : 0.0;
  for (int lev = L - 1; lev >= 0; --lev) {
    const int d = (j >> (2 * lev)) & 3;
    double m01[3], m12[3], m20[3];
    for (int m = 0; m < 3; ++m) {
      m01[m] = 0.5 * (c[0][m] + c[1][m]);
      m12[m] = 0.5 * (c[1][m] + c[2][m]);
      m20[m] = 0.5 * (c[2][m] + c[0][m]);
    }
    for (int m = 0; m < 3; ++m) {
      const double a0 = c[0][m], a1 = c[1][m], a2 = c[2][m];
      if (d == 0) { c[0][m] = a0;      c[1][m] = m01[m]; c[2][m] = m20[m]; }
      else if (d == 1) { c[0][m] = m01[m]; c[1][m] = a1;      c[2][m] = m12[m]; }
      else if (d == 2) { c[0][m] = m20[m]; c[1][m] = m12[m]; c[2][m] = a2; }
      else { c[0][m] = m01[m]; c[1][m] = m12[m]; c[2][m] = m20[m]; }
    }
  }
}

// Point of barycentric coordinates (b . corners) on a triangle with vertex offsets P[3].
__device__ __forceinline__ v3 subdiv_point(const double c[3][3], const double b[3], const v3 P[3]) {
  double w[3];
  for (int m = 0; m < 3; ++m) w[m] = b[0] * c[0][m] + b[1] * c[1][m] + b[2] * c[2][m];
  return w[0] * P[0] + w[1] * P[1] + w[2] * P[2];
}

__device__ __forceinline__ double G(const double* geo, int64_t nt, int f, int64_t t) { return geo[f * nt + t]; }
__device__ __forceinline__ v3 G3(const double* geo, int64_t nt, int f, int64_t t) {
  return mk(geo[f * nt + t], geo[(f + 1) * nt + t], geo[(f + 2) * nt + t]);
}

// ------------------------------------------------------------------ L far
// SUB: the source rule is Q7 on each of the 4^L pieces of the source triangle's level-L split
// (weights 1/4^L), L from |Re k| and the source's longest edge; otherwise plain Q7.
template <bool LOSSY, bool SUB>
__global__ void __launch_bounds__(256) k_fill_L_far(FillLArgs a) {
  const int64_t sl = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // local source index
  if (sl >= a.ns) return;
  const int64_t s = a.s0 + sl;
  const double* geo = a.geo;
  const int64_t nt = a.nt_total;
  const v3 cs = G3(geo, nt, kGeoC, s);
  v3 dl[7];
#pragma unroll
  for (int l = 0; l < 7; ++l) dl[l] = G3(geo, nt, kGeoQ + 3 * l, s);
  v3 pj[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) pj[j] = G3(geo, nt, kGeoP + 3 * j, s);
  const int lev = SUB ? subdiv_level(a.kr, G(geo, nt, kGeoH, s)) : 0;
  const int npiece = 1 << (2 * lev);
  const double wpiece = 1.0 / double(npiece);
  const int64_t tbeg = int64_t(blockIdx.y) * a.tchunk;
  const int64_t tend = min(a.nt_test, tbeg + a.tchunk);
  for (int64_t tl = tbeg; tl < tend; ++tl) {
    const int64_t t = a.t0 + tl;
    const v3 d = G3(geo, nt, kGeoC, t) - cs;  // centroid offset test - source
    cz I0 = {0, 0}, Idd = {0, 0};
    cv3 Id = cvzero(), Idp = cvzero();
    for (int jp = 0; jp < npiece; ++jp) {
      if (SUB && lev > 0) {
        double c[3][3];
        subdiv_corners(lev, jp, c);
        for (int l = 0; l < 7; ++l) dl[l] = subdiv_point(c, cB7[l], pj);
      }
#pragma unroll 1
      for (int k = 0; k < 7; ++k) {
        const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
        const v3 base = d + dk;
        cz s0 = {0, 0};
        cv3 s1 = cvzero();
#pragma unroll
        for (int l = 0; l < 7; ++l) {
          v3 r = base - dl[l];
          double r2 = dot(r, r);
          double inv = rsqrt(r2);
          double R = r2 * inv;
          cz g = green<LOSSY>(a.kr, a.ki, R, inv);
          g = cscale(SUB ? cW7[l] * wpiece : cW7[l], g);
          s0 = cadd(s0, g);
          cv_axpy(s1, g, dl[l]);
        }
        const double wk = cW7[k];
        s0 = cscale(wk, s0);
        s1.x = cscale(wk, s1.x); s1.y = cscale(wk, s1.y); s1.z = cscale(wk, s1.z);
        I0 = cadd(I0, s0);
        cv_axpy(Id, s0, dk);
        cv_add(Idp, s1);
        Idd = cadd(Idd, cv_dot(dk, s1));
      }
    }
    // H_ij = 1/4 [Idd' - p'_j.Id - p_i.Id' + (p_i.p'_j) I0]
    double2* hrow = a.H + (3 * tl) * a.ldH + 3 * sl;
    for (int i = 0; i < 3; ++i) {
      const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);
      const cz pIdp = cv_dot(pi, Idp);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        cz h = csub(csub(Idd, cv_dot(pj[j], Id)), pIdp);
        h = cadd(h, cscale(dot(pi, pj[j]), I0));
        hrow[i * a.ldH + j] = make_double2(0.25 * h.re, 0.25 * h.im);
      }
    }
    a.Lphi[tl * a.ldP + sl] = make_double2(I0.re, I0.im);
  }
}

// ------------------------------------------------------------------ L near
template <bool LOSSY>
__global__ void __launch_bounds__(128) k_fill_L_near(FillLArgs a, const int32_t* pt, const int32_t* ps,
                                                     int64_t npairs) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int64_t t = pt[p], s = ps[p];
  const double* geo = a.geo;
  const int64_t nt = a.nt_total;
  const v3 ct = G3(geo, nt, kGeoC, t), cs = G3(geo, nt, kGeoC, s);
  const double As = G(geo, nt, kGeoA, s);
  // source vertices relative to the test centroid
  v3 sv[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) sv[j] = (cs - ct) + G3(geo, nt, kGeoP + 3 * j, s);
  // the remainder rule: Q7 on each piece of the source's level-L split (L = 0: plain Q7)
  const int lev = a.sub ? subdiv_level(a.kr, G(geo, nt, kGeoH, s)) : 0;
  const int npiece = 1 << (2 * lev);
  v3 pj[3];
  for (int j = 0; j < 3; ++j) pj[j] = G3(geo, nt, kGeoP + 3 * j, s);
  cz S0[7];
  cv3 S1[7];
  for (int k = 0; k < 7; ++k) {
    const v3 rk = G3(geo, nt, kGeoQ + 3 * k, t);  // relative to the test centroid
    StaticInts si = static_ints(rk, sv[0], sv[1], sv[2], false);
    cz s0 = {kInv4Pi * si.i1, 0.0};
    cv3 s1 = cvzero();
    s1.x.re = kInv4Pi * si.iv.x; s1.y.re = kInv4Pi * si.iv.y; s1.z.re = kInv4Pi * si.iv.z;
    if (lev == 0) {
      for (int l = 0; l < 7; ++l) {
        const v3 rl = (cs - ct) + G3(geo, nt, kGeoQ + 3 * l, s);
        const v3 dd = rl - rk;
        const double R = norm(dd);
        cz gr = cscale(cW7[l] * As, green_rem(a.kr, a.ki, R));
        s0 = cadd(s0, gr);
        cv_axpy(s1, gr, dd);
      }
    } else {
      const double wp = As / double(npiece);
      for (int jp = 0; jp < npiece; ++jp) {
        double c[3][3];
        subdiv_corners(lev, jp, c);
        for (int l = 0; l < 7; ++l) {
          const v3 rl = (cs - ct) + subdiv_point(c, cB7[l], pj);
          const v3 dd = rl - rk;
          const double R = norm(dd);
          cz gr = cscale(cW7[l] * wp, green_rem(a.kr, a.ki, R));
          s0 = cadd(s0, gr);
          cv_axpy(s1, gr, dd);
        }
      }
    }
    S0[k] = s0;
    S1[k] = s1;
  }
  double2* hrow = a.H + (3 * (t - a.t0)) * a.ldH + 3 * (s - a.s0);
  for (int i = 0; i < 3; ++i) {
    const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);
    for (int j = 0; j < 3; ++j) {
      cz acc = {0, 0};
      for (int k = 0; k < 7; ++k) {
        const v3 rk = G3(geo, nt, kGeoQ + 3 * k, t);
        // int G (r' - p'_j) dS' = S1 + (r - p'_j) S0
        cv3 in = S1[k];
        cv_axpy(in, S0[k], rk - sv[j]);
        acc = cadd(acc, cscale(cW7[k], cv_dot(rk - pi, in)));
      }
      const double sc = 0.25 / As;
      hrow[i * a.ldH + j] = make_double2(sc * acc.re, sc * acc.im);
    }
  }
  cz lp = {0, 0};
  for (int k = 0; k < 7; ++k) lp = cadd(lp, cscale(cW7[k], S0[k]));
  a.Lphi[(t - a.t0) * a.ldP + (s - a.s0)] = make_double2(lp.re / As, lp.im / As);
}

// ------------------------------------------------------------ gathers
// L^A: out[m][n] = sum_{a in {+,-}} sum_{b in {+,-}} s_a s_b H[row_a(m)][row_b(n)];
// K~: out[m][n] = sum_{a in {+,-}} s_a (Kc[row_a(m)][colS(n)] + Kc[row_a(m)][colT(n)]).
// Chunked gathers.  The half-row matrices hold the test half-RWGs [rlo, rhi) of one chunk of
// test triangles (row h - rlo).  For every listed edge row m with a half in the chunk: both halves
// there give the whole entry (the same sums as one pass over all rows); a half alone gives its
// part, which the first chunk (in chunk order) holding a half of m writes and the second adds.
// Two parts add exactly the same whichever comes first, so the result depends only on the
// chunk boundaries, which the caller fixes from the mesh.
__global__ void __launch_bounds__(256) k_gather_LA_rows(const double2* __restrict__ H, int64_t ldH,
                                                        const int32_t* __restrict__ hp, const int32_t* __restrict__ hm,
                                                        int64_t rlo, int64_t rhi, int64_t coff, int64_t ncol,
                                                        const int32_t* __restrict__ rows, int64_t nrows,
                                                        double2* __restrict__ out, int64_t ldo) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ncol) return;
  const int64_t cp = hp[n] - coff, cm = hm[n] - coff;
  for (int64_t r = blockIdx.y; r < nrows; r += gridDim.y) {
    const int64_t m = rows[r];
    const int64_t hpm = hp[m], hmm = hm[m];
    const bool inp = hpm >= rlo && hpm < rhi, inm = hmm >= rlo && hmm < rhi;
    double2* o = out + m * ldo + n;
    if (inp && inm) {
      const double2* rp = H + (hpm - rlo) * ldH;
      const double2* rm = H + (hmm - rlo) * ldH;
      const double2 a = rp[cp], b = rp[cm], c = rm[cp], d = rm[cm];
      *o = make_double2(a.x - b.x - c.x + d.x, a.y - b.y - c.y + d.y);
    } else if (inp) {
      const double2* rp = H + (hpm - rlo) * ldH;
      const double2 a = rp[cp], b = rp[cm];
      double2 v = make_double2(a.x - b.x, a.y - b.y);
      if (hmm < rlo) v = make_double2(o->x + v.x, o->y + v.y);
      *o = v;
    } else if (inm) {
      const double2* rm = H + (hmm - rlo) * ldH;
      const double2 c = rm[cp], d = rm[cm];
      double2 v = make_double2(d.x - c.x, d.y - c.y);
      if (hpm < rlo) v = make_double2(o->x + v.x, o->y + v.y);
      *o = v;
    }
  }
}

__global__ void __launch_bounds__(256) k_gather_K_rows(const double2* __restrict__ Kc, int64_t ldK,
                                                       const int32_t* __restrict__ hp, const int32_t* __restrict__ hm,
                                                       int64_t rlo, int64_t rhi, const int32_t* __restrict__ cS,
                                                       const int32_t* __restrict__ cT, int64_t ncol,
                                                       const int32_t* __restrict__ rows, int64_t nrows,
                                                       double2* __restrict__ out, int64_t ldo) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= ncol) return;
  const int32_t s = cS[n], u = cT[n];
  for (int64_t r = blockIdx.y; r < nrows; r += gridDim.y) {
    const int64_t m = rows[r];
    const int64_t hpm = hp[m], hmm = hm[m];
    const bool inp = hpm >= rlo && hpm < rhi, inm = hmm >= rlo && hmm < rhi;
    double2* o = out + m * ldo + n;
    if (inp && inm) {
      const double2* rp = Kc + (hpm - rlo) * ldK;
      const double2* rm = Kc + (hmm - rlo) * ldK;
      const double2 a = rp[s], b = rp[u], c = rm[s], d = rm[u];
      *o = make_double2(a.x + b.x - c.x - d.x, a.y + b.y - c.y - d.y);
    } else if (inp) {
      const double2* rp = Kc + (hpm - rlo) * ldK;
      const double2 a = rp[s], b = rp[u];
      double2 v = make_double2(a.x + b.x, a.y + b.y);
      if (hmm < rlo) v = make_double2(o->x + v.x, o->y + v.y);
      *o = v;
    } else if (inm) {
      const double2* rm = Kc + (hmm - rlo) * ldK;
      const double2 c = rm[s], d = rm[u];
      double2 v = make_double2(-(c.x + d.x), -(c.y + d.y));
      if (hpm < rlo) v = make_double2(o->x + v.x, o->y + v.y);
      *o = v;
    }
  }
}

// SUB: the inner rule of a sub-triangle is Q3 on each piece of its level-L split (L from |Re k|
// and the sub-triangle's longest edge); otherwise plain Q3.
// NACC <= MAXV: accumulators per thread, at least the largest valence of the launch's cells
// (MAXV is the padded layout of the cell tables; a smaller NACC frees registers).
template <bool LOSSY, int MAXV, bool SUB, int NACC>
__global__ void __launch_bounds__(128, 2) k_fill_K_far(FillKArgs a) {
  const int64_t cl = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cl >= a.ncells) return;
  const int32_t v = a.cells[cl];
  const int64_t nc = a.ncell_total;
  const double* geo = a.geo;
  const int64_t nt = a.nt_total;
  const int nval = a.nval[v];
  const v3 pv = mk(a.vpos[3 * v], a.vpos[3 * v + 1], a.vpos[3 * v + 2]);
  const int64_t col0 = a.col0[v];
  const int64_t tbeg = int64_t(blockIdx.y) * a.tchunk;
  const int64_t tend = min(a.nt_test, tbeg + a.tchunk);
  for (int64_t tl = tbeg; tl < tend; ++tl) {
    const int64_t t = a.t0 + tl;
    const v3 d = G3(geo, nt, kGeoC, t) - pv;
    cz acc[NACC][3];
#pragma unroll
    for (int b = 0; b < NACC; ++b)
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[b][i] = {0, 0};
    for (int sidx = 0; sidx < 2 * nval; ++sidx) {
      const size_t so = size_t(sidx) * nc + v;
      const v3 sm = mk(a.sub_m[3 * so], a.sub_m[3 * so + 1], a.sub_m[3 * so + 2]);
      const v3 sc = mk(a.sub_c[3 * so], a.sub_c[3 * so + 1], a.sub_c[3 * so + 2]);
      // Q3 points relative to v (the vertex v is the origin)
      v3 dj[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) dj[j] = cB3[j][1] * sm + cB3[j][2] * sc;
      const int lev = SUB ? subdiv_level(a.kr, fmax(fmax(norm(sm), norm(sc)), norm(sc - sm))) : 0;
      const int npiece = 1 << (2 * lev);
      const v3 sv3[3] = {mk(0, 0, 0), sm, sc};
      cz P = {0, 0};
      cv3 Q = cvzero(), Rm = cvzero(), S = cvzero();
#pragma unroll 1
      for (int k = 0; k < 7; ++k) {
        const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
        const v3 Dk = d + dk;
        cz m0 = {0, 0};
        cv3 m1 = cvzero();
        for (int jp = 0; jp < npiece; ++jp) {
          if (SUB && lev > 0) {
            double c[3][3];
            subdiv_corners(lev, jp, c);
            for (int j = 0; j < 3; ++j) dj[j] = subdiv_point(c, cB3[j], sv3);
          }
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            v3 r = Dk - dj[j];
            double r2 = dot(r, r);
            double inv = rsqrt(r2);
            double R = r2 * inv;
            cz g = cscale(1.0 / (3.0 * npiece), grad_green<LOSSY>(a.kr, a.ki, R, inv));
            m0 = cadd(m0, g);
            cv_axpy(m1, g, dj[j]);
          }
        }
        const double wk = cW7[k];
        // u = m1 - Delta m0
        cv3 u = m1;
        cv_axpy(u, cscale(-1.0, m0), Dk);
        cv3 Dxm1 = rc_cross(Dk, m1);
        cv3 dkxu = rc_cross(dk, u);
        P = cadd(P, cscale(wk, cv_dot(dk, rc_cross(d, m1))));
        Q.x = cadd(Q.x, cscale(wk, Dxm1.x)); Q.y = cadd(Q.y, cscale(wk, Dxm1.y)); Q.z = cadd(Q.z, cscale(wk, Dxm1.z));
        Rm.x = cadd(Rm.x, cscale(wk, dkxu.x)); Rm.y = cadd(Rm.y, cscale(wk, dkxu.y)); Rm.z = cadd(Rm.z, cscale(wk, dkxu.z));
        S.x = cadd(S.x, cscale(wk, u.x)); S.y = cadd(S.y, cscale(wk, u.y)); S.z = cadd(S.z, cscale(wk, u.z));
      }
      // per test half i: X_i = P - p_i.Q ;  Y_i = R - p_i x S
      cz X[3];
      cv3 Y[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);  // test vertex relative to the test centroid
        X[i] = csub(P, cv_dot(pi, Q));
        cv3 pxS = rc_cross(pi, S);
        Y[i].x = csub(Rm.x, pxS.x); Y[i].y = csub(Rm.y, pxS.y); Y[i].z = csub(Rm.z, pxS.z);
      }
#pragma unroll
      for (int b = 0; b < NACC; ++b) {
        if (b < nval) {
          const double al = 0.25 * a.alpha[size_t(b) * nc + v];
          const size_t bo = (size_t(b) * (2 * MAXV) + sidx) * nc + v;
          const v3 be = 0.25 * mk(a.beta[3 * bo], a.beta[3 * bo + 1], a.beta[3 * bo + 2]);
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[b][i] = cadd(acc[b][i], cadd(cscale(al, X[i]), cv_dot(be, Y[i])));
        }
      }
    }
    double2* out = a.Kc + (3 * tl) * a.ldK + col0;
#pragma unroll
    for (int b = 0; b < NACC; ++b)
      if (b < nval)
#pragma unroll
        for (int i = 0; i < 3; ++i) out[i * a.ldK + b] = make_double2(acc[b][i].re, acc[b][i].im);
  }
}

// ------------------------------------------------------------------ K near
// 2 MAXV lanes per near (T, cell) pair, one per sub-triangle of the cell (so a small mesh still
// fills the GPU): recompute the whole cell with the far moments for far sub-triangles and, for sub-triangles whose primal triangle is near T and not coplanar with
// it, with the extracted inner integral v_k = int_t g_k (r_k - r') dS':
//   v_k = -J/(4 pi) + k^2/(8 pi) Iv + sum_j w_j A_t h(R_kj) (r_k - r'_j)
// and the contribution 1/(4 A_t) sum_k w_k (r_k - p_i) . [v_k x (alpha (r_k - v) - beta)].
// The lanes' contributions are added by a butterfly over the pair's lanes (fixed order).
template <bool LOSSY, int MAXV>
__global__ void __launch_bounds__(64) k_fill_K_near(FillKArgs a, const int32_t* __restrict__ pt,
                                                    const int32_t* __restrict__ pc, int64_t npairs,
                                                    const int64_t* __restrict__ near_ptr,
                                                    const int32_t* __restrict__ near_idx) {
  constexpr int LANES = 2 * MAXV;  // divides 64: a pair's lanes share a wave
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t p = gid / LANES;
  const int sidx = int(gid % LANES);
  if (p >= npairs) return;  // whole lane groups leave together
  const int64_t t = pt[p];
  const int32_t v = pc[p];
  const int64_t nc = a.ncell_total;
  const double* geo = a.geo;
  const int64_t nt = a.nt_total;
  const int nval = a.nval[v];
  const v3 pv = mk(a.vpos[3 * v], a.vpos[3 * v + 1], a.vpos[3 * v + 2]);
  const v3 ct = G3(geo, nt, kGeoC, t);
  const v3 nT = G3(geo, nt, kGeoN, t);
  const double hT = G(geo, nt, kGeoH, t);
  const v3 d = ct - pv;
  const double kr = a.kr, ki = a.ki;
  cz k2 = cmul({kr, ki}, {kr, ki});
  cz acc[MAXV][3];
  for (int b = 0; b < MAXV; ++b)
    for (int i = 0; i < 3; ++i) acc[b][i] = {0, 0};
  if (sidx < 2 * nval) do {
    const size_t so = size_t(sidx) * nc + v;
    const v3 sm = mk(a.sub_m[3 * so], a.sub_m[3 * so + 1], a.sub_m[3 * so + 2]);
    const v3 sc = mk(a.sub_c[3 * so], a.sub_c[3 * so + 1], a.sub_c[3 * so + 2]);
    const double At = a.sub_area[so];
    const int32_t par = a.sub_parent[so];
    // is (t, par) a near pair?  binary search in the sorted near list of t
    int64_t lo = near_ptr[t], hi = near_ptr[t + 1];
    bool is_near = false;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      int32_t x = near_idx[mid];
      if (x == par) { is_near = true; break; }
      if (x < par) lo = mid + 1; else hi = mid;
    }
    v3 dj[3];
    for (int j = 0; j < 3; ++j) dj[j] = cB3[j][1] * sm + cB3[j][2] * sc;
    // inner rule: Q3 on each piece of the sub-triangle's level-L split (L = 0: plain Q3)
    const int lev = a.sub ? subdiv_level(kr, fmax(fmax(norm(sm), norm(sc)), norm(sc - sm))) : 0;
    const int npiece = 1 << (2 * lev);
    const v3 sv3[3] = {mk(0, 0, 0), sm, sc};
    if (!is_near) {
      cz P = {0, 0};
      cv3 Q = cvzero(), Rm = cvzero(), S = cvzero();
      for (int k = 0; k < 7; ++k) {
        const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
        const v3 Dk = d + dk;
        cz m0 = {0, 0};
        cv3 m1 = cvzero();
        for (int jp = 0; jp < npiece; ++jp) {
          if (lev > 0) {
            double c[3][3];
            subdiv_corners(lev, jp, c);
            for (int j = 0; j < 3; ++j) dj[j] = subdiv_point(c, cB3[j], sv3);
          }
          for (int j = 0; j < 3; ++j) {
            v3 r = Dk - dj[j];
            double r2 = dot(r, r);
            double inv = rsqrt(r2);
            cz g = cscale(1.0 / (3.0 * npiece), grad_green<LOSSY>(kr, ki, r2 * inv, inv));
            m0 = cadd(m0, g);
            cv_axpy(m1, g, dj[j]);
          }
        }
        const double wk = cW7[k];
        cv3 u = m1;
        cv_axpy(u, cscale(-1.0, m0), Dk);
        cv3 Dxm1 = rc_cross(Dk, m1);
        cv3 dkxu = rc_cross(dk, u);
        P = cadd(P, cscale(wk, cv_dot(dk, rc_cross(d, m1))));
        Q.x = cadd(Q.x, cscale(wk, Dxm1.x)); Q.y = cadd(Q.y, cscale(wk, Dxm1.y)); Q.z = cadd(Q.z, cscale(wk, Dxm1.z));
        Rm.x = cadd(Rm.x, cscale(wk, dkxu.x)); Rm.y = cadd(Rm.y, cscale(wk, dkxu.y)); Rm.z = cadd(Rm.z, cscale(wk, dkxu.z));
        S.x = cadd(S.x, cscale(wk, u.x)); S.y = cadd(S.y, cscale(wk, u.y)); S.z = cadd(S.z, cscale(wk, u.z));
      }
      for (int i = 0; i < 3; ++i) {
        const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);
        cz X = csub(P, cv_dot(pi, Q));
        cv3 pxS = rc_cross(pi, S);
        cv3 Y;
        Y.x = csub(Rm.x, pxS.x); Y.y = csub(Rm.y, pxS.y); Y.z = csub(Rm.z, pxS.z);
        for (int b = 0; b < MAXV; ++b) {
          if (b < nval) {
            const double al = 0.25 * a.alpha[size_t(b) * nc + v];
            const size_t bo = (size_t(b) * (2 * MAXV) + sidx) * nc + v;
            const v3 be = 0.25 * mk(a.beta[3 * bo], a.beta[3 * bo + 1], a.beta[3 * bo + 2]);
            acc[b][i] = cadd(acc[b][i], cadd(cscale(al, X), cv_dot(be, Y)));
          }
        }
      }
      break;
    }
    // near: zero when coplanar with the test triangle
    const v3 nP = G3(geo, nt, kGeoN, par);
    const v3 cP = G3(geo, nt, kGeoC, par);
    if (fabs(dot(nP, nT)) > 1.0 - 1e-12 && fabs(dot(cP - ct, nT)) < 1e-10 * hT) break;
    // sub-triangle vertices relative to v: (0, m, c) (the closed forms do not depend on the
    // vertex order)
    const v3 A0 = mk(0, 0, 0), A1 = sm, A2 = sc;
    for (int k = 0; k < 7; ++k) {
      const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
      const v3 Dk = d + dk;  // r_k - v
      StaticInts si = static_ints(Dk, A0, A1, A2, true);
      cv3 vk = cvzero();
      vk.x.re = -kInv4Pi * si.j3.x; vk.y.re = -kInv4Pi * si.j3.y; vk.z.re = -kInv4Pi * si.j3.z;
      cz c8 = cscale(0.5 * kInv4Pi, k2);  // k^2/(8 pi)
      cv_axpy(vk, c8, si.iv);
      for (int jp = 0; jp < npiece; ++jp) {
        if (lev > 0) {
          double c[3][3];
          subdiv_corners(lev, jp, c);
          for (int j = 0; j < 3; ++j) dj[j] = subdiv_point(c, cB3[j], sv3);
        }
        for (int j = 0; j < 3; ++j) {
          const v3 dd = Dk - dj[j];
          const double R = norm(dd);
          cz h = cscale(At / (3.0 * npiece), grad_green_rem(kr, ki, R));
          cv_axpy(vk, h, dd);
        }
      }
      const double wk = cW7[k] / (4.0 * At);
      for (int b = 0; b < MAXV; ++b) {
        if (b < nval) {
          const double al = a.alpha[size_t(b) * nc + v];
          const size_t bo = (size_t(b) * (2 * MAXV) + sidx) * nc + v;
          const v3 be = mk(a.beta[3 * bo], a.beta[3 * bo + 1], a.beta[3 * bo + 2]);
          const v3 gvec = al * Dk - be;
          // v_k x gvec  (complex x real)
          cv3 vxg;
          vxg.x = {vk.y.re * gvec.z - vk.z.re * gvec.y, vk.y.im * gvec.z - vk.z.im * gvec.y};
          vxg.y = {vk.z.re * gvec.x - vk.x.re * gvec.z, vk.z.im * gvec.x - vk.x.im * gvec.z};
          vxg.z = {vk.x.re * gvec.y - vk.y.re * gvec.x, vk.x.im * gvec.y - vk.y.im * gvec.x};
          for (int i = 0; i < 3; ++i) {
            const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);
            acc[b][i] = cadd(acc[b][i], cscale(wk, cv_dot(dk - pi, vxg)));
          }
        }
      }
    }
  } while (false);
  for (int b = 0; b < MAXV; ++b)
    for (int i = 0; i < 3; ++i)
      for (int off = 1; off < LANES; off <<= 1) {
        acc[b][i].re += __shfl_xor(acc[b][i].re, off);
        acc[b][i].im += __shfl_xor(acc[b][i].im, off);
      }
  if (sidx != 0) return;
  double2* out = a.Kc + (3 * (t - a.t0)) * a.ldK + a.col0[v];
  for (int b = 0; b < MAXV; ++b)
    if (b < nval)
      for (int i = 0; i < 3; ++i) out[i * a.ldK + b] = make_double2(acc[b][i].re, acc[b][i].im);
}

// ------------------------------------------------------------------ RHS
// Plane wave (right-hand side of eq. AEFIEextdis): b_m = eta0^-1 int f_m . pol E0 e^{-j k_l khat.r}
// = eta0^-1 sum over the two halves s/2 sum_k w_k (d_k - p_i) . pol E0 e^{-j k_l khat.(c + d_k)}.
__global__ void k_rhs_planewave(RhsArgs a) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int e = blockIdx.y;
  if (m >= a.ne) return;
  const double* geo = a.geo;
  const int64_t nt = a.nt_total;
  const v3 kh = mk(a.khat[3 * e], a.khat[3 * e + 1], a.khat[3 * e + 2]);
  const double2 p0 = a.pol[3 * e], p1 = a.pol[3 * e + 1], p2 = a.pol[3 * e + 2];
  const double2 amp = a.amp[e];
  cz acc = {0, 0};
  for (int h = 0; h < 2; ++h) {
    const int64_t t = h == 0 ? a.tp[m] : a.tm[m];
    const int i = h == 0 ? a.ip[m] : a.im[m];
    const double sg = h == 0 ? 0.5 : -0.5;
    const v3 c = G3(geo, nt, kGeoC, t);
    const v3 pi = G3(geo, nt, kGeoP + 3 * i, t);
    for (int k = 0; k < 7; ++k) {
      const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
      const v3 f = dk - pi;
      const double ph = dot(kh, c + dk);
      double s, co;
      sincos(a.klr * ph, &s, &co);
      const double ea = exp(a.kli * ph);
      const cz e0 = {ea * co, -ea * s};
      const cz fp = {f.x * p0.x + f.y * p1.x + f.z * p2.x, f.x * p0.y + f.y * p1.y + f.z * p2.y};
      acc = cadd(acc, cscale(sg * cW7[k], cmul(fp, e0)));
    }
  }
  const cz r = cscale(a.inv_eta0, cmul(acc, {amp.x, amp.y}));
  a.b[e * a.ldb + m] = make_double2(r.re, r.im);
}

// One block per (direction, column): threads stride over the triangles, then a fixed-order
// tree reduction in LDS.
__global__ void __launch_bounds__(256) k_far_field(FarArgs a) {
  const int64_t d = blockIdx.x;
  const int c = blockIdx.y;
  const double* geo = a.geo;
  const int64_t nt = a.nt;
  const v3 rh = mk(a.rhat[3 * d], a.rhat[3 * d + 1], a.rhat[3 * d + 2]);
  const double2* J = a.J + int64_t(c) * a.ldj;
  cz nx = {0, 0}, ny = {0, 0}, nz = {0, 0};
  for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) {
    const v3 ctr = G3(geo, nt, kGeoC, t);
    cz w[3];
    v3 p[3];
    for (int i = 0; i < 3; ++i) {
      const double2 j = J[a.tri_edge[3 * t + i]];
      const double s = 0.5 * a.tri_sign[3 * t + i];
      w[i] = {s * j.x, s * j.y};
      p[i] = G3(geo, nt, kGeoP + 3 * i, t);
    }
    for (int k = 0; k < 7; ++k) {
      const v3 dk = G3(geo, nt, kGeoQ + 3 * k, t);
      const double ph = dot(rh, ctr + dk);
      double sn, co;
      sincos(a.kr * ph, &sn, &co);
      const double ea = exp(-a.ki * ph);
      const cz e = {cW7[k] * ea * co, cW7[k] * ea * sn};
      for (int i = 0; i < 3; ++i) {
        const v3 f = dk - p[i];
        const cz we = cmul(w[i], e);
        nx = cadd(nx, cscale(f.x, we));
        ny = cadd(ny, cscale(f.y, we));
        nz = cadd(nz, cscale(f.z, we));
      }
    }
  }
  __shared__ double red[6][256];
  red[0][threadIdx.x] = nx.re; red[1][threadIdx.x] = nx.im;
  red[2][threadIdx.x] = ny.re; red[3][threadIdx.x] = ny.im;
  red[4][threadIdx.x] = nz.re; red[5][threadIdx.x] = nz.im;
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (threadIdx.x < half)
      for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + half];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double2* o = a.out + (int64_t(c) * a.ndir + d) * 3;
    o[0] = make_double2(red[0][0], red[1][0]);
    o[1] = make_double2(red[2][0], red[3][0]);
    o[2] = make_double2(red[4][0], red[5][0]);
  }
}

// One block per (point, column group, triangle range): each thread forms the three moments of
// its triangles once and applies them to every column of the group; fixed-order LDS tree per
// column, so the result does not depend on scheduling.
__global__ void __launch_bounds__(256) k_near_field(NearArgs a) {
  const int64_t p = blockIdx.x;
  const int c0 = int(blockIdx.y) * kNearFieldCols;
  const int nc = min(kNearFieldCols, a.ncol - c0);
  const int64_t per = (a.nt + a.nsplit - 1) / a.nsplit;
  const int64_t tb = int64_t(blockIdx.z) * per;
  const int64_t te = min(a.nt, tb + per);
  const double* geo = a.geo;
  const int64_t nt = a.nt;
  const v3 r = mk(a.pts[3 * p], a.pts[3 * p + 1], a.pts[3 * p + 2]);
  const cz k = {a.kr, a.ki};
  const cz k2over8pi = cscale(1.0 / (8.0 * kPi), cmul(k, k));
  const cz jwmu = {a.jwmu.x, a.jwmu.y}, inv_eps = {a.inv_eps.x, a.inv_eps.y};
  cz acc[kNearFieldCols][6];
#pragma unroll
  for (int cl = 0; cl < kNearFieldCols; ++cl)
#pragma unroll
    for (int m = 0; m < 6; ++m) acc[cl][m] = {0.0, 0.0};
  for (int64_t t = tb + threadIdx.x; t < te; t += blockDim.x) {
    const v3 rr = r - G3(geo, nt, kGeoC, t);  // the point relative to the centroid
    const double h = G(geo, nt, kGeoH, t), area = G(geo, nt, kGeoA, t);
    v3 P[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) P[i] = G3(geo, nt, kGeoP + 3 * i, t);
    const bool near = norm(rr) < kNearFactor * h;
    int L = subdiv_level(a.kr, h);
    if (near && L < kNearFieldLevel) L = kNearFieldLevel;
    const int npiece = 1 << (2 * L);
    const double wp = area / double(npiece);
    cz I0 = {0.0, 0.0};
    cv3 I1 = cvzero(), Ig = cvzero();
    for (int jp = 0; jp < npiece; ++jp) {
      double cc[3][3];
      if (L > 0) subdiv_corners(L, jp, cc);
      for (int q = 0; q < 7; ++q) {
        const v3 x = L > 0 ? subdiv_point(cc, cB7[q], P) : G3(geo, nt, kGeoQ + 3 * q, t);
        const v3 d = x - rr;  // r' - r
        const double R2 = dot(d, d);
        const double inv = 1.0 / sqrt(R2);
        const double R = R2 * inv;
        cz g, gg;
        if (near) {
          g = green_rem(a.kr, a.ki, R);
          gg = grad_green_rem(a.kr, a.ki, R);
        } else {
          g = green<true>(a.kr, a.ki, R, inv);
          gg = grad_green<true>(a.kr, a.ki, R, inv);
        }
        const double w = cW7[q] * wp;
        g = cscale(w, g);
        gg = cscale(-w, gg);
        I0 = cadd(I0, g);
        cv_axpy(I1, g, d);
        cv_axpy(Ig, gg, d);
      }
    }
    if (near) {
      // grad G = [g_rem - 1/(4 pi R^3) - k^2/(8 pi R)] (r - r')
      const StaticInts si = static_ints(rr, P[0], P[1], P[2], true);
      I0.re += kInv4Pi * si.i1;
      cv_axpy(I1, cz{kInv4Pi, 0.0}, si.iv);
      cv_axpy(Ig, cz{-kInv4Pi, 0.0}, si.j3);
      cv_axpy(Ig, k2over8pi, si.iv);
    }
    const double half_inv_area = 0.5 / area;
#pragma unroll
    for (int cl = 0; cl < kNearFieldCols; ++cl) {
      if (cl >= nc) continue;
      const int64_t c = c0 + cl;
      // J on t = (C r' - P)/(2 A): C = sum s_i J_i, P = sum s_i J_i v_i;  W = C r - P
      cz Cs = {0.0, 0.0};
      cv3 Q = cvzero();
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 j = a.J[c * a.ldj + a.tri_edge[3 * t + i]];
        const cz js = cscale(double(a.tri_sign[3 * t + i]), cz{j.x, j.y});
        Cs = cadd(Cs, js);
        cv_axpy(Q, js, P[i]);
      }
      cv3 W;
      W.x = csub(cscale(rr.x, Cs), Q.x);
      W.y = csub(cscale(rr.y, Cs), Q.y);
      W.z = csub(cscale(rr.z, Cs), Q.z);
      const double2 rho = a.rho[c * a.ldr + t];
      const cz qs = cscale(1.0 / area, cmul(inv_eps, cz{rho.x, rho.y}));
      // E += -j omega mu (C I1 + W I0)/(2A) - (rho / (eps A)) Ig;  H += Ig x W / (2A)
      const cz Ac[3] = {cscale(half_inv_area, cadd(cmul(Cs, I1.x), cmul(W.x, I0))),
                        cscale(half_inv_area, cadd(cmul(Cs, I1.y), cmul(W.y, I0))),
                        cscale(half_inv_area, cadd(cmul(Cs, I1.z), cmul(W.z, I0)))};
      const cz Igc[3] = {Ig.x, Ig.y, Ig.z};
      const cz Wc[3] = {W.x, W.y, W.z};
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        acc[cl][m] = csub(acc[cl][m], cadd(cmul(jwmu, Ac[m]), cmul(qs, Igc[m])));
        const int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
        const cz hx = csub(cmul(Igc[m1], Wc[m2]), cmul(Igc[m2], Wc[m1]));
        acc[cl][3 + m] = cadd(acc[cl][3 + m], cscale(half_inv_area, hx));
      }
    }
  }
  __shared__ double red[12][256];
#pragma unroll
  for (int cl = 0; cl < kNearFieldCols; ++cl) {
    if (cl >= nc) break;  // nc is the same for the whole block
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      red[2 * m][threadIdx.x] = acc[cl][m].re;
      red[2 * m + 1][threadIdx.x] = acc[cl][m].im;
    }
    __syncthreads();
    for (int half = 128; half > 0; half >>= 1) {
      if (threadIdx.x < half)
        for (int q = 0; q < 12; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + half];
      __syncthreads();
    }
    if (threadIdx.x < 6) {
      const int m = threadIdx.x;
      a.part[((int64_t(blockIdx.z) * a.ncol + c0 + cl) * a.npts + p) * 6 + m] =
          make_double2(red[2 * m][0], red[2 * m + 1][0]);
    }
    __syncthreads();
  }
}

// Sum of the triangle ranges in order, plus the incident plane wave when given:
// E_inc = E0 pol e^{-j k khat . r},  H_inc = khat x E_inc / eta.
__global__ void k_near_field_finish(NearArgs a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // c npts + p
  if (i >= int64_t(a.ncol) * a.npts) return;
  const int64_t c = i / a.npts, p = i - c * a.npts;
  cz f[6];
  for (int m = 0; m < 6; ++m) f[m] = {0.0, 0.0};
  for (int s = 0; s < a.nsplit; ++s)
    for (int m = 0; m < 6; ++m) {
      const double2 v = a.part[((int64_t(s) * a.ncol + c) * a.npts + p) * 6 + m];
      f[m] = cadd(f[m], cz{v.x, v.y});
    }
  if (a.inc) {
    const double* w = a.inc + 11 * c;
    const double ph = w[0] * a.pts[3 * p] + w[1] * a.pts[3 * p + 1] + w[2] * a.pts[3 * p + 2];
    // e^{-j k ph} with k = kr + j ki: e^{ki ph} (cos(kr ph) - j sin(kr ph))
    double sn, cs;
    sincos(a.kr * ph, &sn, &cs);
    const double ea = exp(a.ki * ph);
    const cz e0 = cmul(cz{w[9], w[10]}, cz{ea * cs, -ea * sn});
    cz Ei[3];
    for (int m = 0; m < 3; ++m) Ei[m] = cmul(e0, cz{w[3 + m], w[6 + m]});
    const cz ie = {a.inv_eta.x, a.inv_eta.y};
    for (int m = 0; m < 3; ++m) {
      const int m1 = (m + 1) % 3, m2 = (m + 2) % 3;
      f[m] = cadd(f[m], Ei[m]);
      const cz hx = csub(cscale(w[m1], Ei[m2]), cscale(w[m2], Ei[m1]));
      f[3 + m] = cadd(f[3 + m], cmul(ie, hx));
    }
  }
  for (int m = 0; m < 3; ++m) {
    a.E[i * 3 + m] = make_double2(f[m].re, f[m].im);
    a.H[i * 3 + m] = make_double2(f[3 + m].re, f[3 + m].im);
  }
}

}  // namespace dev

// ------------------------------------------------------------------ launchers

void launch_far_field(const FarArgs& a, int ncol, hipStream_t st) {
  if (a.ndir <= 0 || ncol <= 0) return;
  hipLaunchKernelGGL(dev::k_far_field, dim3(unsigned(a.ndir), unsigned(ncol)), dim3(256), 0, st, a);
  BEM_HIP(hipGetLastError());
}

void launch_near_field(const NearArgs& a, hipStream_t st) {
  if (a.npts <= 0 || a.ncol <= 0 || a.nt <= 0) return;
  const int64_t groups = (a.ncol + kNearFieldCols - 1) / kNearFieldCols;
  if (a.npts > 0x7fffffffLL || groups > 65535 || a.nsplit < 1 || a.nsplit > 65535)
    throw Error(BEM_E_INVALID, "near field: launch shape out of range");
  hipLaunchKernelGGL(dev::k_near_field, dim3(unsigned(a.npts), unsigned(groups), unsigned(a.nsplit)), dim3(256), 0,
                     st, a);
  BEM_HIP(hipGetLastError());
  const int64_t n = int64_t(a.ncol) * a.npts;
  hipLaunchKernelGGL(dev::k_near_field_finish, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, a);
  BEM_HIP(hipGetLastError());
}

void launch_rhs_planewave(const RhsArgs& a, int nexc, hipStream_t st) {
  if (a.ne <= 0 || nexc <= 0) return;
  hipLaunchKernelGGL(dev::k_rhs_planewave, dim3(unsigned((a.ne + 127) / 128), unsigned(nexc)), dim3(128), 0, st, a);
  BEM_HIP(hipGetLastError());
}

void fill_set_rules(const double w7[7], const double b7[7][3], const double b3[3][3], hipStream_t st) {
  // the rules never change: written once per device, complete before any fill reads them
  static std::mutex mu;
  static bool done[256] = {};
  int dev = 0;
  BEM_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  if (dev >= 0 && dev < 256 && done[dev]) return;
  BEM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(dev::cW7), w7, sizeof(double) * 7, 0, hipMemcpyHostToDevice, st));
  BEM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(dev::cB7), b7, sizeof(double) * 21, 0, hipMemcpyHostToDevice, st));
  BEM_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(dev::cB3), b3, sizeof(double) * 9, 0, hipMemcpyHostToDevice, st));
  BEM_HIP(hipStreamSynchronize(st));
  if (dev >= 0 && dev < 256) done[dev] = true;
}

void launch_fill_L(const FillLArgs& a, const int32_t* near_t, const int32_t* near_s, int64_t npairs,
                   hipStream_t st) {
  if (a.ns <= 0 || a.nt_test <= 0) return;
  dim3 grid(unsigned((a.ns + 255) / 256), unsigned((a.nt_test + a.tchunk - 1) / a.tchunk));
  bool lossy = a.ki != 0.0;
  {
    const double pairs = double(a.ns) * a.nt_test;
    ProfScope ps(st, KC_FILL_L, pairs * 10 * 16, pairs * 49);
    if (a.sub) {
      if (lossy) hipLaunchKernelGGL((dev::k_fill_L_far<true, true>), grid, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((dev::k_fill_L_far<false, true>), grid, dim3(256), 0, st, a);
    } else {
      if (lossy) hipLaunchKernelGGL((dev::k_fill_L_far<true, false>), grid, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((dev::k_fill_L_far<false, false>), grid, dim3(256), 0, st, a);
    }
    BEM_HIP(hipGetLastError());
  }
  if (npairs > 0) {
    ProfScope ps(st, KC_FILL_NEAR, double(npairs) * 10 * 16, double(npairs));
    dim3 g2(unsigned((npairs + 127) / 128));
    if (lossy) hipLaunchKernelGGL(dev::k_fill_L_near<true>, g2, dim3(128), 0, st, a, near_t, near_s, npairs);
    else hipLaunchKernelGGL(dev::k_fill_L_near<false>, g2, dim3(128), 0, st, a, near_t, near_s, npairs);
    BEM_HIP(hipGetLastError());
  }
}

void launch_fill_K(const FillKArgs& a, const int32_t* near_t, const int32_t* near_c, int64_t npairs,
                   const int64_t* near_ptr, const int32_t* near_idx, int maxv, hipStream_t st) {
  if (a.ncells <= 0 || a.nt_test <= 0) return;
  dim3 grid(unsigned((a.ncells + 127) / 128), unsigned((a.nt_test + a.tchunk - 1) / a.tchunk));
  bool lossy = a.ki != 0.0;
  dim3 g2(unsigned((npairs * 2 * maxv + 63) / 64));
  // every primal triangle of the object contributes 6 sub-triangles, 7 x 3 evaluations each
  const double kwork = double(a.nt_test) * 6.0 * a.nt_test * 21.0;
  const double kbytes = 3.0 * a.nt_test * a.ldK * 16.0;
#define BEM_KLAUNCH(L, MV)                                                                            \
  {                                                                                                   \
    ProfScope ps(st, KC_FILL_K, kbytes, kwork);                                                       \
    if (MV == 8 && a.valence > 0 && a.valence <= 6) {                                                \
      if (a.sub) hipLaunchKernelGGL((dev::k_fill_K_far<L, MV, true, 6>), grid, dim3(128), 0, st, a);  \
      else hipLaunchKernelGGL((dev::k_fill_K_far<L, MV, false, 6>), grid, dim3(128), 0, st, a);       \
    } else {                                                                                          \
      if (a.sub) hipLaunchKernelGGL((dev::k_fill_K_far<L, MV, true, MV>), grid, dim3(128), 0, st, a); \
      else hipLaunchKernelGGL((dev::k_fill_K_far<L, MV, false, MV>), grid, dim3(128), 0, st, a);      \
    }                                                                                                 \
    BEM_HIP(hipGetLastError());                                                                       \
  }                                                                                                   \
  if (npairs > 0) {                                                                                   \
    ProfScope ps(st, KC_FILL_NEAR, double(npairs) * 3 * MV * 16, double(npairs));                     \
    hipLaunchKernelGGL((dev::k_fill_K_near<L, MV>), g2, dim3(64), 0, st, a, near_t, near_c, npairs,   \
                       near_ptr, near_idx);                                                           \
    BEM_HIP(hipGetLastError());                                                                       \
  }
  if (maxv == 8) {
    if (lossy) { BEM_KLAUNCH(true, 8) } else { BEM_KLAUNCH(false, 8) }
  } else if (maxv == 16) {
    if (lossy) { BEM_KLAUNCH(true, 16) } else { BEM_KLAUNCH(false, 16) }
  } else {
    throw Error(BEM_E_INVALID, "unsupported padded valence");
  }
#undef BEM_KLAUNCH
}

void launch_gather_LA_rows(const double2* H, int64_t ldH, const int32_t* hp, const int32_t* hm, int64_t rlo,
                           int64_t rhi, int64_t coff, int64_t ncol, const int32_t* rows, int64_t nrows, double2* out,
                           int64_t ldo, hipStream_t st) {
  if (nrows <= 0 || ncol <= 0) return;
  dim3 grid(unsigned((ncol + 255) / 256), unsigned(std::min<int64_t>(nrows, 32768)));
  ProfScope ps(st, KC_GATHER, double(nrows) * ncol * 5 * 16, double(nrows) * ncol);
  hipLaunchKernelGGL(dev::k_gather_LA_rows, grid, dim3(256), 0, st, H, ldH, hp, hm, rlo, rhi, coff, ncol, rows, nrows,
                     out, ldo);
  BEM_HIP(hipGetLastError());
}

void launch_gather_K_rows(const double2* Kc, int64_t ldK, const int32_t* hp, const int32_t* hm, int64_t rlo, int64_t rhi,
                          const int32_t* cS, const int32_t* cT, int64_t ncol, const int32_t* rows, int64_t nrows,
                          double2* out, int64_t ldo, hipStream_t st) {
  if (nrows <= 0 || ncol <= 0) return;
  dim3 grid(unsigned((ncol + 255) / 256), unsigned(std::min<int64_t>(nrows, 32768)));
  ProfScope ps(st, KC_GATHER, double(nrows) * ncol * 5 * 16, double(nrows) * ncol);
  hipLaunchKernelGGL(dev::k_gather_K_rows, grid, dim3(256), 0, st, Kc, ldK, hp, hm, rlo, rhi, cS, cT, ncol, rows,
                     nrows, out, ldo);
  BEM_HIP(hipGetLastError());
}

}  // namespace bem
