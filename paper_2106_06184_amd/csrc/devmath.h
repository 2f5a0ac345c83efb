// Device helpers for the fill kernels: complex arithmetic on double2, the Green's function and
// its gradient (eq. hgf), their singular-part remainders, and the closed-form static integrals
// over a flat triangle (potential-integral formulas of Wilton et al. / Graglia).
#pragma once

#include <hip/hip_runtime.h>

namespace bem {
namespace dev {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInv4Pi = 1.0 / (4.0 * kPi);
// |kR| below which the regularised kernels use their power series (cancellation-free).
constexpr double kSeriesKR = 0.5;

struct v3 {
  double x, y, z;
};
__device__ __forceinline__ v3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ v3 operator+(v3 a, v3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ v3 operator-(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ v3 operator*(double s, v3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ v3 cross(v3 a, v3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double norm(v3 a) { return sqrt(dot(a, a)); }

// complex double and complex 3-vectors
struct cz {
  double re, im;
};
struct cv3 {
  cz x, y, z;
};
__device__ __forceinline__ cz cmul(cz a, cz b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cz cadd(cz a, cz b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cz csub(cz a, cz b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cz cscale(double s, cz a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cv3 cvzero() { return {{0, 0}, {0, 0}, {0, 0}}; }
// a += w * c * v   (c complex scalar, v real vector)
__device__ __forceinline__ void cv_axpy(cv3& a, cz c, v3 v) {
  a.x.re += c.re * v.x; a.x.im += c.im * v.x;
  a.y.re += c.re * v.y; a.y.im += c.im * v.y;
  a.z.re += c.re * v.z; a.z.im += c.im * v.z;
}
__device__ __forceinline__ cz cv_dot(v3 v, cv3 a) {
  return {v.x * a.x.re + v.y * a.y.re + v.z * a.z.re, v.x * a.x.im + v.y * a.y.im + v.z * a.z.im};
}
// v x a for real v and complex a
__device__ __forceinline__ cv3 rc_cross(v3 v, cv3 a) {
  cv3 r;
  r.x = {v.y * a.z.re - v.z * a.y.re, v.y * a.z.im - v.z * a.y.im};
  r.y = {v.z * a.x.re - v.x * a.z.re, v.z * a.x.im - v.x * a.z.im};
  r.z = {v.x * a.y.re - v.y * a.x.re, v.x * a.y.im - v.y * a.x.im};
  return r;
}
__device__ __forceinline__ void cv_add(cv3& a, cv3 b) {
  a.x = cadd(a.x, b.x); a.y = cadd(a.y, b.y); a.z = cadd(a.z, b.z);
}

// sin and cos of x for |x| < 2^20: x = n pi/2 + r with n = rint(2x / pi) and r reduced by the
// three-part split of pi/2 (Cody and Waite), each part subtracted by a fused multiply-add;
// Taylor polynomials of sin and cos on |r| <= pi/4 (truncation below 7e-17 relative); the
// quadrant n mod 4 picks and signs the pair.
__device__ __forceinline__ void sincos_reduced(double x, double* s, double* c) {
  constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
  constexpr double kP1 = 0x1.921fb54442d18p+0, kP2 = 0x1.1a62633145c07p-54, kP3 = -0x1.f1976b7ed8fbcp-110;
  const double n = rint(x * kTwoOverPi);
  const double r = fma(-n, kP3, fma(-n, kP2, fma(-n, kP1, x)));
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ... - r^14/15!),  cos r = 1 - r^2/2! + ... + r^16/16!
  double ps = -7.6471637318198164759e-13;              // -1/15!
  ps = fma(ps, r2, 1.6059043836821614599e-10);        //  1/13!
  ps = fma(ps, r2, -2.5052108385441718775e-08);       // -1/11!
  ps = fma(ps, r2, 2.7557319223985890653e-06);        //  1/9!
  ps = fma(ps, r2, -1.9841269841269841270e-04);       // -1/7!
  ps = fma(ps, r2, 8.3333333333333333333e-03);        //  1/5!
  ps = fma(ps, r2, -1.6666666666666666667e-01);       // -1/3!
  const double sr = fma(r * r2, ps, r);
  double pc = 4.7794773323873852974e-14;               //  1/16!
  pc = fma(pc, r2, -1.1470745597729724714e-11);       // -1/14!
  pc = fma(pc, r2, 2.0876756987868098979e-09);        //  1/12!
  pc = fma(pc, r2, -2.7557319223985890653e-07);       // -1/10!
  pc = fma(pc, r2, 2.4801587301587301587e-05);        //  1/8!
  pc = fma(pc, r2, -1.3888888888888888889e-03);       // -1/6!
  pc = fma(pc, r2, 4.1666666666666666667e-02);        //  1/4!
  pc = fma(pc, r2, -0.5);                              // -1/2!
  const double cr = fma(r2, pc, 1.0);
  const int q = int(int64_t(n) & 3);
  const double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// e^{-jkR} for k = kr + j ki  ->  e^{ki R} (cos kr R - j sin kr R)
template <bool LOSSY>
__device__ __forceinline__ cz expjkr(double kr, double ki, double R) {
  double s, c;
  sincos_reduced(kr * R, &s, &c);
  if (LOSSY) {
    double a = exp(ki * R);
    return {a * c, -a * s};
  }
  return {c, -s};
}

// G_k(R) = e^{-jkR}/(4 pi R), given R and 1/R
template <bool LOSSY>
__device__ __forceinline__ cz green(double kr, double ki, double R, double invR) {
  cz e = expjkr<LOSSY>(kr, ki, R);
  double s = kInv4Pi * invR;
  return {s * e.re, s * e.im};
}

// g_k(R) with grad_r G = g_k(R) (r - r'):  -(1 + jkR) e^{-jkR} / (4 pi R^3)
template <bool LOSSY>
__device__ __forceinline__ cz grad_green(double kr, double ki, double R, double invR) {
  cz e = expjkr<LOSSY>(kr, ki, R);
  // 1 + jkR = (1 - ki R) + j kr R
  cz f = {1.0 - ki * R, kr * R};
  cz p = cmul(f, e);
  double s = -kInv4Pi * invR * invR * invR;
  return {s * p.re, s * p.im};
}

// G_k(R) - 1/(4 pi R) = (e^{-jkR} - 1)/(4 pi R); bounded at R = 0.
__device__ inline cz green_rem(double kr, double ki, double R) {
  // z = -jkR = (ki R) - j (kr R)
  cz z = {ki * R, -kr * R};
  double az = sqrt(z.re * z.re + z.im * z.im);
  if (az >= kSeriesKR) {
    double ea = exp(z.re), s, c;
    sincos_reduced(z.im, &s, &c);
    cz em1 = {ea * c - 1.0, ea * s};
    double w = kInv4Pi / R;
    return {w * em1.re, w * em1.im};
  }
  // (e^z - 1)/R = (-jk) sum_{n>=1} z^{n-1}/n!
  cz term = {1.0, 0.0}, acc = {1.0, 0.0};
  for (int n = 2; n < 30; ++n) {
    term = cscale(1.0 / n, cmul(term, z));
    acc = cadd(acc, term);
  }
  cz mjk = {ki, -kr};  // -jk
  cz r = cmul(mjk, acc);
  return {kInv4Pi * r.re, kInv4Pi * r.im};
}

// g_k(R) + 1/(4 pi R^3) + k^2/(8 pi R); tends to j k^3/(12 pi) at R = 0.
__device__ inline cz grad_green_rem(double kr, double ki, double R) {
  double akr = sqrt(kr * kr + ki * ki) * R;
  cz k = {kr, ki};
  cz k2 = cmul(k, k);
  if (akr >= kSeriesKR) {
    double invR = 1.0 / R;
    cz g = grad_green<true>(kr, ki, R, invR);
    double i3 = kInv4Pi * invR * invR * invR;
    double s = 0.5 * kInv4Pi * invR;
    return {g.re + i3 + s * k2.re, g.im + s * k2.im};
  }
  // (1/4pi) sum_{n>=3} (-1)^n (n-1)/n! (jk)^n R^{n-3}
  cz jk = {-ki, kr};
  cz jkn = cmul(cmul(jk, jk), jk);  // (jk)^3
  double rp = 1.0, fact = 6.0;
  cz acc = {0.0, 0.0};
  for (int n = 3; n < 40; ++n) {
    double c = ((n & 1) ? -1.0 : 1.0) * (n - 1) / fact * rp;
    acc = cadd(acc, cscale(c, jkn));
    jkn = cmul(jkn, jk);
    rp *= R;
    fact *= (n + 1);
  }
  return {kInv4Pi * acc.re, kInv4Pi * acc.im};
}

// Closed-form static integrals over the flat triangle (a, b, c) (counter-clockwise about its
// normal n) at observation point r.  Outputs:
//   i1  = int 1/R dS'
//   iv  = int (r' - r)/R dS'
//   j3  = int (r - r')/R^3 dS'   (only when want_j3; r must not lie on the closed triangle)
struct StaticInts {
  double i1;
  v3 iv;
  v3 j3;
};

__device__ inline StaticInts static_ints(v3 r, v3 a, v3 b, v3 c, bool want_j3) {
  v3 n = cross(b - a, c - a);
  n = (1.0 / norm(n)) * n;
  double d = dot(r - a, n);
  double ad = fabs(d);
  v3 rho = r - d * n;
  StaticInts out;
  out.i1 = 0.0;
  out.iv = mk(0, 0, 0);
  out.j3 = mk(0, 0, 0);
  double bsum = 0.0;
  v3 irho = mk(0, 0, 0);
  v3 ends[4] = {a, b, c, a};
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    v3 p0 = ends[e], p1 = ends[e + 1];
    v3 s = p1 - p0;
    s = (1.0 / norm(s)) * s;
    v3 m = cross(s, n);
    double sm = dot(p0 - rho, s), sp = dot(p1 - rho, s), t0 = dot(p0 - rho, m);
    double r02 = t0 * t0 + d * d;
    double rm = sqrt(r02 + sm * sm), rp = sqrt(r02 + sp * sp);
    double f;
    if (sm >= 0.0)
      f = log((rp + sp) / (rm + sm));
    else if (sp <= 0.0)
      f = log((rm - sm) / (rp - sp));
    else
      f = log((rp + sp) * (rm - sm) / r02);
    double beta = atan2(t0 * sp, r02 + ad * rp) - atan2(t0 * sm, r02 + ad * rm);
    if (t0 != 0.0) out.i1 += t0 * f;
    out.i1 -= ad * beta;
    double term = (r02 > 0.0 ? r02 * f : 0.0) + sp * rp - sm * rm;
    irho = irho + (0.5 * term) * m;
    if (want_j3) out.j3 = out.j3 + f * m;
    bsum += beta;
  }
  out.iv = irho - (d * out.i1) * n;
  if (want_j3) out.j3 = out.j3 + ((d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0)) * bsum) * n;
  return out;
}

}  // namespace dev
}  // namespace bem
