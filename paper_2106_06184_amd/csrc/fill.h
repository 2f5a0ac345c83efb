// Fill-kernel interface shared by the host driver and fill.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bem {

// Per-triangle geometry table (float64, field-major: field f of triangle t at geo[f * nt + t]).
enum : int {
  kGeoC = 0,    // centroid (3)
  kGeoQ = 3,    // Q7 points relative to the centroid (7 x 3)
  kGeoP = 24,   // vertices relative to the centroid (3 x 3); vertex i is the free vertex of half-RWG i
  kGeoA = 33,   // area
  kGeoN = 34,   // unit outward normal (3)
  kGeoH = 37,   // longest edge
  kGeoFields = 38
};

struct FillLArgs {
  const double* geo;
  int64_t nt_total;
  int64_t t0, nt_test;  // test triangle range
  int64_t s0, ns;       // source triangle range
  int64_t tchunk;       // test triangles per block (grid.y)
  double kr, ki;        // wavenumber
  double2* H;           // half-RWG block matrix, rows 3*(T-t0)+i, cols 3*(T'-s0)+j
  int64_t ldH;
  double2* Lphi;        // rows T-t0, cols T'-s0
  int64_t ldP;
  int sub;              // 1: some source triangle needs its rule subdivided (|Re k| h > 2)
};

struct FillKArgs {
  const double* geo;
  int64_t nt_total;
  int64_t t0, nt_test;
  int64_t tchunk;
  double kr, ki;
  const int32_t* cells;   // cell (vertex) ids of this object
  int64_t ncells;
  int64_t ncell_total;    // stride of the cell tables
  const int32_t* nval;
  const double* vpos;
  const int64_t* col0;
  const double* sub_m;
  const double* sub_c;
  const double* sub_area;
  const int32_t* sub_parent;
  const double* alpha;
  const double* beta;
  double2* Kc;            // rows 3*(T-t0)+i, cols = object-local (cell, BC) columns
  int64_t ldK;
  int sub;                // 1: some source sub-triangle needs its rule subdivided
  int valence = 0;        // largest valence of the cells (0: not known, the padded one is assumed)
};

// Source-rule subdivision for highly conductive objects: a source piece of longest edge h is
// split 4-to-1 L times, the least L with |Re k| h / 2^L <= kSubdivKh, at most kSubdivMax.
constexpr double kSubdivKh = 2.0;
constexpr int kSubdivMax = 4;
inline int subdiv_level_host(double kr, double h) {
  const double x = (kr < 0 ? -kr : kr) * h;
  int L = 0;
  while (L < kSubdivMax && x / double(1 << L) > kSubdivKh) ++L;
  return L;
}

struct RhsArgs {
  const double* geo;
  int64_t nt_total;
  const int32_t* tp;
  const int32_t* tm;
  const int8_t* ip;
  const int8_t* im;
  int64_t ne;
  const double* khat;   // 3 per excitation
  const double2* pol;   // 3 per excitation
  const double2* amp;   // 1 per excitation
  double klr, kli;      // background wavenumber
  double inv_eta0;
  double2* b;           // column-major ne x nexc
  int64_t ldb;
};
void launch_rhs_planewave(const RhsArgs& a, int nexc, hipStream_t st);

// N(rhat) = int J(r') exp(+j k rhat . r') dS' of RWG coefficients J (column c at J + c ldj),
// 7-point rule per triangle; out[(c ndir + d) 3 + i], i = x, y, z.
struct FarArgs {
  const double* geo;
  int64_t nt;
  const int32_t* tri_edge;  // 3 nt
  const int8_t* tri_sign;   // 3 nt
  const double2* J;
  int64_t ldj;
  double kr, ki;            // background wavenumber
  const double* rhat;       // 3 per direction
  int64_t ndir;
  double2* out;
};
void launch_far_field(const FarArgs& a, int ncol, hipStream_t st);

// Near field at exterior points of the sources J (RWG coefficients, column c at J + c ldj) and
// rho (area-normalised pulse coefficients, rho + c ldr) radiating in the background:
//   E = -j omega mu A - grad Phi,  H = curl A,  A = int G J,  Phi = (1/eps) int G rho.
// Triangle t's part is formed from its moments I0 = int G, I1 = int G (r' - r),
// Ig = int grad_r G (7-point rule on the 4^L pieces of the fill's source split; for a point
// closer than kNearFactor longest edges to the centroid the static parts in closed form and
// the remainders on at least the kNearFieldLevel split).  Blocks: (point, group of
// kNearFieldCols columns, triangle range); the range sums go to `part` and a second kernel adds
// them in range order (and the incident plane wave of column c when `inc` is set), writing
// E[(c npts + p) 3 + i] and H likewise.
constexpr int kNearFieldCols = 4;
constexpr int kNearFieldLevel = 2;
struct NearArgs {
  const double* geo;
  int64_t nt;
  const int32_t* tri_edge;  // 3 nt
  const int8_t* tri_sign;   // 3 nt
  const double2* J;
  int64_t ldj;
  const double2* rho;
  int64_t ldr;
  int ncol;
  double kr, ki;            // background wavenumber
  double2 jwmu;             // j omega mu0 mu_l
  double2 inv_eps;          // 1 / (eps0 eps_l)
  double2 inv_eta;          // 1 / eta_l
  const double* pts;        // 3 per point
  int64_t npts;
  const double* inc;        // null, or 11 per column: khat (3), Re pol (3), Im pol (3), Re E0, Im E0
  int nsplit;               // triangle ranges
  double2* part;            // nsplit x ncol x npts x 6
  double2* E;               // ncol x npts x 3
  double2* H;
};
void launch_near_field(const NearArgs& a, hipStream_t st);

// Quadrature rules into constant memory (once per device; later calls return at once).
void fill_set_rules(const double w7[7], const double b7[7][3], const double b3[3][3], hipStream_t st);
void launch_fill_L(const FillLArgs& a, const int32_t* near_t, const int32_t* near_s, int64_t npairs,
                   hipStream_t st);
void launch_fill_K(const FillKArgs& a, const int32_t* near_t, const int32_t* near_c, int64_t npairs,
                   const int64_t* near_ptr, const int32_t* near_idx, int maxv, hipStream_t st);
// Chunked gathers: the listed edge rows `rows` (indices into hp/hm) with a half-RWG in the chunk's
// half-rows [rlo, rhi) (half-row matrix row h - rlo); a row with both halves in the chunk is
// written whole, a half alone is written by the first chunk (in chunk order) holding a half of the
// row and added by the second.  hp/hm hold the global half-RWG indices 3 T + i of the block's
// edges.  L: columns n < ncol at half-columns hp[n] - coff, hm[n] - coff (coff = 3 x the first
// source triangle).  K~: columns n < ncol from the cell-expanded columns cS[n], cT[n].
void launch_gather_LA_rows(const double2* H, int64_t ldH, const int32_t* hp, const int32_t* hm, int64_t rlo,
                           int64_t rhi, int64_t coff, int64_t ncol, const int32_t* rows, int64_t nrows, double2* out,
                           int64_t ldo, hipStream_t st);
void launch_gather_K_rows(const double2* Kc, int64_t ldK, const int32_t* hp, const int32_t* hm, int64_t rlo, int64_t rhi,
                          const int32_t* cS, const int32_t* cT, int64_t ncol, const int32_t* rows, int64_t nrows,
                          double2* out, int64_t ldo, hipStream_t st);

}  // namespace bem
