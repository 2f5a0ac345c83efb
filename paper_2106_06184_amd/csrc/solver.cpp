// Operator assembly, block application, the nested equivalent-configuration solve, GMRES and
// the float32/float64 refinement driver.
//
// Final system (eq. finalsystem) with unknowns [a; e; x3] = [jk0 H; E/eta0; -c0 rho'] and a
// homogeneous background (L^A_m = mu_l L^A_l, L^phi_m = L^phi_l / eps_l):
//   y1 = L^A_m (a - u) + D^T L^phi_m B (x3 + w) + I_x e
//   y2 = mu_r L^A a - (K~ + I_x/2) e + eps_c^-1 D^T L^phi B x3
//   y3 = F D (a - u) + k0^2 (x3 + w)
// where [u; w] = [Y11 e; Y21 e] solves eq. AEFIEeqvdis, M_eq [u; w] = [(K~_l + I_x/2) e; 0],
// for every product (Sec. III: Y is never formed).  Two readings of the printed system are
// used: the middle block is -K (it follows from eq. AEFIEintdis with x3 = -c0 rho'), and
// C1 carries L^phi_m as eq. AEFIEextdis does.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>

#include "ctx.h"
#include "dense.h"
#include "prof.h"

namespace bem {

// part 1: nested-solve inverses; part 2: block preconditioners.
void build_inner_and_precond(OpObj& op, const std::vector<double>& ixdiag, hipStream_t st, int part);

namespace {

inline double2 c2(double re, double im = 0.0) { return make_double2(re, im); }
inline double2 c2(cd z) { return make_double2(z.real(), z.imag()); }
inline int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

// Product work vectors: 15 fields per column, each padded to the equivalent-system size.
constexpr int kWorkFields = 15;
int64_t work_ld(const OpObj& op) { return pad64(op.Neq); }

// Largest relative deviation of the float32 final-system product from the float64 one for which
// a mixed-precision solve uses float32 products (in the late steps of its sweeps).
constexpr double kFp32ProbeTol = 1e-4;

// Smallest |k_l| h_max for which the nested solve eliminates the charges (S of build_s): its
// D^T L^phi D / k0^2 term grows like (k h)^-2 against the L^A term.
constexpr double kSchurMinKh = 0.01;

// Radon 7-point degree-5 rule (barycentric points, weights summing to 1) and the 3-point rule.
struct Rules {
  double b7[7][3];
  double w7[7];
  double b3[3][3];
  Rules() {
    const double s = std::sqrt(15.0);
    const double a1 = (6.0 - s) / 21.0, a2 = (6.0 + s) / 21.0;
    const double w1 = (155.0 - s) / 1200.0, w2 = (155.0 + s) / 1200.0;
    const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, a1, 1 - 2 * a1}, {a1, 1 - 2 * a1, a1},
                              {1 - 2 * a1, a1, a1},        {a2, a2, 1 - 2 * a2}, {a2, 1 - 2 * a2, a2},
                              {1 - 2 * a2, a2, a2}};
    const double ws[7] = {9.0 / 40, w1, w1, w1, w2, w2, w2};
    std::memcpy(b7, pts, sizeof(b7));
    std::memcpy(w7, ws, sizeof(w7));
    const double p3[3][3] = {{2.0 / 3, 1.0 / 6, 1.0 / 6}, {1.0 / 6, 2.0 / 3, 1.0 / 6}, {1.0 / 6, 1.0 / 6, 2.0 / 3}};
    std::memcpy(b3, p3, sizeof(b3));
  }
};
const Rules& rules() {
  static Rules r;
  return r;
}

Dense alloc_dense(DevArena& mem, int64_t rows, int64_t cols, bool fp32) {
  Dense d;
  d.rows = rows;
  d.cols = cols;
  d.ld = pad64(std::max<int64_t>(cols, 1));
  d.d64 = mem.alloc<double2>(size_t(rows) * d.ld);
  BEM_HIP(hipMemsetAsync(d.d64, 0, sizeof(double2) * size_t(rows) * d.ld, mem.stream()));
  if (fp32) d.d32 = mem.alloc<float2>(size_t(rows) * d.ld);
  return d;
}

void to_f32(Dense& d, hipStream_t st) {
  if (d.d32) launch_cast_f32(d.d64, d.rows, d.cols, d.ld, d.d32, d.ld, st);
}

GemvDesc desc(const Dense& A, bool fp32, int64_t roff, int64_t coff, int64_t rows, int64_t cols, const double2* x,
              double2* y, double2 alpha, int acc) {
  GemvDesc d{};
  // a block whose float64 entries were dropped (BEM_FP32) is read in float32; a float64 product
  // of it keeps float64 arithmetic (the refinement's residuals)
  d.fp32 = fp32 ? 1 : 0;
  if (!A.d64) {
    d.fp32 = fp32 ? 1 : 2;
    fp32 = true;
  }
  if (fp32) d.A = A.d32 + roff * A.ld + coff;
  else d.A = A.d64 + roff * A.ld + coff;
  d.lda = A.ld;
  d.rows = rows;
  d.cols = cols;
  d.x = x;
  d.y = y;
  d.alpha = alpha;
  d.accumulate = acc;
  return d;
}

void add_second(GemvDesc& d, const Dense& A, bool fp32, int64_t roff, int64_t coff, const double2* x, double2 alpha) {
  (void)fp32;  // one launch reads both matrices in the first one's storage precision
  if (d.fp32) d.A2 = A.d32 + roff * A.ld + coff;
  else d.A2 = A.d64 + roff * A.ld + coff;
  d.lda2 = A.ld;
  d.x2 = x;
  d.alpha2 = alpha;
}

}  // namespace

// BEM_VERBOSE=1 prints one line per GMRES iteration (outer) and per nested solve to stderr.
static bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("BEM_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

// BEM_TIMING=1 prints the host wall time of each assembly phase (the stream is synchronised at
// every mark, so the device work of a phase is inside it).
static bool timing() {
  static const bool v = [] {
    const char* e = std::getenv("BEM_TIMING");
    return e && *e && *e != '0';
  }();
  return v;
}

// ----------------------------------------------------------------- arena / ctx

namespace {
// Allocation granule of the block cache: sizes are rounded up so that repeated assemblies of
// similar problems find their blocks again.
size_t granule(size_t bytes) {
  const size_t g = bytes >= (size_t(64) << 20) ? (size_t(2) << 20) : (bytes >= (size_t(1) << 20) ? 65536 : 256);
  return (bytes + g - 1) / g * g;
}
}  // namespace

void* DevArena::raw(size_t bytes) {
  bytes = granule(std::max<size_t>(bytes, 1));
  std::vector<void*> evict;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> g(ctx_->mu);
    // reuse an idle block of this size (at most 1/8 larger)
    auto it = ctx_->cache.lower_bound(bytes);
    if (it != ctx_->cache.end() && it->first <= bytes + bytes / 8) {
      bytes = it->first;
      p = it->second;
      ctx_->cache.erase(it);
      ctx_->cached -= bytes;
    } else {
      // make room: drop idle blocks (largest first) until the request fits the budget
      while (ctx_->used + ctx_->cached + bytes > ctx_->budget && !ctx_->cache.empty()) {
        auto last = std::prev(ctx_->cache.end());
        evict.push_back(last->second);
        ctx_->cached -= last->first;
        ctx_->cache.erase(last);
      }
      if (ctx_->used + ctx_->cached + bytes > ctx_->budget)
        throw Error(BEM_E_NOMEM, "device memory budget exceeded (" + std::to_string(ctx_->used + bytes) + " > " +
                                     std::to_string(ctx_->budget) + " bytes)");
    }
    ctx_->used += bytes;
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (void* q : evict) (void)hipFree(q);
  if (verbose() && !evict.empty())
    std::fprintf(stderr, "[bem] alloc: evicted %zu idle blocks in %.2f ms\n", evict.size(),
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
  if (!p) {
    const auto t1 = std::chrono::steady_clock::now();
    hipError_t e = hipMalloc(&p, bytes);
    if (verbose())
      std::fprintf(stderr, "[bem] alloc: hipMalloc %.1f MB in %.2f ms\n", double(bytes) / 1e6,
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count());
    if (e != hipSuccess) {
      (void)hipGetLastError();
      // the device may hold idle blocks of other contexts' sizes: drop ours and retry once
      std::vector<void*> all;
      {
        std::lock_guard<std::mutex> g(ctx_->mu);
        for (auto& kv : ctx_->cache) all.push_back(kv.second);
        ctx_->cache.clear();
        ctx_->cached = 0;
      }
      for (void* q : all) (void)hipFree(q);
      e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        std::lock_guard<std::mutex> g(ctx_->mu);
        ctx_->used -= bytes;
        (void)hipGetLastError();
        throw Error(BEM_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
      }
    }
  }
  blocks_.push_back({p, bytes});
  total_ += bytes;
  return p;
}

void DevArena::release(void* p) {
  for (size_t i = 0; i < blocks_.size(); ++i) {
    if (blocks_[i].first == p) {
      if (stream_) (void)hipStreamSynchronize(stream_);  // the block is idle before it is reused
      std::lock_guard<std::mutex> g(ctx_->mu);
      ctx_->used -= blocks_[i].second;
      ctx_->cached += blocks_[i].second;
      ctx_->cache.emplace(blocks_[i].second, p);
      total_ -= blocks_[i].second;
      blocks_.erase(blocks_.begin() + long(i));
      return;
    }
  }
}

DevArena::~DevArena() {
  if (blocks_.empty()) return;
  if (stream_) (void)hipStreamSynchronize(stream_);
  std::lock_guard<std::mutex> g(ctx_->mu);
  for (auto& b : blocks_) {
    ctx_->used -= b.second;
    ctx_->cached += b.second;
    ctx_->cache.emplace(b.second, b.first);
  }
}

OpObj::~OpObj() {}

// ----------------------------------------------------------------- assembly

// BEM_FP32: once the float32 copies and the inverses exist, the float64 entries of every dense
// block are released (shared copies of an object's blocks point at the same memory, so every
// descriptor of a released buffer is cleared); products then read float32 storage (desc).
void drop_f64_blocks(OpObj& op) {
  BEM_HIP(hipStreamSynchronize(op.stream));
  std::vector<Dense*> all;
  for (auto* v : {&op.LA_int, &op.Lphi_int, &op.K_int, &op.K_bg, &op.Minv, &op.SigP, &op.SigEq})
    for (Dense& d : *v) all.push_back(&d);
  for (Dense* d : {&op.LA_bg, &op.Lphi_bg, &op.Km}) all.push_back(d);
  std::vector<double2*> done;
  for (Dense* d : all) {
    if (!d->d64) continue;
    if (!d->d32) throw Error(BEM_E_INVALID, "float32 copy missing");
    double2* p = d->d64;
    if (std::find(done.begin(), done.end(), p) == done.end()) {
      // views into a larger block (the eAEFIE's per-object K~_l) are released with that block
      if (op.mem.owns(p)) op.mem.release(p);
      done.push_back(p);
    }
  }
  for (Dense* d : all) d->d64 = nullptr;
}

// Test triangles per fill chunk: the half-row scratch of a chunk (3 rows per triangle, row_len
// complex entries each) stays within kFillScratchBytes, and the chunks of nt triangles are of
// equal size (no short last chunk).  A function of the mesh alone.
int64_t fill_chunk_triangles(int64_t nt, int64_t row_len) {
  const int64_t per_tri = 3 * row_len * int64_t(sizeof(double2));
  const int64_t most = std::max<int64_t>(1, std::min<int64_t>(nt, int64_t(kFillScratchBytes) / std::max<int64_t>(per_tri, 1)));
  const int64_t nchunk = (nt + most - 1) / most;
  return (nt + nchunk - 1) / nchunk;
}

void assemble_op(OpObj& op, MeshObj& mo, const bem_problem& prob) {
  auto tmark = std::chrono::steady_clock::now();
  const Mesh& m = *mo.mesh;
  if (!mo.cells) mo.cells = std::make_unique<CellData>(build_cells(m));
  const CellData& cdat = *mo.cells;
  op.m = &m;
  op.cells = &cdat;
  hipStream_t st = op.stream;
  auto mark = [&](const char* what) {
    if (!timing()) return;
    BEM_HIP(hipStreamSynchronize(st));
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[bem] assemble %-22s %8.2f ms\n", what,
                 std::chrono::duration<double, std::milli>(now - tmark).count());
    tmark = now;
  };
  mark("cells");
  op.mem.set_stream(st);
  const Rules& R = rules();
  fill_set_rules(R.w7, R.b7, R.b3, st);

  // ---- problem constants (eq. epsrc; k = sqrt(eps_c mu_r) k0 with Im k <= 0)
  if (!(prob.freq_hz > 0) || !std::isfinite(prob.freq_hz)) throw Error(BEM_E_INVALID, "frequency must be positive");
  if (prob.n_obj != m.nobj || (m.nobj > 0 && !prob.obj)) throw Error(BEM_E_INVALID, "one material per object required");
  if (prob.precision != BEM_FP64 && prob.precision != BEM_MIXED && prob.precision != BEM_FP32)
    throw Error(BEM_E_INVALID, "unknown precision");
  op.precision = prob.precision;
  op.freq = prob.freq_hz;
  const double w = 2 * kPi * prob.freq_hz;
  op.k0 = w / kC0;
  auto wavenumber = [&](cd eps, double mu) {
    cd k = std::sqrt(eps * mu) * op.k0;
    if (k.imag() > 0) k = -k;
    return k;
  };
  op.epsc.clear();
  op.kint.clear();
  op.mur.clear();
  for (int64_t o = 0; o < m.nobj; ++o) {
    const bem_material& mt = prob.obj[o];
    cd e = cd(mt.eps_r.re, mt.eps_r.im) - cd(0, mt.sigma / (w * kEps0));
    if (std::abs(e) == 0 || !std::isfinite(e.real()) || !std::isfinite(e.imag()) || !(mt.mu_r > 0))
      throw Error(BEM_E_INVALID, "invalid material of object " + std::to_string(o));
    op.epsc.push_back(e);
    op.mur.push_back(mt.mu_r);
    op.kint.push_back(wavenumber(e, mt.mu_r));
  }
  op.eps_bg = cd(prob.eps_bg.re, prob.eps_bg.im);
  op.mu_bg = prob.mu_bg;
  if (std::abs(op.eps_bg) == 0 || !(op.mu_bg > 0)) throw Error(BEM_E_INVALID, "invalid background medium");
  op.kbg = wavenumber(op.eps_bg, op.mu_bg);
  if (prob.formulation != BEM_FORM_SLDM && prob.formulation != BEM_FORM_EAEFIE)
    throw Error(BEM_E_INVALID, "unknown formulation");
  op.formulation = prob.formulation;
  const bool eaefie = op.formulation == BEM_FORM_EAEFIE;
  op.geo_rep.assign(m.nobj, 0);
  op.mat_rep.assign(m.nobj, 0);
  for (int64_t o = 0; o < m.nobj; ++o) {
    op.geo_rep[o] = prob.no_reuse ? o : m.geo_proto[o];
    op.mat_rep[o] = o;
    for (int64_t p = op.geo_rep[o]; p < o; ++p)
      if (op.geo_rep[p] == op.geo_rep[o] && op.mat_rep[p] == p && op.epsc[p] == op.epsc[o] && op.mur[p] == op.mur[o]) {
        op.mat_rep[o] = p;
        break;
      }
  }

  op.ne = m.ne;
  op.nt = m.nt;
  op.nobj = m.nobj;
  op.nq = m.nt - m.nobj;
  op.N = 2 * op.ne + op.nq;
  op.Neq = op.ne + op.nq;
  op.obj_tri = m.obj_tri;
  op.obj_edge = m.obj_edge;
  op.obj_q.assign(m.nobj + 1, 0);
  for (int64_t o = 0; o < m.nobj; ++o) op.obj_q[o + 1] = m.obj_tri[o + 1] - (o + 1);

  // ---- geometry table
  const int64_t nt = m.nt;
  std::vector<double> geo(size_t(kGeoFields) * nt);
  for (int64_t t = 0; t < nt; ++t) {
    double V[3][3], c[3];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) V[i][k] = m.xyz[3 * m.tri[3 * t + i] + k];
    for (int k = 0; k < 3; ++k) c[k] = m.centroid[3 * t + k];
    for (int k = 0; k < 3; ++k) geo[(kGeoC + k) * nt + t] = c[k];
    for (int q = 0; q < 7; ++q)
      for (int k = 0; k < 3; ++k)
        geo[(kGeoQ + 3 * q + k) * nt + t] =
            R.b7[q][0] * V[0][k] + R.b7[q][1] * V[1][k] + R.b7[q][2] * V[2][k] - c[k];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) geo[(kGeoP + 3 * i + k) * nt + t] = V[i][k] - c[k];
    geo[kGeoA * nt + t] = m.area[t];
    for (int k = 0; k < 3; ++k) geo[(kGeoN + k) * nt + t] = m.normal[3 * t + k];
    geo[kGeoH * nt + t] = m.hmax[t];
  }
  op.geo = op.mem.upload(geo);
  op.tp = op.mem.upload(m.tp);
  op.tm = op.mem.upload(m.tm);
  op.ip = op.mem.upload(m.ip);
  op.im = op.mem.upload(m.im);
  op.tri_edge = op.mem.upload(m.tri_edge);
  op.tri_sign = op.mem.upload(m.tri_sign);
  op.obj_tri_d = op.mem.upload(m.obj_tri);
  std::vector<int32_t> kept;
  for (int64_t o = 0; o < m.nobj; ++o)
    for (int64_t t = m.obj_tri[o]; t < m.obj_tri[o + 1] - 1; ++t) kept.push_back(int32_t(t));
  op.kept = op.mem.upload(kept);
  std::vector<double2> einv(m.ne);
  for (int64_t n = 0; n < m.ne; ++n) einv[n] = c2(1.0 / op.epsc[m.obj[m.tp[n]]]);
  op.eps_inv_edge = op.mem.upload(einv);

  mark("geometry+uploads");
  // ---- Gram matrix I_x: int (n x f_m) . g_n dS, exact with the 3-point rule on every sub-triangle
  // (host work, run while the fill kernels are on the GPU: called once they are enqueued)
  std::vector<double> ixdiag(m.ne, 0.0);
  auto build_ix = [&]() {
    // rows collect (column, value) pairs in fixed-capacity slots: the columns of row m are the
    // BC functions of the dual cells of the (at most four) vertices of T+(m) and T-(m)
    const int cap = 4 * cdat.maxv + 4;
    std::vector<int32_t> rcnt(m.ne, 0), rcol(size_t(m.ne) * cap);
    std::vector<double> rval(size_t(m.ne) * cap);
    auto add = [&](int32_t row, int32_t col, double v) {
      int32_t* c = &rcol[size_t(row) * cap];
      double* x = &rval[size_t(row) * cap];
      int k = 0;
      while (k < rcnt[row] && c[k] != col) ++k;
      if (k == rcnt[row]) {
        if (k == cap) throw Error(BEM_E_MESH, "I_x row wider than the dual-cell bound");
        c[k] = col;
        x[k] = 0.0;
        ++rcnt[row];
      }
      x[k] += v;
    };
    const int64_t nc = cdat.ncell;
    const int ns = 2 * cdat.maxv;
    for (int64_t v = 0; v < nc; ++v) {
      const int N = cdat.nval[v];
      const double* pv = &cdat.vpos[3 * v];
      for (int b = 0; b < N; ++b) {
        const int32_t n = m.vedge[m.vptr[v] + b];
        const double al = cdat.alpha[size_t(b) * nc + v];
        for (int s = 0; s < 2 * N; ++s) {
          const size_t so = size_t(s) * nc + v;
          const int32_t P = cdat.sub_parent[so];
          const double* sm = &cdat.sub_m[3 * so];
          const double* sc = &cdat.sub_c[3 * so];
          const double As = cdat.sub_area[so];
          const double* be = &cdat.beta[((size_t(b) * ns + s) * nc + v) * 3];
          const double* nP = &m.normal[3 * P];
          double acc[3] = {0.0, 0.0, 0.0};
          for (int j = 0; j < 3; ++j) {
            double rl[3], r[3], g[3];
            for (int k = 0; k < 3; ++k) {
              rl[k] = R.b3[j][1] * sm[k] + R.b3[j][2] * sc[k];  // relative to v
              r[k] = pv[k] + rl[k];
              g[k] = (al * rl[k] - be[k]) / (2 * As);
            }
            for (int i = 0; i < 3; ++i) {
              const double sg = m.tri_sign[3 * P + i];
              const double* pi = &m.xyz[3 * m.tri[3 * P + i]];
              double f[3], nf[3];
              for (int k = 0; k < 3; ++k) f[k] = sg * (r[k] - pi[k]) / (2 * m.area[P]);
              nf[0] = nP[1] * f[2] - nP[2] * f[1];
              nf[1] = nP[2] * f[0] - nP[0] * f[2];
              nf[2] = nP[0] * f[1] - nP[1] * f[0];
              acc[i] += As * (1.0 / 3.0) * (nf[0] * g[0] + nf[1] * g[1] + nf[2] * g[2]);
            }
          }
          for (int i = 0; i < 3; ++i) add(m.tri_edge[3 * P + i], n, acc[i]);
        }
      }
    }
    std::vector<int64_t> ptr(m.ne + 1, 0);
    std::vector<int32_t> idx;
    std::vector<double> val;
    idx.reserve(size_t(m.ne) * 24);
    val.reserve(size_t(m.ne) * 24);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t r = 0; r < m.ne; ++r) {
      row.clear();
      for (int k = 0; k < rcnt[r]; ++k) row.emplace_back(rcol[size_t(r) * cap + k], rval[size_t(r) * cap + k]);
      std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (auto& kv : row) {
        idx.push_back(kv.first);
        val.push_back(kv.second);
        if (kv.first == r) ixdiag[r] = kv.second;
      }
      ptr[r + 1] = int64_t(idx.size());
    }
    op.ix_ptr = op.mem.upload(ptr);
    op.ix_idx = op.mem.upload(idx);
    op.ix_val = op.mem.upload(val);
  };

  // ---- near-pair lists (all pairs, and per object) for L, near cells per object for K~
  std::vector<int32_t> na_t, na_s;
  std::vector<std::vector<int32_t>> no_t(m.nobj), no_s(m.nobj);
  na_t.reserve(m.near_idx.size());
  na_s.reserve(m.near_idx.size());
  if (m.nobj == 1) {
    no_t[0].reserve(m.near_idx.size());
    no_s[0].reserve(m.near_idx.size());
  }
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t p = m.near_ptr[t]; p < m.near_ptr[t + 1]; ++p) {
      const int32_t s = m.near_idx[p];
      na_t.push_back(int32_t(t));
      na_s.push_back(s);
      if (m.obj[s] == m.obj[t]) {
        no_t[m.obj[t]].push_back(int32_t(t));
        no_s[m.obj[t]].push_back(s);
      }
    }
  std::vector<int64_t> ncp;
  std::vector<int32_t> nci;
  near_cells(m, ncp, nci);
  std::vector<int32_t> vobj(m.nv, -1);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) vobj[m.tri[3 * t + i]] = m.obj[t];
  std::vector<std::vector<int32_t>> nc_t(m.nobj), nc_c(m.nobj);
  if (m.nobj == 1) {
    nc_t[0].reserve(nci.size());
    nc_c[0].reserve(nci.size());
  }
  for (int64_t t = 0; t < nt; ++t)
    for (int64_t p = ncp[t]; p < ncp[t + 1]; ++p)
      if (vobj[nci[p]] == m.obj[t]) {
        nc_t[m.obj[t]].push_back(int32_t(t));
        nc_c[m.obj[t]].push_back(nci[p]);
      }
  // eAEFIE: near (triangle, cell) pairs of every test triangle with the cells of each object
  std::vector<std::vector<int32_t>> ncm_t(eaefie ? m.nobj : 0), ncm_c(eaefie ? m.nobj : 0);
  if (eaefie)
    for (int64_t t = 0; t < nt; ++t)
      for (int64_t p = ncp[t]; p < ncp[t + 1]; ++p) {
        ncm_t[vobj[nci[p]]].push_back(int32_t(t));
        ncm_c[vobj[nci[p]]].push_back(nci[p]);
      }

  mark("near lists");
  // ---- cell tables
  int32_t* d_cells = op.mem.upload(cdat.obj_cells);
  int32_t* d_nval = op.mem.upload(cdat.nval);
  double* d_vpos = op.mem.upload(cdat.vpos);
  int64_t* d_col0 = op.mem.upload(cdat.col0);
  double* d_sub_m = op.mem.upload(cdat.sub_m);
  double* d_sub_c = op.mem.upload(cdat.sub_c);
  double* d_sub_area = op.mem.upload(cdat.sub_area);
  int32_t* d_sub_parent = op.mem.upload(cdat.sub_parent);
  double* d_alpha = op.mem.upload(cdat.alpha);
  double* d_beta = op.mem.upload(cdat.beta);
  std::vector<int32_t> hp(m.ne), hm(m.ne), cS(m.ne), cT(m.ne);
  for (int64_t n = 0; n < m.ne; ++n) {
    hp[n] = int32_t(3 * m.tp[n] + m.ip[n]);
    hm[n] = int32_t(3 * m.tm[n] + m.im[n]);
    cS[n] = int32_t(cdat.colS[n]);
    cT[n] = int32_t(cdat.colT[n]);
  }
  int32_t* d_hp = op.mem.upload(hp);
  int32_t* d_hm = op.mem.upload(hm);
  int32_t* d_cS = op.mem.upload(cS);
  int32_t* d_cT = op.mem.upload(cT);
  int64_t* d_near_ptr = op.mem.upload(m.near_ptr);
  int32_t* d_near_idx = op.mem.upload(m.near_idx);

  mark("cell tables");
  // ---- nested-solve mode
  int64_t max_neq = 0;
  for (int64_t o = 0; o < m.nobj; ++o)
    max_neq = std::max(max_neq, (m.obj_edge[o + 1] - m.obj_edge[o]) + (m.obj_tri[o + 1] - m.obj_tri[o]) - 1);
  int64_t max_ne = 0;
  for (int64_t o = 0; o < m.nobj; ++o) max_ne = std::max(max_ne, m.obj_edge[o + 1] - m.obj_edge[o]);
  const double hmax = *std::max_element(m.hmax.begin(), m.hmax.end());
  op.inner_mode = eaefie ? kInnerNone : prob.inner_mode;
  if (op.inner_mode == BEM_INNER_AUTO) {
    // charge elimination while the elements are not electrically tiny (its k0^-2 term sets the
    // conditioning), the augmented inverse below that, nested GMRES for very large objects
    const double kh = std::abs(op.kbg) * hmax;
    if (kh >= kSchurMinKh && max_ne <= 32768) op.inner_mode = BEM_INNER_SCHUR;
    else if (max_neq <= 16384) op.inner_mode = BEM_INNER_DIRECT;
    else op.inner_mode = BEM_INNER_GMRES;
  }
  if (op.inner_mode != BEM_INNER_DIRECT && op.inner_mode != BEM_INNER_GMRES && op.inner_mode != BEM_INNER_SCHUR &&
      !(eaefie && op.inner_mode == kInnerNone))
    throw Error(BEM_E_INVALID, "unknown inner_mode");
  // ---- dense blocks
  const bool f32 = op.precision != BEM_FP64;
  op.LA_int.clear();
  op.Lphi_int.clear();
  op.K_int.clear();
  op.K_bg.clear();
  for (int64_t o = 0; o < m.nobj; ++o) {
    const int64_t neo = m.obj_edge[o + 1] - m.obj_edge[o];
    const int64_t nto = m.obj_tri[o + 1] - m.obj_tri[o];
    const int64_t mr = op.mat_rep[o], gr = op.geo_rep[o];
    op.LA_int.push_back(mr == o ? alloc_dense(op.mem, neo, neo, f32) : op.LA_int[mr]);
    op.Lphi_int.push_back(mr == o ? alloc_dense(op.mem, nto, nto, f32) : op.Lphi_int[mr]);
    op.K_int.push_back(mr == o ? alloc_dense(op.mem, neo, neo, f32) : op.K_int[mr]);
    if (!eaefie) op.K_bg.push_back(gr == o ? alloc_dense(op.mem, neo, neo, f32) : op.K_bg[gr]);
  }
  op.LA_bg = alloc_dense(op.mem, m.ne, m.ne, f32);
  op.Lphi_bg = alloc_dense(op.mem, nt, nt, f32);
  op.Km = Dense{};
  if (eaefie) {
    op.Km = alloc_dense(op.mem, m.ne, m.ne, f32);
    for (int64_t o = 0; o < m.nobj; ++o) {
      const int64_t e0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - e0;
      Dense v;
      v.d64 = op.Km.d64 + e0 * op.Km.ld + e0;
      v.d32 = op.Km.d32 ? op.Km.d32 + e0 * op.Km.ld + e0 : nullptr;
      v.rows = v.cols = neo;
      v.ld = op.Km.ld;
      op.K_bg.push_back(v);
    }
  }

  // scratch for the half-RWG and cell-expanded matrices of one chunk of test triangles: every
  // fill runs over chunks of at most ct test triangles of its test range (boundaries fixed by
  // the mesh alone, so every assembly of a mesh sums its entries the same way)
  int64_t row_len = 3 * nt;
  for (int64_t o = 0; o < m.nobj; ++o) row_len = std::max<int64_t>(row_len, cdat.obj_ncol[o]);
  const int64_t ct = fill_chunk_triangles(nt, row_len);
  const int64_t scratch_elems = 3 * ct * row_len;
  double2* H = op.mem.alloc<double2>(size_t(scratch_elems));
  // BEM_POISON=1 fills the fill scratch with NaN first, so that a read of an entry the fill
  // kernels did not write shows up in the blocks (a check used by the tests)
  if (const char* e = std::getenv("BEM_POISON"); e && *e == '1')
    BEM_HIP(hipMemsetAsync(H, 0xFF, sizeof(double2) * size_t(scratch_elems), st));

  hipEvent_t ev0, ev1;
  BEM_HIP(hipEventCreate(&ev0));
  BEM_HIP(hipEventCreate(&ev1));
  BEM_HIP(hipEventRecord(ev0, st));
  std::vector<void*> tmp_dev;
  auto up32 = [&](const std::vector<int32_t>& v) {
    int32_t* p = op.mem.upload(v);
    tmp_dev.push_back(p);
    return p;
  };
  // test triangles per block of a far-fill launch: 8 (the per-source set-up is shared by 8
  // rows), fewer while that leaves under 2048 blocks (small meshes: one CU per block row
  // would leave most of the GPU idle).  Each entry is computed the same way in any chunking.
  auto tchunk_for = [](int64_t nsrc, int64_t per_block, int64_t ntest) {
    const int64_t bx = (nsrc + per_block - 1) / per_block;
    return std::max<int64_t>(1, std::min<int64_t>(8, bx * ntest / 2048));
  };
  // source triangles [s0, s0 + ns) of which some need their rules subdivided at k (the
  // barycentric sub-triangles are smaller than their parents, so this covers K~ as well)
  auto needs_sub = [&](cd k, int64_t s0, int64_t ns) {
    double h = 0;
    for (int64_t t = s0; t < s0 + ns; ++t) h = std::max(h, m.hmax[t]);
    return subdiv_level_host(k.real(), h) > 0 ? 1 : 0;
  };
  // near pairs of a list sorted by test triangle whose test triangle lies in [lo, hi)
  auto pair_span = [](const std::vector<int32_t>& tl, int64_t lo, int64_t hi) {
    const auto b = std::lower_bound(tl.begin(), tl.end(), int32_t(lo));
    const auto e = std::lower_bound(b, tl.end(), int32_t(hi));
    return std::make_pair(int64_t(b - tl.begin()), int64_t(e - b));
  };
  // rows (edges e0 + r, r < nrow) with a half-RWG on a test triangle in [lo, hi), uploaded without
  // waiting for the stream (the host copies live until the fills have run), so that the launches
  // of the chunks follow each other and the host work below overlaps them
  std::deque<std::vector<int32_t>> row_lists;
  auto chunk_rows = [&](int64_t e0, int64_t nrow, int64_t lo, int64_t hi, int64_t* count) -> int32_t* {
    std::vector<int32_t> r;
    for (int64_t n = 0; n < nrow; ++n) {
      const int64_t tp = m.tp[e0 + n], tm = m.tm[e0 + n];
      if ((tp >= lo && tp < hi) || (tm >= lo && tm < hi)) r.push_back(int32_t(n));
    }
    *count = int64_t(r.size());
    if (r.empty()) return nullptr;
    row_lists.push_back(std::move(r));
    const std::vector<int32_t>& h = row_lists.back();
    int32_t* d = op.mem.alloc<int32_t>(h.size());
    tmp_dev.push_back(d);
    BEM_HIP(hipMemcpyAsync(d, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, st));
    return d;
  };
  // background L^A, L^phi (the coupling blocks; the nested-solve inverses are formed from them)
  {
    int32_t* pt = up32(na_t);
    int32_t* ps = up32(na_s);
    const int sub = needs_sub(op.kbg, 0, nt);
    for (int64_t c0 = 0; c0 < nt; c0 += ct) {
      const int64_t c1 = std::min(nt, c0 + ct);
      const auto [p0, np] = pair_span(na_t, c0, c1);
      FillLArgs la{op.geo, nt, c0, c1 - c0, 0, nt, tchunk_for(nt, 256, c1 - c0), op.kbg.real(), op.kbg.imag(), H,
                   3 * nt, op.Lphi_bg.d64 + c0 * op.Lphi_bg.ld, op.Lphi_bg.ld};
      la.sub = sub;
      launch_fill_L(la, pt + p0, ps + p0, np, st);
      int64_t nr = 0;
      const int32_t* rows = chunk_rows(0, m.ne, c0, c1, &nr);
      launch_gather_LA_rows(H, 3 * nt, d_hp, d_hm, 3 * c0, 3 * c1, 0, m.ne, rows, nr, op.LA_bg.d64, op.LA_bg.ld, st);
    }
  }
  for (int64_t o = 0; o < m.nobj; ++o) {
    const int64_t t0 = m.obj_tri[o], nto = m.obj_tri[o + 1] - t0;
    const int64_t e0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - e0;
    const bool own_int = op.mat_rep[o] == o, own_bg = op.geo_rep[o] == o && !eaefie;
    if (!own_int && !own_bg) continue;  // a translated copy: every object-local block is shared
    // interior L^A, L^phi at k_int
    if (own_int) {
      int32_t* pt = up32(no_t[o]);
      int32_t* ps = up32(no_s[o]);
      const int sub = needs_sub(op.kint[o], t0, nto);
      for (int64_t c0 = t0; c0 < t0 + nto; c0 += ct) {
        const int64_t c1 = std::min(t0 + nto, c0 + ct);
        const auto [p0, np] = pair_span(no_t[o], c0, c1);
        FillLArgs la{op.geo, nt, c0, c1 - c0, t0, nto, tchunk_for(nto, 256, c1 - c0), op.kint[o].real(),
                     op.kint[o].imag(), H, 3 * nto, op.Lphi_int[o].d64 + (c0 - t0) * op.Lphi_int[o].ld,
                     op.Lphi_int[o].ld};
        la.sub = sub;
        launch_fill_L(la, pt + p0, ps + p0, np, st);
        int64_t nr = 0;
        const int32_t* rows = chunk_rows(e0, neo, c0, c1, &nr);
        launch_gather_LA_rows(H, 3 * nto, d_hp + e0, d_hm + e0, 3 * c0, 3 * c1, 3 * t0, neo, rows, nr,
                              op.LA_int[o].d64, op.LA_int[o].ld, st);
      }
    }
    // K~ at k_int and at k_bg (object-local blocks)
    int32_t* pct = up32(nc_t[o]);
    int32_t* pcc = up32(nc_c[o]);
    for (int which = 0; which < 2; ++which) {
      if (which == 0 && !own_int) continue;
      // eAEFIE: K~ at k_l is filled below over every test triangle (K_bg[o] are views of it)
      if (which == 1 && !own_bg) break;
      const cd k = which == 0 ? op.kint[o] : op.kbg;
      Dense& dst = which == 0 ? op.K_int[o] : op.K_bg[o];
      const int64_t ncell_o = cdat.obj_cell_ptr[o + 1] - cdat.obj_cell_ptr[o];
      const int sub = needs_sub(k, t0, nto);
      for (int64_t c0 = t0; c0 < t0 + nto; c0 += ct) {
        const int64_t c1 = std::min(t0 + nto, c0 + ct);
        const auto [p0, np] = pair_span(nc_t[o], c0, c1);
        FillKArgs ka{op.geo, nt, c0, c1 - c0, tchunk_for(ncell_o, 128, c1 - c0), k.real(), k.imag(),
                     d_cells + cdat.obj_cell_ptr[o], ncell_o, cdat.ncell, d_nval, d_vpos, d_col0, d_sub_m, d_sub_c,
                     d_sub_area, d_sub_parent, d_alpha, d_beta, H, cdat.obj_ncol[o]};
        ka.sub = sub;
        ka.valence = m.max_valence;
        launch_fill_K(ka, pct + p0, pcc + p0, np, d_near_ptr, d_near_idx, cdat.maxv, st);
        int64_t nr = 0;
        const int32_t* rows = chunk_rows(e0, neo, c0, c1, &nr);
        launch_gather_K_rows(H, cdat.obj_ncol[o], d_hp + e0, d_hm + e0, 3 * c0, 3 * c1, d_cS + e0, d_cT + e0, neo,
                             rows, nr, dst.d64, dst.ld, st);
      }
    }
  }
  if (eaefie) {
    // K~_m (Sec. II-F): every test triangle against the BC cells of object o, at k_l; rows are
    // all edges, columns the edges of object o
    for (int64_t o = 0; o < m.nobj; ++o) {
      const int64_t e0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - e0;
      int32_t* pct = up32(ncm_t[o]);
      int32_t* pcc = up32(ncm_c[o]);
      const int64_t ncell_o = cdat.obj_cell_ptr[o + 1] - cdat.obj_cell_ptr[o];
      const int sub = needs_sub(op.kbg, m.obj_tri[o], m.obj_tri[o + 1] - m.obj_tri[o]);
      for (int64_t c0 = 0; c0 < nt; c0 += ct) {
        const int64_t c1 = std::min(nt, c0 + ct);
        const auto [p0, np] = pair_span(ncm_t[o], c0, c1);
        FillKArgs ka{op.geo, nt, c0, c1 - c0, tchunk_for(ncell_o, 128, c1 - c0), op.kbg.real(), op.kbg.imag(),
                     d_cells + cdat.obj_cell_ptr[o], ncell_o, cdat.ncell, d_nval, d_vpos, d_col0, d_sub_m, d_sub_c,
                     d_sub_area, d_sub_parent, d_alpha, d_beta, H, cdat.obj_ncol[o]};
        ka.sub = sub;
        ka.valence = m.max_valence;
        launch_fill_K(ka, pct + p0, pcc + p0, np, d_near_ptr, d_near_idx, cdat.maxv, st);
        int64_t nr = 0;
        const int32_t* rows = chunk_rows(0, m.ne, c0, c1, &nr);
        launch_gather_K_rows(H, cdat.obj_ncol[o], d_hp, d_hm, 3 * c0, 3 * c1, d_cS + e0, d_cT + e0, neo, rows, nr,
                             op.Km.d64 + e0, op.Km.ld, st);
      }
    }
  }
  if (f32) {
    for (int64_t o = 0; o < m.nobj; ++o) {
      if (op.mat_rep[o] == o) {
        to_f32(op.LA_int[o], st);
        to_f32(op.Lphi_int[o], st);
        to_f32(op.K_int[o], st);
      }
      if (!eaefie && op.geo_rep[o] == o) to_f32(op.K_bg[o], st);
    }
    if (eaefie) to_f32(op.Km, st);
    to_f32(op.LA_bg, st);
    to_f32(op.Lphi_bg, st);
  }
  BEM_HIP(hipEventRecord(ev1, st));
  build_ix();
  BEM_HIP(hipStreamSynchronize(st));
  float ms = 0;
  BEM_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  op.fill_seconds = ms * 1e-3;
  op.fill_bytes = 16.0 * (double(m.ne) * m.ne + double(nt) * nt);
  op.kernel_evals = 49.0 * double(nt) * nt;
  for (int64_t o = 0; o < m.nobj; ++o) {
    const double neo = double(m.obj_edge[o + 1] - m.obj_edge[o]), nto = double(m.obj_tri[o + 1] - m.obj_tri[o]);
    const double n_int = op.mat_rep[o] == o ? 1 : 0, n_bg = (op.geo_rep[o] == o && !eaefie) ? 1 : 0;
    op.fill_bytes += 16.0 * (n_int * (2 * neo * neo + nto * nto) + n_bg * neo * neo);
    op.kernel_evals += n_int * (49.0 + 126.0) * nto * nto + n_bg * 126.0 * nto * nto;
  }
  if (eaefie) {
    op.fill_bytes += 16.0 * double(m.ne) * m.ne;
    op.kernel_evals += 126.0 * double(nt) * nt;
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  op.mem.release(H);
  for (void* p : tmp_dev) op.mem.release(p);
  for (void* p : {(void*)d_cells, (void*)d_nval, (void*)d_vpos, (void*)d_col0, (void*)d_sub_m, (void*)d_sub_c,
                  (void*)d_sub_area, (void*)d_sub_parent, (void*)d_alpha, (void*)d_beta, (void*)d_hp, (void*)d_hm,
                  (void*)d_cS, (void*)d_cT, (void*)d_near_ptr, (void*)d_near_idx})
    op.mem.release(p);

  mark("fill (and I_x on the host)");
  op.precond = prob.precond != 0;
  build_inner_and_precond(op, ixdiag, st, 1);
  build_inner_and_precond(op, ixdiag, st, 2);

  mark("inner+precond");
  if (op.precision == BEM_FP32) drop_f64_blocks(op);
  // ---- work vectors and Krylov spaces
  op.work_len = int64_t(kWorkFields) * work_ld(op);
  op.work = op.mem.alloc<double2>(size_t(op.work_len));
  if (op.inner_mode == BEM_INNER_GMRES) {
    op.inner_ws = make_gmres_work(op.mem, op.Neq, op.inner_restart);
    op.inner_ws->tag = nullptr;
  }
  mark("work");
}

// Direct inner solve (inverse of M_eq per object) and the block preconditioners: the per-edge
// 2x2 inverses and the charge Schur complements of eq. pcext (final system) and of its
// equivalent-configuration counterpart, both inverted on the device.
void build_inner_and_precond(OpObj& op, const std::vector<double>& ixdiag, hipStream_t st, int part) {
  const Mesh& m = *op.m;
  auto tmark = std::chrono::steady_clock::now();
  auto mark = [&](const char* what) {
    if (!timing()) return;
    BEM_HIP(hipStreamSynchronize(st));
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[bem]   %-28s %8.2f ms\n", what, std::chrono::duration<double, std::milli>(now - tmark).count());
    tmark = now;
  };
  const bool f32 = op.precision != BEM_FP64;
  int64_t maxn = 0;
  for (int64_t o = 0; o < m.nobj; ++o)
    maxn = std::max(maxn, (m.obj_edge[o + 1] - m.obj_edge[o]) + (m.obj_tri[o + 1] - m.obj_tri[o]) - 1);
  std::vector<void*> tmp;
  auto talloc = [&](size_t n) {
    double2* p = op.mem.alloc<double2>(n);
    tmp.push_back(p);
    return p;
  };
  DenseScratch ds = dense_scratch_at(talloc(dense_scratch_elems(maxn)), maxn);
  // every inverse is checked (pivots, probe vector); a broken-down elimination fails the assembly
  auto checked = [&](const char* what, int64_t o) {
    const DenseHealth h = dense_health(ds, st);
    op.inv_min_pivot = std::min(op.inv_min_pivot, std::isnan(h.min_pivot_ratio) ? 0.0 : h.min_pivot_ratio);
    op.inv_probe_err = std::max(op.inv_probe_err, std::isnan(h.probe_error) ? HUGE_VAL : h.probe_error);
    if (!dense_health_ok(h)) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "inversion of %s of object %lld broke down (no pivoting): smallest pivot ratio %.3e, "
                    "probe error %.3e",
                    what, (long long)o, h.min_pivot_ratio, h.probe_error);
      throw Error(BEM_E_NUMERIC, msg);
    }
  };
  // diagonals through a gather kernel and a stream-ordered copy (complete on return)
  const int64_t nbuf = std::max(std::max(m.ne, m.nt), maxn);
  double2* dbuf = talloc(size_t(nbuf));
  auto diag_of = [&](const Dense& A) {
    std::vector<double2> d(A.rows);
    launch_diag(A.d64, A.ld, A.rows, dbuf, st);
    BEM_HIP(hipMemcpyAsync(d.data(), dbuf, sizeof(double2) * A.rows, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    return d;
  };
  auto cdv = [](double2 v) { return cd(v.x, v.y); };
  // Inversion of an equilibrated matrix: M' = diag(r) M diag(c) is inverted in place and turned
  // back into M^-1 = diag(c) M'^-1 diag(r).  The scales change only the rounding: the blocks of
  // M_eq differ by many orders of magnitude on graded meshes of small objects (|L^A| ~ h,
  // |L^phi| ~ 1/h), and Gauss-Jordan without pivoting needs them balanced.
  // (on the device, without host round trips)
  double* rdev = reinterpret_cast<double*>(talloc(size_t(nbuf)));
  double* cdev = reinterpret_cast<double*>(talloc(size_t(nbuf)));
  double* udev = reinterpret_cast<double*>(talloc(size_t(nbuf)));
  double* odev = reinterpret_cast<double*>(talloc(size_t(nbuf)));
  double* tdev = reinterpret_cast<double*>(talloc(size_t(nbuf)));
  // symmetric Jacobi scaling |diag|^-1/2 (S and the charge Schur complements)
  auto invert_jacobi = [&](Dense& M, int64_t n, const char* what, int64_t o) {
    jacobi_vec(M.d64, M.ld, 0, n, rdev, st);
    scale_rows_cols(M.d64, M.ld, n, n, rdev, rdev, st);
    dense_invert(M.d64, n, M.ld, ds, st);
    checked(what, o);
    scale_rows_cols(M.d64, M.ld, n, n, rdev, rdev, st);
  };
  // M_eq: Jacobi on the edge block, then the charge columns and rows normalised by their
  // largest entries (those of the coupling blocks).  r, c accumulate the total row and column
  // scales; u holds the partial scale of one step, o is all ones.
  auto invert_meq = [&](Dense& M, int64_t neo, int64_t n, int64_t o) {
    const int64_t nq = n - neo;
    fill_vec(rdev, n, 1.0, st);
    fill_vec(odev, n, 1.0, st);
    jacobi_vec(M.d64, M.ld, 0, neo, rdev, st);
    BEM_HIP(hipMemcpyAsync(cdev, rdev, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    scale_rows_cols(M.d64, M.ld, n, n, rdev, cdev, st);
    col_maxabs(M.d64, M.ld, 0, neo, neo, nq, tdev, st);
    fill_vec(udev, neo, 1.0, st);
    recip_vec(tdev, nq, cdev + neo, udev + neo, st);
    scale_rows_cols(M.d64, M.ld, n, n, odev, udev, st);
    row_maxabs(M.d64, M.ld, neo, nq, n, tdev, st);
    recip_vec(tdev, nq, rdev + neo, udev + neo, st);
    scale_rows_cols(M.d64, M.ld, n, n, udev, odev, st);
    dense_invert(M.d64, n, M.ld, ds, st);
    checked("M_eq", o);
    scale_rows_cols(M.d64, M.ld, n, n, cdev, rdev, st);
  };
  if (part == 1) op.Minv.clear();
  if (part == 1 && op.inner_mode == BEM_INNER_DIRECT) {
    for (int64_t o = 0; o < m.nobj; ++o) {
      if (op.geo_rep[o] != o) {  // a translated copy shares the inverse
        const Dense shared = op.Minv[op.geo_rep[o]];
        op.Minv.push_back(shared);
        continue;
      }
      const int64_t t0 = m.obj_tri[o], nto = m.obj_tri[o + 1] - t0;
      const int64_t e0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - e0;
      const int64_t n = neo + nto - 1;
      Dense M = alloc_dense(op.mem, n, n, f32);
      build_meq(op.LA_bg.d64 + e0 * op.LA_bg.ld + e0, op.LA_bg.ld, op.Lphi_bg.d64 + t0 * op.Lphi_bg.ld + t0,
                op.Lphi_bg.ld, op.tp + e0, op.tm + e0, int32_t(t0), neo, nto, c2(op.mu_bg), c2(-1.0 / op.eps_bg),
                op.k0 * op.k0, M.d64, M.ld, st);
      invert_meq(M, neo, n, o);
      to_f32(M, st);
      op.Minv.push_back(M);
    }
  }
  if (part == 1 && op.inner_mode == BEM_INNER_SCHUR) {
    for (int64_t o = 0; o < m.nobj; ++o) {
      if (op.geo_rep[o] != o) {
        const Dense shared = op.Minv[op.geo_rep[o]];
        op.Minv.push_back(shared);
        continue;
      }
      const int64_t t0 = m.obj_tri[o];
      const int64_t e0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - e0;
      Dense S = alloc_dense(op.mem, neo, neo, f32);
      build_s(op.LA_bg.d64 + e0 * op.LA_bg.ld + e0, op.LA_bg.ld, op.Lphi_bg.d64 + t0 * op.Lphi_bg.ld + t0,
              op.Lphi_bg.ld, op.tp + e0, op.tm + e0, int32_t(t0), neo, c2(op.mu_bg),
              c2(-1.0 / (op.eps_bg * op.k0 * op.k0)), S.d64, S.ld, st);
      invert_jacobi(S, neo, "S", o);
      to_f32(S, st);
      op.Minv.push_back(S);
    }
  }
  mark("nested inverses");
  if (part == 1) {
    for (void* p : tmp) op.mem.release(p);
    return;
  }
  op.SigP.clear();
  op.SigEq.clear();
  if (!op.precond) {
    for (void* p : tmp) op.mem.release(p);
    return;
  }
  // diagonals of the dense blocks
  std::vector<double2> dLAbg = diag_of(op.LA_bg), dLpbg = diag_of(op.Lphi_bg);
  std::vector<double2> dLAint(m.ne), dKint(m.ne), dLpint(m.nt);
  for (int64_t o = 0; o < m.nobj; ++o) {
    const int64_t r = op.mat_rep[o];
    if (r != o) {  // shared interior blocks: the same diagonals
      const int64_t neo = m.obj_edge[o + 1] - m.obj_edge[o], nto = m.obj_tri[o + 1] - m.obj_tri[o];
      std::copy_n(dLAint.begin() + m.obj_edge[r], neo, dLAint.begin() + m.obj_edge[o]);
      std::copy_n(dKint.begin() + m.obj_edge[r], neo, dKint.begin() + m.obj_edge[o]);
      std::copy_n(dLpint.begin() + m.obj_tri[r], nto, dLpint.begin() + m.obj_tri[o]);
      continue;
    }
    auto a = diag_of(op.LA_int[o]), k = diag_of(op.K_int[o]), p = diag_of(op.Lphi_int[o]);
    std::copy(a.begin(), a.end(), dLAint.begin() + m.obj_edge[o]);
    std::copy(k.begin(), k.end(), dKint.begin() + m.obj_edge[o]);
    std::copy(p.begin(), p.end(), dLpint.begin() + m.obj_tri[o]);
  }
  const cd inv_epsl = 1.0 / op.eps_bg;
  // the (1,2) block: diag I_x (eq. pcext); for the eAEFIE the diagonal of its C1 = I_x/2 - K~_m
  std::vector<double2> dKm;
  if (op.formulation == BEM_FORM_EAEFIE) dKm = diag_of(op.Km);
  // per-edge 2x2 diagonal block of P and its inverse
  std::vector<double2> W(4 * m.ne), eqd(m.ne);
  for (int64_t n = 0; n < m.ne; ++n) {
    const int o = m.obj[m.tp[n]];
    const cd l11 = op.mu_bg * cdv(dLAbg[n]);
    const cd l12 = dKm.empty() ? cd(ixdiag[n]) : 0.5 * ixdiag[n] - cdv(dKm[n]);
    const cd l21 = op.mur[o] * cdv(dLAint[n]), l22 = -(cdv(dKint[n]) + 0.5 * ixdiag[n]);
    const cd det = l11 * l22 - l12 * l21;
    W[4 * n] = c2(l22 / det);
    W[4 * n + 1] = c2(-l12 / det);
    W[4 * n + 2] = c2(-l21 / det);
    W[4 * n + 3] = c2(l11 / det);
    eqd[n] = c2(1.0 / (op.mu_bg * cdv(dLAbg[n])));
  }
  op.pcW = op.mem.upload(W);
  op.eq_d = op.mem.upload(eqd);
  op.lam_bg = op.mem.upload(dLpbg);
  op.lam_int = op.mem.upload(dLpint);
  mark("diagonals and 2x2 blocks");
  // charge Schur complements, per object (local numbering)
  for (int64_t o = 0; o < m.nobj; ++o) {
    const int64_t t0 = m.obj_tri[o], nto = m.obj_tri[o + 1] - t0, nq = nto - 1;
    const cd inv_epsc = 1.0 / op.epsc[o];
    for (int which = 0; which < 2; ++which) {
      if (which == 1 && op.inner_mode != BEM_INNER_GMRES) break;
      // Sigma_P depends on the interior blocks, Sigma_eq on the background ones only
      std::vector<Dense>& dst = which == 0 ? op.SigP : op.SigEq;
      const int64_t rep = which == 0 ? op.mat_rep[o] : op.geo_rep[o];
      if (rep != o) {
        const Dense shared = dst[rep];
        dst.push_back(shared);
        continue;
      }
      // G[q][t] = sum over the edges n of triangle q: D[q][n] D[t][n] c_n(t), t in {T+(n), T-(n)}
      std::vector<int64_t> ptr(nq + 1, 0);
      std::vector<int32_t> idx;
      std::vector<double2> val;
      for (int64_t q = 0; q < nq; ++q) {
        const int64_t tq = t0 + q;
        std::map<int32_t, cd> row;
        for (int i = 0; i < 3; ++i) {
          const int32_t n = m.tri_edge[3 * tq + i];
          const double s = m.tri_sign[3 * tq + i];
          for (int side = 0; side < 2; ++side) {
            const int32_t t = side == 0 ? m.tp[n] : m.tm[n];
            const double dt = side == 0 ? 1.0 : -1.0;
            cd c;
            if (which == 0) {
              c = cdv(W[4 * n]) * inv_epsl * cdv(dLpbg[t]) + cdv(W[4 * n + 1]) * inv_epsc * cdv(dLpint[t]);
              c = -c;  // Sigma_P = k0^2 I - G B
            } else {
              c = cdv(eqd[n]) * inv_epsl * cdv(dLpbg[t]);  // Sigma_eq = G B - k0^2 I
            }
            row[int32_t(t - t0)] += s * dt * c;
          }
        }
        for (auto& kv : row) {
          idx.push_back(kv.first);
          val.push_back(c2(kv.second));
        }
        ptr[q + 1] = int64_t(idx.size());
      }
      int64_t* dptr = op.mem.upload(ptr);
      int32_t* didx = op.mem.upload(idx);
      double2* dval = op.mem.upload(val);
      Dense S = alloc_dense(op.mem, nq, nq, f32);
      const double k02 = op.k0 * op.k0;
      build_schur(dptr, didx, dval, nq, nto - 1, which == 0 ? c2(k02) : c2(-k02), S.d64, S.ld, st);
      invert_jacobi(S, nq, which == 0 ? "the charge Schur complement" : "the equivalent charge Schur complement", o);
      to_f32(S, st);
      BEM_HIP(hipStreamSynchronize(st));
      op.mem.release(dptr);
      op.mem.release(didx);
      op.mem.release(dval);
      (which == 0 ? op.SigP : op.SigEq).push_back(S);
    }
  }
  for (void* p : tmp) op.mem.release(p);
}

// ----------------------------------------------------------------- products

namespace {
// Work vectors of the products for R columns: column c of a field at field + c * ld.
struct WorkView {
  double2 *rin, *sol, *t1, *z1, *z2, *am, *xw, *mt, *mz;
  double2 *pc_t, *pc_z, *pc_v, *eq_t, *eq_z, *eq_v;
  int64_t ld = 0;
  int R = 1;
  void* gws = nullptr;  // matrix-core GEMM workspace (R > 1)
  size_t gws_bytes = 0;
};
WorkView slice_work(double2* base, int64_t ld, int R) {
  WorkView v;
  double2** f[kWorkFields] = {&v.rin,  &v.sol,  &v.t1,   &v.z1,   &v.z2,   &v.am,   &v.xw,  &v.mt,
                              &v.mz,   &v.pc_t, &v.pc_z, &v.pc_v, &v.eq_t, &v.eq_z, &v.eq_v};
  for (int i = 0; i < kWorkFields; ++i) *f[i] = base + int64_t(i) * R * ld;
  v.ld = ld;
  v.R = R;
  return v;
}

// Column c of a batched view, as a one-column view.
WorkView column_view(const WorkView& w, int c) {
  WorkView v = w;
  double2** f[kWorkFields] = {&v.rin,  &v.sol,  &v.t1,   &v.z1,   &v.z2,   &v.am,   &v.xw,  &v.mt,
                              &v.mz,   &v.pc_t, &v.pc_z, &v.pc_v, &v.eq_t, &v.eq_z, &v.eq_v};
  for (int i = 0; i < kWorkFields; ++i) *f[i] += int64_t(c) * w.ld;
  v.R = 1;
  return v;
}

WorkView views(OpObj& op) { return slice_work(op.work, work_ld(op), 1); }

// Work of R-column products, owned by `mem`.
WorkView batch_views(OpObj& op, DevArena& mem, int R) {
  WorkView v = slice_work(mem.alloc<double2>(size_t(kWorkFields) * R * work_ld(op)), work_ld(op), R);
  if (R > 1) {
    v.gws_bytes = gemm_workspace_bytes(std::max(op.ne, op.nt), R);
    v.gws = mem.alloc<char>(v.gws_bytes);
  }
  return v;
}

// Matrix bytes below which a one- or two-column product is handed to the serving loop's
// combiner (it would not fill the GPU alone).
constexpr double kCombineMaxBytes = 256.0 * 1024 * 1024;

void products(OpObj& op, const std::vector<GemvDesc>& ds, const WorkView& wv, hipStream_t st) {
  const int R = wv.R;
  if (ds.empty()) return;
  if (op.comb && R <= 2) {
    double bytes = 0;
    for (const GemvDesc& d : ds) bytes += double(d.rows) * d.cols * (d.fp32 ? 8.0 : 16.0) * (d.A2 ? 2 : 1);
    if (bytes < kCombineMaxBytes) {
      std::vector<GemvDesc> all;
      for (int r = 0; r < R; ++r)
        for (const GemvDesc& d : ds) {
          GemvDesc c = d;
          c.x = d.x + r * d.ldx;
          if (d.x2) c.x2 = d.x2 + r * d.ldx2;
          c.y = d.y + r * d.ldy;
          all.push_back(c);
        }
      op.comb->run(all, st);
      return;
    }
  }
  launch_products(ds, R, wv.gws, wv.gws_bytes, st);
}

GemvDesc with_ld(GemvDesc d, int64_t ldx, int64_t ldy, int64_t ldx2 = 0) {
  d.ldx = ldx;
  d.ldy = ldy;
  d.ldx2 = ldx2;
  return d;
}

// Block preconditioner of the final system (eq. pcext) applied to the R columns of
// r = [r1; r2; r3] (column stride ld; x likewise):
//   x3 = Sigma_P^-1 (r3 - F D (W11 r1 + W12 r2)),  [x1; x2] = W ([r1; r2] - [S1; S2] x3)
void precond_cols(OpObj& op, const WorkView& wv, const double2* r, double2* x, int64_t ld, bool fp32,
                  hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, L = wv.ld;
  const double2 *r1 = r, *r2 = r + ne, *r3 = r + 2 * ne;
  double2 *x1 = x, *x2 = x + ne, *x3 = x + 2 * ne;
  launch_pc_stage1(op.pcW, r1, r2, ne, wv.pc_t, st, R, ld, L);
  launch_FD(wv.pc_t, op.tri_edge, op.tri_sign, op.kept, op.nq, c2(-1.0), r3, c2(1.0), wv.pc_z, st, R, L, ld, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t q0 = op.obj_q[o], nq = op.obj_q[o + 1] - q0;
    ds.push_back(with_ld(desc(op.SigP[o], fp32, 0, 0, nq, nq, wv.pc_z + q0, x3 + q0, c2(1.0), 0), L, ld));
  }
  products(op, ds, wv, st);
  launch_expand_charge(x3, wv.pc_v, op.obj_tri_d, op.nobj, c2(1.0), st, R, ld, L);
  launch_pc_stage2(op.pcW, r1, r2, wv.pc_v, op.lam_bg, op.lam_int, c2(1.0 / op.eps_bg), op.eps_inv_edge, op.tp,
                   op.tm, ne, x1, x2, st, R, ld, L);
}

// Equivalent-configuration counterpart for the nested GMRES (diagonal L blocks, exact charge
// constraint): x2 = Sigma_eq^-1 (r2 - F D d r1), x1 = d (r1 + eps_l^-1 D^T diag(L^phi_l) B x2)
void precond_eq_cols(OpObj& op, const WorkView& wv, const double2* r, double2* x, int64_t ld, bool fp32,
                     hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, L = wv.ld;
  const double2 *r1 = r, *r2 = r + ne;
  double2 *x1 = x, *x2 = x + ne;
  launch_peq_stage1(op.eq_d, r1, ne, wv.eq_t, st, R, ld, L);
  launch_FD(wv.eq_t, op.tri_edge, op.tri_sign, op.kept, op.nq, c2(-1.0), r2, c2(1.0), wv.eq_z, st, R, L, ld, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t q0 = op.obj_q[o], nq = op.obj_q[o + 1] - q0;
    ds.push_back(with_ld(desc(op.SigEq[o], fp32, 0, 0, nq, nq, wv.eq_z + q0, x2 + q0, c2(1.0), 0), L, ld));
  }
  products(op, ds, wv, st);
  launch_expand_charge(x2, wv.eq_v, op.obj_tri_d, op.nobj, c2(1.0), st, R, ld, L);
  launch_peq_stage2(op.eq_d, wv.eq_t, wv.eq_v, op.lam_bg, c2(1.0 / op.eps_bg), op.tp, op.tm, ne, x1, st, R, ld, L);
}

// Equivalent-configuration matrix (eq. AEFIEeqvdis), block-diagonal over objects:
//   y_u = mu_l L^A_l u - eps_l^-1 D^T L^phi_l B w ;  y_w = F D u - k0^2 w
void meq_cols(OpObj& op, const WorkView& wv, const double2* x, int64_t ldx, double2* y, int64_t ldy, bool fp32,
              hipStream_t st) {
  const int R = wv.R;
  const int64_t L = wv.ld;
  const double2* u = x;
  const double2* w = x + op.ne;
  double2* yu = y;
  double2* yw = y + op.ne;
  launch_expand_charge(w, wv.mt, op.obj_tri_d, op.nobj, c2(1.0), st, R, ldx, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t t0 = op.obj_tri[o], nto = op.obj_tri[o + 1] - t0;
    const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
    ds.push_back(with_ld(desc(op.Lphi_bg, fp32, t0, t0, nto, nto, wv.mt + t0, wv.mz + t0, c2(1.0), 0), L, L));
    ds.push_back(with_ld(desc(op.LA_bg, fp32, e0, e0, neo, neo, u + e0, yu + e0, c2(op.mu_bg), 0), ldx, ldy));
  }
  products(op, ds, wv, st);
  launch_DT(wv.mz, op.tp, op.tm, op.ne, c2(-1.0 / op.eps_bg), nullptr, yu, 1, st, R, L, ldy);
  launch_FD(u, op.tri_edge, op.tri_sign, op.kept, op.nq, c2(1.0), w, c2(-op.k0 * op.k0), yw, st, R, ldx, ldx, ldy);
}

// Nested solve (eq. AEFIEeqvdis) of R columns: [u; w] = M_eq^-1 [r_in; 0] from wv.rin into wv.sol,
// directly (augmented inverse or charge-eliminated S^-1) or by nested GMRES column by column.
void nested_from_rin(OpObj& op, const WorkView& wv, bool fp32, double inner_tol, hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, nq = op.nq, L = wv.ld;
  if (op.inner_mode == BEM_INNER_DIRECT) {
    // [u_o; w_o] = M_eq,o^-1 [r_in,o; 0]: only the edge columns of the inverse are read
    std::vector<GemvDesc> di;
    for (int64_t o = 0; o < op.nobj; ++o) {
      const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
      const int64_t q0 = op.obj_q[o], nqo = op.obj_q[o + 1] - q0;
      di.push_back(with_ld(desc(op.Minv[o], fp32, 0, 0, neo, neo, wv.rin + e0, wv.sol + e0, c2(1.0), 0), L, L));
      di.push_back(
          with_ld(desc(op.Minv[o], fp32, neo, 0, nqo, neo, wv.rin + e0, wv.sol + ne + q0, c2(1.0), 0), L, L));
    }
    products(op, di, wv, st);
    op.last_inner_iters = 0;
  } else if (op.inner_mode == BEM_INNER_SCHUR) {
    // u = S^-1 r_in with the charges eliminated, then w = k0^-2 F D u
    std::vector<GemvDesc> di;
    for (int64_t o = 0; o < op.nobj; ++o) {
      const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
      di.push_back(with_ld(desc(op.Minv[o], fp32, 0, 0, neo, neo, wv.rin + e0, wv.sol + e0, c2(1.0), 0), L, L));
    }
    products(op, di, wv, st);
    launch_FD(wv.sol, op.tri_edge, op.tri_sign, op.kept, nq, c2(1.0 / (op.k0 * op.k0)), nullptr, c2(0.0),
              wv.sol + ne, st, R, L, 0, L);
    op.last_inner_iters = 0;
  } else {
    launch_axpby(nq, c2(0.0), nullptr, c2(0.0), nullptr, wv.rin + ne, st, R, 0, 0, L);
    for (int c = 0; c < R; ++c) {
      const WorkView cv = column_view(wv, c);
      ApplyFn meq = [&op, cv, fp32, st](const double2* xi, double2* yi) { meq_cols(op, cv, xi, 0, yi, 0, fp32, st); };
      ApplyFn peq = [&op, cv, fp32, st](const double2* xi, double2* yi) {
        precond_eq_cols(op, cv, xi, yi, 0, fp32, st);
      };
      GmresResult gr = gmres(*op.inner_ws, op.pinned, meq, cv.rin, cv.sol, true, inner_tol, op.inner_maxit, st,
                             op.precond ? &peq : nullptr);
      op.last_inner_iters = gr.iters;
      op.max_inner_iters = std::max(op.max_inner_iters, gr.iters);
      if (verbose()) std::fprintf(stderr, "[bem] inner its %d res %.3e\n", gr.iters, gr.relres);
    }
  }
}

// eAEFIE counterpart of the final system (Sec. II-F) on R columns, no equivalent problem:
//   y1 = L^A_m a + (I_x/2 - K~_m) e + D^T L^phi_m B x3
//   y2 = mu_r L^A a - (K~ + I_x/2) e + eps_c^-1 D^T L^phi B x3      (as in eq. finalsystem)
//   y3 = F D a + k0^2 x3
void eaefie_cols(OpObj& op, const WorkView& wv, const double2* x, int64_t ldx, double2* y, int64_t ldy, bool fp32,
                 hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, L = wv.ld;
  const double2* a = x;
  const double2* e = x + ne;
  const double2* x3 = x + 2 * ne;
  double2* y1 = y;
  double2* y2 = y + ne;
  double2* y3 = y + 2 * ne;
  launch_expand_charge(x3, wv.t1, op.obj_tri_d, op.nobj, c2(1.0), st, R, ldx, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t t0 = op.obj_tri[o], nto = op.obj_tri[o + 1] - t0;
    const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
    GemvDesc d2 = desc(op.LA_int[o], fp32, 0, 0, neo, neo, a + e0, y2 + e0, c2(op.mur[o]), 0);
    add_second(d2, op.K_int[o], fp32, 0, 0, e + e0, c2(-1.0));
    ds.push_back(with_ld(d2, ldx, ldy, ldx));
    ds.push_back(with_ld(desc(op.Lphi_int[o], fp32, 0, 0, nto, nto, wv.t1 + t0, wv.z1 + t0, c2(1.0), 0), L, L));
  }
  GemvDesc d1 = desc(op.LA_bg, fp32, 0, 0, ne, ne, a, y1, c2(op.mu_bg), 0);
  add_second(d1, op.Km, fp32, 0, 0, e, c2(-1.0));
  ds.push_back(with_ld(d1, ldx, ldy, ldx));
  ds.push_back(with_ld(desc(op.Lphi_bg, fp32, 0, 0, op.nt, op.nt, wv.t1, wv.z2, c2(1.0), 0), L, L));
  products(op, ds, wv, st);
  launch_spmv2(op.ix_ptr, op.ix_idx, op.ix_val, ne, e, ldx, c2(-0.5), y2, ldy, 1, c2(0.5), y1, ldy, 1, st, R);
  launch_DT(wv.z1, op.tp, op.tm, ne, c2(1.0), op.eps_inv_edge, y2, 1, st, R, L, ldy);
  launch_DT(wv.z2, op.tp, op.tm, ne, c2(1.0 / op.eps_bg), nullptr, y1, 1, st, R, L, ldy);
  launch_FD(a, op.tri_edge, op.tri_sign, op.kept, op.nq, c2(1.0), x3, c2(op.k0 * op.k0), y3, st, R, ldx, ldx, ldy);
  op.last_inner_iters = 0;
}

// Final system (eq. finalsystem) on R columns; the nested solve [u; w] = M_eq^-1 [r_in; 0]
// runs for every column (directly, or by nested GMRES column by column).
void final_cols(OpObj& op, const WorkView& wv, const double2* x, int64_t ldx, double2* y, int64_t ldy, bool fp32,
                double inner_tol, hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, nq = op.nq, L = wv.ld;
  const double2* a = x;
  const double2* e = x + ne;
  const double2* x3 = x + 2 * ne;
  double2* y1 = y;
  double2* y2 = y + ne;
  double2* y3 = y + 2 * ne;
  if (op.formulation == BEM_FORM_EAEFIE) {
    eaefie_cols(op, wv, x, ldx, y, ldy, fp32, st);
    return;
  }
  // B x3 for the interior charge term
  launch_expand_charge(x3, wv.t1, op.obj_tri_d, op.nobj, c2(1.0), st, R, ldx, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t t0 = op.obj_tri[o], nto = op.obj_tri[o + 1] - t0;
    const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
    // r_in = K~_l e ;  y2 = mu_r L^A a - K~ e ;  z1 = L^phi B x3
    ds.push_back(with_ld(desc(op.K_bg[o], fp32, 0, 0, neo, neo, e + e0, wv.rin + e0, c2(1.0), 0), ldx, L));
    GemvDesc d2 = desc(op.LA_int[o], fp32, 0, 0, neo, neo, a + e0, y2 + e0, c2(op.mur[o]), 0);
    add_second(d2, op.K_int[o], fp32, 0, 0, e + e0, c2(-1.0));
    ds.push_back(with_ld(d2, ldx, ldy, ldx));
    ds.push_back(with_ld(desc(op.Lphi_int[o], fp32, 0, 0, nto, nto, wv.t1 + t0, wv.z1 + t0, c2(1.0), 0), L, L));
  }
  products(op, ds, wv, st);
  // r_in += I_x e / 2 ; y2 += -I_x e / 2 + eps_c^-1 D^T z1
  launch_spmv2(op.ix_ptr, op.ix_idx, op.ix_val, ne, e, ldx, c2(0.5), wv.rin, L, 1, c2(-0.5), y2, ldy, 1, st, R);
  launch_DT(wv.z1, op.tp, op.tm, ne, c2(1.0), op.eps_inv_edge, y2, 1, st, R, L, ldy);
  nested_from_rin(op, wv, fp32, inner_tol, st);
  const double2* u = wv.sol;
  const double2* w = wv.sol + ne;
  // a - u, x3 + w, B (x3 + w)
  launch_axpby(ne, c2(1.0), a, c2(-1.0), u, wv.am, st, R, ldx, L, L);
  launch_axpby(nq, c2(1.0), x3, c2(1.0), w, wv.xw, st, R, ldx, L, L);
  launch_expand_charge(wv.xw, wv.t1, op.obj_tri_d, op.nobj, c2(1.0), st, R, L, L);
  std::vector<GemvDesc> g2 = {with_ld(desc(op.LA_bg, fp32, 0, 0, ne, ne, wv.am, y1, c2(op.mu_bg), 0), L, ldy),
                              with_ld(desc(op.Lphi_bg, fp32, 0, 0, op.nt, op.nt, wv.t1, wv.z2, c2(1.0), 0), L, L)};
  products(op, g2, wv, st);
  // y1 += eps_l^-1 D^T z2 + I_x e ;  y3 = F D (a - u) + k0^2 (x3 + w)
  launch_DT(wv.z2, op.tp, op.tm, ne, c2(1.0 / op.eps_bg), nullptr, y1, 1, st, R, L, ldy);
  launch_spmv(op.ix_ptr, op.ix_idx, op.ix_val, ne, e, c2(1.0), y1, 1, st, R, ldx, ldy);
  launch_FD(wv.am, op.tri_edge, op.tri_sign, op.kept, nq, c2(1.0), wv.xw, c2(op.k0 * op.k0), y3, st, R, L, L, ldy);
}

}  // namespace

void apply_precond(OpObj& op, const double2* r, double2* x, bool fp32, hipStream_t st) {
  precond_cols(op, views(op), r, x, 0, fp32, st);
}

void apply_precond_eq(OpObj& op, const double2* r, double2* x, bool fp32, hipStream_t st) {
  precond_eq_cols(op, views(op), r, x, 0, fp32, st);
}

void apply_meq(OpObj& op, const double2* x, double2* y, bool fp32, hipStream_t st) {
  meq_cols(op, views(op), x, 0, y, 0, fp32, st);
}

void apply_final(OpObj& op, const double2* x, double2* y, bool fp32, double inner_tol, hipStream_t st) {
  final_cols(op, views(op), x, 0, y, 0, fp32, inner_tol, st);
}

void apply_block(OpObj& op, int block, const double2* x, double2* y, int64_t nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  const int R = int(nrhs);
  DevArena tmp(op.ctx);
  tmp.set_stream(st);
  const WorkView wv = R == 1 ? views(op) : batch_views(op, tmp, R);
  std::vector<GemvDesc> ds;
  switch (block) {
    case BEM_BLOCK_LA_INT:
    case BEM_BLOCK_K_INT:
    case BEM_BLOCK_K_BG:
      for (int64_t o = 0; o < op.nobj; ++o) {
        const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
        const Dense& A = block == BEM_BLOCK_LA_INT ? op.LA_int[o] : block == BEM_BLOCK_K_INT ? op.K_int[o] : op.K_bg[o];
        ds.push_back(with_ld(desc(A, false, 0, 0, neo, neo, x + e0, y + e0, c2(1.0), 0), op.ne, op.ne));
      }
      break;
    case BEM_BLOCK_LPHI_INT:
      for (int64_t o = 0; o < op.nobj; ++o) {
        const int64_t t0 = op.obj_tri[o], nto = op.obj_tri[o + 1] - t0;
        ds.push_back(with_ld(desc(op.Lphi_int[o], false, 0, 0, nto, nto, x + t0, y + t0, c2(1.0), 0), op.nt, op.nt));
      }
      break;
    case BEM_BLOCK_LA_BG:
      ds.push_back(with_ld(desc(op.LA_bg, false, 0, 0, op.ne, op.ne, x, y, c2(1.0), 0), op.ne, op.ne));
      break;
    case BEM_BLOCK_LPHI_BG:
      ds.push_back(with_ld(desc(op.Lphi_bg, false, 0, 0, op.nt, op.nt, x, y, c2(1.0), 0), op.nt, op.nt));
      break;
    case BEM_BLOCK_K_M:
      if (!op.Km.d64 && !op.Km.d32) throw Error(BEM_E_INVALID, "K~_m is formed only by the eAEFIE formulation");
      ds.push_back(with_ld(desc(op.Km, false, 0, 0, op.ne, op.ne, x, y, c2(1.0), 0), op.ne, op.ne));
      break;
    case BEM_BLOCK_IX:
      launch_spmv(op.ix_ptr, op.ix_idx, op.ix_val, op.ne, x, c2(1.0), y, 0, st, R, op.ne, op.ne);
      break;
    case BEM_BLOCK_MEQ:
      meq_cols(op, wv, x, op.Neq, y, op.Neq, false, st);
      break;
    case BEM_BLOCK_FINAL:
      final_cols(op, wv, x, op.N, y, op.N, false, op.inner_tol, st);
      break;
    default:
      throw Error(BEM_E_INVALID, "unknown block");
  }
  products(op, ds, wv, st);
  // the batch work is freed on return: let the launches that read it finish first
  if (R > 1) BEM_HIP(hipStreamSynchronize(st));
}

namespace {
// The equivalent configuration of a solution (eq. AEFIEeqvdis, same E): e = E / eta0 in place,
// r_in = (K~_l + I_x/2) e, [u; w] = M_eq^-1 [r_in; 0] in float64 into wv.sol, and the
// differential current J_delta = H - u / (j k0) in place of h (eq. diffsourcesdis).
void equivalent_solve(OpObj& op, const WorkView& wv, double2* e, double2* h, hipStream_t st) {
  const int R = wv.R;
  const int64_t ne = op.ne, L = wv.ld;
  launch_axpby(ne, c2(1.0 / kEta0), e, c2(0.0), nullptr, e, st, R, L, 0, L);
  std::vector<GemvDesc> ds;
  for (int64_t o = 0; o < op.nobj; ++o) {
    const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0;
    ds.push_back(with_ld(desc(op.K_bg[o], false, 0, 0, neo, neo, e + e0, wv.rin + e0, c2(1.0), 0), L, L));
  }
  products(op, ds, wv, st);
  launch_spmv(op.ix_ptr, op.ix_idx, op.ix_val, ne, e, c2(0.5), wv.rin, 1, st, R, L, L);
  nested_from_rin(op, wv, false, op.inner_tol, st);
  launch_axpby(ne, c2(1.0), h, c2(-cd(1.0) / cd(0.0, op.k0)), wv.sol, h, st, R, L, L, L);
}
}  // namespace

void far_field(OpObj& op, const bem_c64* H, const bem_c64* E, int64_t nexc, const double* rhat, int64_t ndir,
               bem_c64* N, double* rcs, hipStream_t st) {
  if (op.formulation != BEM_FORM_SLDM)
    throw Error(BEM_E_INVALID, "the far field is radiated by the differential current of the proposed formulation");
  if (nexc <= 0 || ndir <= 0 || !H || !E || !rhat) throw Error(BEM_E_INVALID, "invalid far-field arguments");
  for (int64_t d = 0; d < ndir; ++d) {
    const double n2 = rhat[3 * d] * rhat[3 * d] + rhat[3 * d + 1] * rhat[3 * d + 1] + rhat[3 * d + 2] * rhat[3 * d + 2];
    if (!(std::fabs(n2 - 1.0) < 1e-9)) throw Error(BEM_E_INVALID, "directions must be unit vectors");
  }
  const int64_t ne = op.ne;
  const cd eta_l = kEta0 * std::sqrt(op.mu_bg / op.eps_bg);
  const double pref = std::norm(op.kbg * eta_l) / (4.0 * M_PI);
  DevArena tmp(op.ctx);
  tmp.set_stream(st);
  double* d_rhat = tmp.alloc<double>(size_t(3 * ndir));
  BEM_HIP(hipMemcpyAsync(d_rhat, rhat, sizeof(double) * 3 * ndir, hipMemcpyHostToDevice, st));
  std::vector<double2> hN;
  for (int64_t c0 = 0; c0 < nexc; c0 += 256) {
    const int R = int(std::min<int64_t>(256, nexc - c0));
    const WorkView wv = R == 1 ? views(op) : batch_views(op, tmp, R);
    const int64_t L = wv.ld;
    double2* e = tmp.alloc<double2>(size_t(L) * R);
    double2* h = tmp.alloc<double2>(size_t(L) * R);
    double2* out = tmp.alloc<double2>(size_t(3 * ndir) * R);
    for (int c = 0; c < R; ++c) {
      BEM_HIP(hipMemcpyAsync(e + c * L, E + (c0 + c) * ne, sizeof(double2) * ne, hipMemcpyHostToDevice, st));
      BEM_HIP(hipMemcpyAsync(h + c * L, H + (c0 + c) * ne, sizeof(double2) * ne, hipMemcpyHostToDevice, st));
    }
    equivalent_solve(op, wv, e, h, st);
    FarArgs fa{op.geo, op.nt, op.tri_edge, op.tri_sign, h, L, op.kbg.real(), op.kbg.imag(), d_rhat, ndir, out};
    launch_far_field(fa, R, st);
    hN.resize(size_t(3 * ndir) * R);
    BEM_HIP(hipMemcpyAsync(hN.data(), out, sizeof(double2) * hN.size(), hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < R; ++c)
      for (int64_t d = 0; d < ndir; ++d) {
        const double2* v = &hN[(size_t(c) * ndir + d) * 3];
        const cd n[3] = {cd(v[0].x, v[0].y), cd(v[1].x, v[1].y), cd(v[2].x, v[2].y)};
        const double* r = rhat + 3 * d;
        const cd nr = n[0] * r[0] + n[1] * r[1] + n[2] * r[2];
        double s = 0;
        for (int i = 0; i < 3; ++i) {
          const cd perp = n[i] - nr * r[i];
          s += std::norm(perp);
          if (N) N[((c0 + c) * ndir + d) * 3 + i] = {n[i].real(), n[i].imag()};
        }
        if (rcs) rcs[(c0 + c) * ndir + d] = pref * s;
      }
  }
}

void near_field(OpObj& op, const bem_c64* H, const bem_c64* E, const bem_c64* rho, int64_t nexc,
                const bem_excitation* exc, const double* pts, int64_t npts, bem_c64* Eout, bem_c64* Hout,
                hipStream_t st) {
  if (op.formulation != BEM_FORM_SLDM)
    throw Error(BEM_E_INVALID, "the near field is radiated by the differential sources of the proposed formulation");
  if (nexc <= 0 || npts < 0 || !H || !E || !rho || (npts > 0 && !pts))
    throw Error(BEM_E_INVALID, "invalid near-field arguments");
  if (npts == 0) return;
  for (int64_t i = 0; i < 3 * npts; ++i)
    if (!std::isfinite(pts[i])) throw Error(BEM_E_INVALID, "non-finite observation point");
  std::vector<double> inc;
  if (exc) {
    inc.resize(size_t(11 * nexc));
    for (int64_t c = 0; c < nexc; ++c) {
      const bem_excitation& x = exc[c];
      if (x.kind != BEM_EXC_PLANE_WAVE)
        throw Error(BEM_E_INVALID, "the incident field is defined for plane waves only");
      double* w = &inc[size_t(11 * c)];
      for (int i = 0; i < 3; ++i) {
        w[i] = x.khat[i];
        w[3 + i] = x.pol[i].re;
        w[6 + i] = x.pol[i].im;
      }
      w[9] = x.amp.re;
      w[10] = x.amp.im;
    }
  }
  const int64_t ne = op.ne, nt = op.nt;
  const cd eps_l = kEps0 * op.eps_bg;
  const cd jwmu(0.0, op.k0 * kC0 * kMu0 * op.mu_bg);
  const cd inv_eps = 1.0 / eps_l;
  const cd inv_eta = 1.0 / (kEta0 * std::sqrt(op.mu_bg / op.eps_bg));
  DevArena tmp(op.ctx);
  tmp.set_stream(st);
  double* d_pts = tmp.alloc<double>(size_t(3 * npts));
  BEM_HIP(hipMemcpyAsync(d_pts, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, st));
  double* d_inc = nullptr;
  if (exc) {
    d_inc = tmp.alloc<double>(inc.size());
    BEM_HIP(hipMemcpyAsync(d_inc, inc.data(), sizeof(double) * inc.size(), hipMemcpyHostToDevice, st));
  }
  // triangle ranges: about 2048 blocks in all, each range at least 512 triangles
  for (int64_t c0 = 0; c0 < nexc; c0 += 256) {
    const int R = int(std::min<int64_t>(256, nexc - c0));
    const WorkView wv = R == 1 ? views(op) : batch_views(op, tmp, R);
    const int64_t L = wv.ld;
    double2* e = tmp.alloc<double2>(size_t(L) * R);
    double2* h = tmp.alloc<double2>(size_t(L) * R);
    double2* q = tmp.alloc<double2>(size_t(nt) * R);
    for (int c = 0; c < R; ++c) {
      BEM_HIP(hipMemcpyAsync(e + c * L, E + (c0 + c) * ne, sizeof(double2) * ne, hipMemcpyHostToDevice, st));
      BEM_HIP(hipMemcpyAsync(h + c * L, H + (c0 + c) * ne, sizeof(double2) * ne, hipMemcpyHostToDevice, st));
      BEM_HIP(hipMemcpyAsync(q + c * nt, rho + (c0 + c) * nt, sizeof(double2) * nt, hipMemcpyHostToDevice, st));
    }
    equivalent_solve(op, wv, e, h, st);
    // rho_delta = rho - rho_eq, rho_eq = B w / c0 (w: the reduced charges of the equivalent solve)
    double2* qeq = tmp.alloc<double2>(size_t(nt) * R);
    launch_expand_charge(wv.sol + ne, qeq, op.obj_tri_d, op.nobj, c2(1.0 / kC0), st, R, L, nt);
    launch_axpby(nt, c2(1.0), q, c2(-1.0), qeq, q, st, R, nt, nt, nt);
    const int64_t groups = (R + kNearFieldCols - 1) / kNearFieldCols;
    const int64_t want = (2048 + npts * groups - 1) / (npts * groups);
    const int nsplit = int(std::max<int64_t>(1, std::min<int64_t>({want, (nt + 511) / 512, 64})));
    double2* part = tmp.alloc<double2>(size_t(nsplit) * R * npts * 6);
    double2* dE = tmp.alloc<double2>(size_t(R) * npts * 3);
    double2* dH = tmp.alloc<double2>(size_t(R) * npts * 3);
    NearArgs na{op.geo, nt, op.tri_edge, op.tri_sign, h, L, q, nt, R, op.kbg.real(), op.kbg.imag(),
                c2(jwmu), c2(inv_eps), c2(inv_eta), d_pts, npts, d_inc ? d_inc + 11 * c0 : nullptr, nsplit,
                part, dE, dH};
    launch_near_field(na, st);
    if (Eout)
      BEM_HIP(hipMemcpyAsync(Eout + c0 * npts * 3, dE, sizeof(double2) * R * npts * 3, hipMemcpyDeviceToHost, st));
    if (Hout)
      BEM_HIP(hipMemcpyAsync(Hout + c0 * npts * 3, dH, sizeof(double2) * R * npts * 3, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
  }
}

void export_block(OpObj& op, int block, bem_c64* host) {
  // a BEM_FP32 block is widened on the host
  std::vector<float2> row32;
  auto copy_row = [&](const Dense& A, int64_t r, bem_c64* dst) {
    if (A.d64) {
      BEM_HIP(hipMemcpy(dst, A.d64 + r * A.ld, sizeof(double2) * A.cols, hipMemcpyDeviceToHost));
      return;
    }
    row32.resize(size_t(A.cols));
    BEM_HIP(hipMemcpy(row32.data(), A.d32 + r * A.ld, sizeof(float2) * A.cols, hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < A.cols; ++c) dst[c] = {double(row32[c].x), double(row32[c].y)};
  };
  auto copy_dense = [&](const Dense& A, int64_t roff, int64_t coff, int64_t ldh) {
    for (int64_t r = 0; r < A.rows; ++r) copy_row(A, r, host + (roff + r) * ldh + coff);
  };
  BEM_HIP(hipStreamSynchronize(op.stream));
  switch (block) {
    case BEM_BLOCK_LA_INT:
    case BEM_BLOCK_K_INT:
    case BEM_BLOCK_K_BG:
      std::memset(host, 0, sizeof(bem_c64) * op.ne * op.ne);
      for (int64_t o = 0; o < op.nobj; ++o) {
        const Dense& A = block == BEM_BLOCK_LA_INT ? op.LA_int[o] : block == BEM_BLOCK_K_INT ? op.K_int[o] : op.K_bg[o];
        copy_dense(A, op.obj_edge[o], op.obj_edge[o], op.ne);
      }
      return;
    case BEM_BLOCK_LPHI_INT:
      std::memset(host, 0, sizeof(bem_c64) * op.nt * op.nt);
      for (int64_t o = 0; o < op.nobj; ++o) copy_dense(op.Lphi_int[o], op.obj_tri[o], op.obj_tri[o], op.nt);
      return;
    case BEM_BLOCK_LA_BG:
      copy_dense(op.LA_bg, 0, 0, op.ne);
      return;
    case BEM_BLOCK_LPHI_BG:
      copy_dense(op.Lphi_bg, 0, 0, op.nt);
      return;
    case BEM_BLOCK_K_M:
      if (!op.Km.d64 && !op.Km.d32) throw Error(BEM_E_INVALID, "K~_m is formed only by the eAEFIE formulation");
      copy_dense(op.Km, 0, 0, op.ne);
      return;
    case BEM_BLOCK_MEQ_INV: {
      if (op.inner_mode != BEM_INNER_DIRECT) throw Error(BEM_E_INVALID, "M_eq^-1 is formed only by the augmented direct nested solve");
      std::memset(host, 0, sizeof(bem_c64) * op.Neq * op.Neq);
      // object o occupies rows/columns: edges [e0, e0+ne_o) and charges ne + [q0, q0+nq_o)
      for (int64_t o = 0; o < op.nobj; ++o) {
        const Dense& A = op.Minv[o];
        const int64_t e0 = op.obj_edge[o], neo = op.obj_edge[o + 1] - e0, q0 = op.obj_q[o];
        std::vector<bem_c64> row(A.cols);
        for (int64_t r = 0; r < A.rows; ++r) {
          copy_row(A, r, row.data());
          const int64_t gr = r < neo ? e0 + r : op.ne + q0 + (r - neo);
          for (int64_t c = 0; c < A.cols; ++c) {
            const int64_t gc = c < neo ? e0 + c : op.ne + q0 + (c - neo);
            host[gr * op.Neq + gc] = row[c];
          }
        }
      }
      return;
    }
    case BEM_BLOCK_IX: {
      std::vector<int64_t> ptr(op.ne + 1);
      BEM_HIP(hipMemcpy(ptr.data(), op.ix_ptr, sizeof(int64_t) * (op.ne + 1), hipMemcpyDeviceToHost));
      std::vector<int32_t> idx(ptr[op.ne]);
      std::vector<double> val(ptr[op.ne]);
      BEM_HIP(hipMemcpy(idx.data(), op.ix_idx, sizeof(int32_t) * idx.size(), hipMemcpyDeviceToHost));
      BEM_HIP(hipMemcpy(val.data(), op.ix_val, sizeof(double) * val.size(), hipMemcpyDeviceToHost));
      std::memset(host, 0, sizeof(bem_c64) * op.ne * op.ne);
      for (int64_t r = 0; r < op.ne; ++r)
        for (int64_t p = ptr[r]; p < ptr[r + 1]; ++p) host[r * op.ne + idx[p]] = {val[p], 0.0};
      return;
    }
    default:
      throw Error(BEM_E_INVALID, "block cannot be exported");
  }
}

// ----------------------------------------------------------------- GMRES

std::unique_ptr<GmresWork> make_gmres_work(DevArena& mem, int64_t n, int m) {
  auto w = std::make_unique<GmresWork>();
  w->n = n;
  w->m = m;
  w->ldv = pad64(n);
  w->V = mem.alloc<double2>(size_t(m + 1) * w->ldv);
  w->H = mem.alloc<double2>(size_t(m + 1) * (m + 2));
  w->cs = mem.alloc<double2>(m + 1);
  w->sn = mem.alloc<double2>(m + 1);
  w->g = mem.alloc<double2>(m + 2);
  w->y = mem.alloc<double2>(m + 1);
  w->h2 = mem.alloc<double2>(m + 2);
  w->z = mem.alloc<double2>(size_t(w->ldv));
  w->z2 = mem.alloc<double2>(size_t(w->ldv));
  w->nrm = mem.alloc<double2>(2);
  w->res = mem.alloc<double>(2);
  w->ks.partial = mem.alloc<double2>(1024);
  w->ks.nblk = 128;
  return w;
}

static double read_scalar(double* pinned, const double* d, hipStream_t st) {
  BEM_HIP(hipMemcpyAsync(pinned, d, sizeof(double), hipMemcpyDeviceToHost, st));
  BEM_HIP(hipStreamSynchronize(st));
  return pinned[0];
}

GmresResult gmres(GmresWork& w, double* ctx, const ApplyFn& A, const double2* b, double2* x, bool x_zero,
                  double tol, int maxit, hipStream_t st, const ApplyFn* M) {
  GmresResult res;
  const int64_t n = w.n;
  const int64_t ldh = w.m + 2;
  launch_norm(b, n, w.nrm, w.ks, st);
  const double bnorm = read_scalar(ctx, reinterpret_cast<const double*>(w.nrm), st);
  if (!std::isfinite(bnorm)) throw Error(BEM_E_NUMERIC, "non-finite right-hand side");
  if (x_zero) launch_axpby(n, c2(0.0), nullptr, c2(0.0), nullptr, x, st);
  if (bnorm == 0.0) {
    launch_axpby(n, c2(0.0), nullptr, c2(0.0), nullptr, x, st);
    res.converged = true;
    return res;
  }
  bool first = true;
  while (true) {
    // r = b - A x  (stored in V[0])
    if (first && x_zero) {
      launch_axpby(n, c2(1.0), b, c2(0.0), nullptr, w.V, st);
    } else {
      A(x, w.V);
      launch_axpby(n, c2(1.0), b, c2(-1.0), w.V, w.V, st);
    }
    first = false;
    launch_norm(w.V, n, w.nrm, w.ks, st);
    const double beta = read_scalar(ctx, reinterpret_cast<const double*>(w.nrm), st);
    if (!std::isfinite(beta)) throw Error(BEM_E_NUMERIC, "non-finite residual in GMRES");
    res.relres = beta / bnorm;
    if (res.relres <= tol) {
      res.converged = true;
      break;
    }
    if (res.iters >= maxit) break;
    launch_scale_inv(w.V, n, w.nrm, w.V, st);
    launch_init_g(w.g, w.m, w.nrm, st);
    int j = 0;
    for (; j < w.m && res.iters < maxit; ++j) {
      double2* vj = w.V + int64_t(j) * w.ldv;
      double2* vn = w.V + int64_t(j + 1) * w.ldv;
      double2* Hcol = w.H + int64_t(j) * ldh;
      if (M) {
        (*M)(vj, w.z);
        A(w.z, vn);
      } else {
        A(vj, vn);
      }
      // CGS2
      launch_mdot(w.V, w.ldv, j + 1, vn, n, Hcol, w.ks, st);
      launch_mupdate(w.V, w.ldv, j + 1, Hcol, -1.0, vn, n, st);
      launch_mdot(w.V, w.ldv, j + 1, vn, n, w.h2, w.ks, st);
      launch_mupdate(w.V, w.ldv, j + 1, w.h2, -1.0, vn, n, st);
      launch_norm(vn, n, Hcol + j + 1, w.ks, st);
      launch_scale_inv(vn, n, Hcol + j + 1, vn, st);
      launch_givens(Hcol, j, w.cs, w.sn, w.g, w.res, w.h2, st);
      ++res.iters;
      const double r = read_scalar(ctx, w.res, st);
      if (!std::isfinite(r)) throw Error(BEM_E_NUMERIC, "non-finite Arnoldi residual");
      res.relres = r / bnorm;
      if (verbose() && w.n > 0 && w.tag)
        std::fprintf(stderr, "[bem] %s it %d res %.3e\n", w.tag, res.iters, res.relres);
      if (res.relres <= tol) {
        ++j;
        break;
      }
    }
    launch_backsolve(w.H, ldh, j, w.g, w.y, st);
    if (M) {
      // x += M (V y)
      launch_axpby(n, c2(0.0), nullptr, c2(0.0), nullptr, w.z2, st);
      launch_mupdate(w.V, w.ldv, j, w.y, +1.0, w.z2, n, st);
      (*M)(w.z2, w.z);
      launch_axpby(n, c2(1.0), x, c2(1.0), w.z, x, st);
    } else {
      launch_mupdate(w.V, w.ldv, j, w.y, +1.0, x, n, st);
    }
    if (res.relres <= tol) {
      res.converged = true;
      break;
    }
    if (res.iters >= maxit) break;
  }
  return res;
}

// ----------------------------------------------------------------- batched GMRES

namespace {

using BApplyFn = std::function<void(const double2* x, int64_t ldx, double2* y, int64_t ldy, int R)>;

// Krylov state of R independent restarted GMRES runs that share their operator products:
// basis vector i of column c at V + (i R + c) ldv, so every step's R vectors form one n x R
// column-major block for the matrix-core products.
struct BGmres {
  int64_t n = 0, ldv = 0, hs = 0, ldh = 0;
  int m = 0, Rmax = 0;
  double2 *V = nullptr, *H = nullptr, *HR = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double2 *nrm = nullptr, *part = nullptr, *part2 = nullptr, *coef = nullptr, *Z = nullptr, *U = nullptr, *T = nullptr;
  int64_t cstride = 0;  // per-column coefficients of the delayed reorthogonalisation
  double *res = nullptr, *rinv = nullptr;
  int *d_frozen = nullptr, *d_jr = nullptr, *d_idx = nullptr;
  // pinned host mirrors
  double2* h_nrm = nullptr;
  double* h_res = nullptr;
  int *h_frozen = nullptr, *h_jr = nullptr, *h_idx = nullptr, *h_fz = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};  // residuals of even / odd Arnoldi steps copied
  // pin: pinned host staging of at least pinned_bytes(R) bytes, owned by the caller
  static size_t pinned_bytes(int R) {
    return size_t(R) * (sizeof(double2) + 2 * sizeof(double) + 5 * sizeof(int)) + 64;
  }
  BGmres(DevArena& mem, int64_t n_, int m_, int R, void* pin) : n(n_), m(m_), Rmax(R) {
    ldv = pad64(n);
    alloc_cycle(mem);
    nrm = mem.alloc<double2>(R);
    rinv = mem.alloc<double>(R);
    Z = mem.alloc<double2>(size_t(R) * ldv);
    U = mem.alloc<double2>(size_t(R) * ldv);
    T = mem.alloc<double2>(size_t(R) * ldv);
    res = mem.alloc<double>(R);
    d_frozen = mem.alloc<int>(R);
    d_jr = mem.alloc<int>(R);
    d_idx = mem.alloc<int>(R);
    char* p = static_cast<char*>(pin);
    h_nrm = reinterpret_cast<double2*>(p);
    p += sizeof(double2) * R;
    h_res = reinterpret_cast<double*>(p);  // two slots of R
    p += 2 * sizeof(double) * R;
    h_frozen = reinterpret_cast<int*>(p);
    h_jr = h_frozen + R;
    h_idx = h_jr + R;
    h_fz = h_idx + R;  // two slots of R
    for (auto& e : ev) BEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // the arrays whose size follows the cycle length m: basis, Hessenberg matrices, rotations,
  // projections and reorthogonalisation coefficients
  void alloc_cycle(DevArena& mem) {
    const int R = Rmax;
    ldh = m + 2;
    hs = int64_t(m + 1) * ldh;
    V = mem.alloc<double2>(size_t(m + 1) * R * ldv);
    H = mem.alloc<double2>(size_t(R) * hs);   // Hessenberg columns as finished
    HR = mem.alloc<double2>(size_t(R) * hs);  // the same rotated to triangular (Givens)
    cs = mem.alloc<double2>(size_t(R) * (m + 1));
    sn = mem.alloc<double2>(size_t(R) * (m + 1));
    y = mem.alloc<double2>(size_t(R) * (m + 1));
    g = mem.alloc<double2>(size_t(R) * (m + 2));
    part = mem.alloc<double2>(size_t(R) * (m + 1) * bkry_chunks(n));
    part2 = mem.alloc<double2>(size_t(R) * (m + 1) * bkry_chunks(n));
    cstride = 2 * int64_t(m + 2);
    coef = mem.alloc<double2>(size_t(R) * cstride);
  }
  // A longer cycle for the same columns (between GMRES calls): the cycle's arrays are made anew
  // for m_ steps and the old ones returned to the arena.
  void grow(DevArena& mem, int m_) {
    for (void* p : {static_cast<void*>(V), static_cast<void*>(H), static_cast<void*>(HR), static_cast<void*>(cs),
                    static_cast<void*>(sn), static_cast<void*>(y), static_cast<void*>(g), static_cast<void*>(part),
                    static_cast<void*>(part2), static_cast<void*>(coef)})
      mem.release(p);
    m = m_;
    alloc_cycle(mem);
  }
  ~BGmres() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  BGmres(const BGmres&) = delete;
  void upload(int* d, const int* h, int R, hipStream_t st) {
    BEM_HIP(hipMemcpyAsync(d, h, sizeof(int) * R, hipMemcpyHostToDevice, st));
  }
  // column norms of X (n x R, ldx) into h_nrm
  void norms(const double2* X, int64_t ldx, int R, hipStream_t st) {
    launch_bnorm(X, ldx, R, n, part, nrm, 1, st);
    BEM_HIP(hipMemcpyAsync(h_nrm, nrm, sizeof(double2) * R, hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
  }
};

struct BResult {
  std::vector<int> iters;        // Arnoldi steps taken by each column
  std::vector<double> relres;    // estimated relative residual of each column
  std::vector<char> converged;
  int products = 0;              // batched operator products
  int graph_steps = 0;           // Arnoldi steps replayed from a captured graph
};

// Restarted GMRES (CGS2 Arnoldi, complex Givens, float64) for the R0 columns of B (n x R0,
// ldb) at once; X (ldx) is zeroed and receives the solutions.  Every Arnoldi step applies A
// (and the right preconditioner M) to the block of the still-active columns in one call.
// A column stops contributing basis vectors once its estimated residual reaches tol; at
// every restart the unconverged columns are compacted.
// Relaxed products (A_lo, M_lo: a cheaper operator and preconditioner): once the largest
// estimated relative residual of the active columns is at most `relax`, the Arnoldi steps use
// them in place of A and M (M_lo must equal M unless the steps and the solution update agree
// on it: the update applies M to V y).  The error a cruder product adds to the solution is
// scaled by the basis coefficients of its step, which shrink with the residual, so early steps
// get accurate products and late ones cheap products (relaxation in inexact Krylov methods:
// Bouras and Fraysse 2005, Simoncini and Szyld 2003).  Only the first cycle relaxes: a
// restarted cycle works on the slowly converging components, whose large coefficients take the
// cruder products' error whole (float32 cycles after a restart made no true progress on the
// 5120-triangle sphere).  Restart residuals and the solution update use A and M.
// Captured step products: the launch chain of one Arnoldi step's product A (M x), recorded once
// per (column count, precision) into a HIP graph on fixed buffers (w.U in, w.Z between, w.T
// out) and replayed between two device copies.  For small operators the chain (20-30 launches
// of a few microseconds each) is bound by launch overhead; the replay submits it at once.  The
// same kernels run with the same arguments, so results are bitwise those of direct launches.
struct StepGraphs {
  struct Entry {
    int R;
    bool lo;
    hipGraph_t g;
    hipGraphExec_t e;
  };
  std::vector<Entry> v;
  bool failed = false;
  StepGraphs() = default;
  StepGraphs(const StepGraphs&) = delete;
  ~StepGraphs() {
    for (auto& c : v) {
      if (c.e) (void)hipGraphExecDestroy(c.e);
      if (c.g) (void)hipGraphDestroy(c.g);
    }
  }
  // the replayable chain for R columns, captured on first use; null if capture is not possible
  hipGraphExec_t get(int R, bool lo, const std::function<void()>& chain, hipStream_t st) {
    for (auto& c : v)
      if (c.R == R && c.lo == lo) return c.e;
    if (failed) return nullptr;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      failed = true;
      return nullptr;
    }
    try {
      chain();
    } catch (...) {
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      throw;
    }
    if (hipStreamEndCapture(st, &g) != hipSuccess || !g) {
      (void)hipGetLastError();
      failed = true;
      return nullptr;
    }
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipGraphDestroy(g);
      failed = true;
      return nullptr;
    }
    v.push_back({R, lo, g, e});
    if (verbose()) std::fprintf(stderr, "[bem] captured the step product for %d columns%s\n", R, lo ? " (relaxed)" : "");
    return e;
  }
};

BResult gmres_batched(BGmres& w, const BApplyFn& A, const double2* B, int64_t ldb, double2* X, int64_t ldx, int R0,
                      double tol, int maxit, hipStream_t st, const BApplyFn* M, const BApplyFn* A_lo = nullptr,
                      const BApplyFn* M_lo = nullptr, double relax = 0.0, bool graphs = false) {
  StepGraphs sg;
  BResult out;
  out.iters.assign(R0, 0);
  out.relres.assign(R0, 0.0);
  out.converged.assign(R0, 0);
  if (R0 > w.Rmax) throw Error(BEM_E_INVALID, "batch wider than its Krylov state");
  const int64_t n = w.n, ldv = w.ldv;
  const int m = w.m;
  w.norms(B, ldb, R0, st);
  std::vector<double> bn(R0);
  std::vector<int> active;
  for (int c = 0; c < R0; ++c) {
    bn[c] = w.h_nrm[c].x;
    if (!std::isfinite(bn[c])) throw Error(BEM_E_NUMERIC, "non-finite right-hand side");
    if (bn[c] > 0) active.push_back(c);
    else out.converged[c] = 1;
  }
  launch_axpby(n, c2(0.0), nullptr, c2(0.0), nullptr, X, st, R0, 0, 0, ldx);
  int total = 0;  // batched Arnoldi steps
  bool first = true, first_cycle = true;
  while (!active.empty()) {
    const int Rc = int(active.size());
    for (int c = 0; c < Rc; ++c) w.h_idx[c] = active[c];
    w.upload(w.d_idx, w.h_idx, Rc, st);
    // residual block V_0 = B - A X over the active columns
    double2* V0 = w.V;
    launch_gather_cols(B, ldb, V0, ldv, w.d_idx, n, Rc, st);
    if (!first) {
      launch_gather_cols(X, ldx, w.U, ldv, w.d_idx, n, Rc, st);
      A(w.U, ldv, w.T, ldv, Rc);
      ++out.products;
      launch_axpby(n, c2(1.0), V0, c2(-1.0), w.T, V0, st, Rc, ldv, ldv, ldv);
    }
    first = false;
    w.norms(V0, ldv, Rc, st);
    int live = 0;
    double worst_est = 0.0;  // largest estimated relative residual of the active columns
    for (int c = 0; c < Rc; ++c) {
      const int col = active[c];
      const double beta = w.h_nrm[c].x;
      if (!std::isfinite(beta)) throw Error(BEM_E_NUMERIC, "non-finite residual in GMRES");
      out.relres[col] = beta / bn[col];
      if (out.relres[col] > tol) worst_est = std::max(worst_est, out.relres[col]);
      w.h_frozen[c] = out.relres[col] <= tol ? 1 : 0;
      w.h_jr[c] = 0;
      if (w.h_frozen[c]) out.converged[col] = 1;
      else ++live;
    }
    if (live == 0 || total >= maxit) break;
    w.upload(w.d_frozen, w.h_frozen, Rc, st);
    launch_bscale_inv(V0, ldv, Rc, n, w.nrm, 1, w.d_frozen, st);
    launch_binit_g(w.g, m, w.nrm, 1, Rc, st);
    // Arnoldi steps.  The residual estimates of step j are examined while step j + 1 runs: the
    // host waits for the copy of step j - 1 only after enqueuing step j, so the GPU never idles
    // on the convergence check; a column converged at step j - 1 stops contributing vectors
    // from step j + 1 on (its extra vectors are not used by the back-solve).
    std::vector<char> frozen(Rc);
    for (int c = 0; c < Rc; ++c) frozen[c] = char(w.h_frozen[c]);
    int j = 0;
    auto examine = [&](int s) {
      BEM_HIP(hipEventSynchronize(w.ev[s & 1]));
      const double* hr = w.h_res + size_t(s & 1) * w.Rmax;
      bool changed = false;
      double worst = 0.0;
      for (int c = 0; c < Rc; ++c) {
        if (frozen[c]) continue;
        const int col = active[c];
        const double rr = hr[c] / bn[col];
        if (!std::isfinite(rr)) throw Error(BEM_E_NUMERIC, "non-finite Arnoldi residual");
        ++out.iters[col];
        out.relres[col] = rr;
        worst = std::max(worst, rr);
        if (rr <= tol) {
          frozen[c] = 1;
          w.h_jr[c] = s + 1;
          out.converged[col] = 1;
          --live;
          changed = true;
        }
      }
      if (verbose())
        std::fprintf(stderr, "[bem] batched step %d: %d of %d columns active, worst res %.3e\n", s + 1, live, Rc,
                     worst);
      worst_est = worst;
      return changed;
    };
    // Givens rotation of the finished Hessenberg column s and the copy of its residual estimates
    auto estimate = [&](int s) {
      launch_bgivens(w.H, w.HR, w.hs, w.ldh, s, w.cs, w.sn, w.g, w.res, nullptr, m, Rc, st);
      BEM_HIP(hipMemcpyAsync(w.h_res + size_t(s & 1) * w.Rmax, w.res, sizeof(double) * Rc, hipMemcpyDeviceToHost,
                             st));
      BEM_HIP(hipEventRecord(w.ev[s & 1], st));
    };
    bool lo = false;
    for (; j < m && total < maxit; ++j) {
      double2* Vj = w.V + int64_t(j) * Rc * ldv;
      double2* Vn = w.V + int64_t(j + 1) * Rc * ldv;
      double2* Hj = w.H + int64_t(j) * w.ldh;
      if (A_lo && first_cycle && !lo && worst_est <= relax) {
        lo = true;
        if (verbose()) std::fprintf(stderr, "[bem] relaxed products from step %d (residual %.3e)\n", j, worst_est);
      }
      const BApplyFn& Aj = lo ? *A_lo : A;
      const BApplyFn* Mj = lo ? M_lo : M;
      hipGraphExec_t ge = nullptr;
      if (graphs)
        ge = sg.get(Rc, lo, [&]() {
          if (Mj) {
            (*Mj)(w.U, ldv, w.Z, ldv, Rc);
            Aj(w.Z, ldv, w.T, ldv, Rc);
          } else {
            Aj(w.U, ldv, w.T, ldv, Rc);
          }
        }, st);
      if (ge) {
        // (U and T are free during the Arnoldi steps: they serve the restart and the update)
        BEM_HIP(hipMemcpyAsync(w.U, Vj, sizeof(double2) * Rc * ldv, hipMemcpyDeviceToDevice, st));
        BEM_HIP(hipGraphLaunch(ge, st));
        BEM_HIP(hipMemcpyAsync(Vn, w.T, sizeof(double2) * Rc * ldv, hipMemcpyDeviceToDevice, st));
        ++out.graph_steps;
      } else if (Mj) {
        (*Mj)(Vj, ldv, w.Z, ldv, Rc);
        Aj(w.Z, ldv, Vn, ldv, Rc);
      } else {
        Aj(Vj, ldv, Vn, ldv, Rc);
      }
      ++out.products;
      // Gram-Schmidt with delayed reorthogonalisation: V_j left the previous step after one
      // projection; this step's single pass over the basis reorthogonalises V_j (finishing
      // Hessenberg column j - 1, whose Givens rotation and residual estimate follow) and
      // projects the product, which then also leaves after one projection.
      if (j == 0) {
        launch_bmdot(w.V, ldv, Rc, 1, Vn, ldv, n, w.part, Hj, w.hs, st);
        launch_bmupdate(w.V, ldv, Rc, 1, nullptr, Hj, w.hs, -1.0, Vn, ldv, n, st);
      } else {
        launch_bdcgs2(w.V, ldv, Rc, j, Vn, ldv, n, w.part, w.part2, w.H, w.hs, w.ldh, w.coef, w.cstride, w.rinv,
                      w.d_frozen, true, st);
        estimate(j - 1);
      }
      launch_bnorm(Vn, ldv, Rc, n, w.part, Hj + j + 1, w.hs, st);
      launch_bscale_inv(Vn, ldv, Rc, n, Hj + j + 1, w.hs, w.d_frozen, st);
      ++total;
      if (j >= 2) {
        if (examine(j - 2)) {
          // stage the new flags in this step's slot (the slot of step j - 2 is free: its copy
          // was enqueued before the event just waited for)
          int* fz = w.h_fz + size_t(j & 1) * w.Rmax;
          for (int c = 0; c < Rc; ++c) fz[c] = frozen[c];
          w.upload(w.d_frozen, fz, Rc, st);
        }
        if (live == 0) {
          ++j;
          break;
        }
      }
    }
    if (live > 0 && j >= 1) {
      // the last column: reorthogonalise the last vector against the basis (no new product)
      launch_bdcgs2(w.V, ldv, Rc, j, w.V + int64_t(j) * Rc * ldv, ldv, n, w.part, w.part2, w.H, w.hs, w.ldh, w.coef,
                    w.cstride, w.rinv, w.d_frozen, false, st);
      estimate(j - 1);
      if (j >= 2) examine(j - 2);
      if (live > 0) examine(j - 1);
    }
    for (int c = 0; c < Rc; ++c)
      if (!frozen[c]) w.h_jr[c] = j;
    w.upload(w.d_jr, w.h_jr, Rc, st);
    launch_bbacksolve(w.HR, w.hs, w.ldh, w.d_jr, w.g, w.y, m, Rc, st);
    // X[:, active] += M (V y)
    launch_axpby(n, c2(0.0), nullptr, c2(0.0), nullptr, w.U, st, Rc, 0, 0, ldv);
    launch_bmupdate(w.V, ldv, Rc, 0, w.d_jr, w.y, m + 1, +1.0, w.U, ldv, n, st);
    if (M) {
      (*M)(w.U, ldv, w.T, ldv, Rc);
      launch_scatter_cols(w.T, ldv, X, ldx, w.d_idx, n, Rc, 1, st);
    } else {
      launch_scatter_cols(w.U, ldv, X, ldx, w.d_idx, n, Rc, 1, st);
    }
    BEM_HIP(hipStreamSynchronize(st));
    std::vector<int> next;
    for (int c = 0; c < Rc; ++c)
      if (!out.converged[active[c]]) next.push_back(active[c]);
    active.swap(next);
    first_cycle = false;
    if (total >= maxit) break;
  }
  return out;
}

}  // namespace

// ----------------------------------------------------------------- solve

namespace {

// Right-hand sides (N_E x nexc, column-major) of eq. finalsystem's first block row.
void build_rhs(OpObj& op, DevArena& tmp, const bem_excitation* exc, int64_t nexc, double2* B, hipStream_t st) {
  const int64_t ne = op.ne;
  std::vector<double> khat;
  std::vector<double2> pol, amp;
  std::vector<int64_t> pw;  // plane-wave excitations
  launch_axpby(ne * nexc, c2(0.0), nullptr, c2(0.0), nullptr, B, st);
  for (int64_t e = 0; e < nexc; ++e) {
    const bem_excitation& x = exc[e];
    if (x.kind == BEM_EXC_PLANE_WAVE) {
      for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(x.khat[k]) || !std::isfinite(x.pol[k].re) || !std::isfinite(x.pol[k].im))
          throw Error(BEM_E_NUMERIC, "non-finite excitation");
        khat.push_back(x.khat[k]);
        pol.push_back(c2(x.pol[k].re, x.pol[k].im));
      }
      if (!std::isfinite(x.amp.re) || !std::isfinite(x.amp.im)) throw Error(BEM_E_NUMERIC, "non-finite amplitude");
      amp.push_back(c2(x.amp.re, x.amp.im));
      pw.push_back(e);
    } else if (x.kind == BEM_EXC_DELTA_GAP) {
      // gap field across each listed edge, along the RWG of the directed pair (a -> b):
      // b_m = +V/eta0 when (a, b) = (va, vb) of edge m, -V/eta0 when reversed
      if (!x.gap_edges || x.n_gap <= 0) throw Error(BEM_E_INVALID, "delta gap without edges");
      std::vector<double2> col(ne, c2(0.0));
      std::map<std::pair<int32_t, int32_t>, int64_t> eid;
      for (int64_t n = 0; n < ne; ++n) eid[{op.m->ev[2 * n], op.m->ev[2 * n + 1]}] = n;
      for (int64_t g = 0; g < x.n_gap; ++g) {
        int32_t a = x.gap_edges[2 * g], b = x.gap_edges[2 * g + 1];
        double s = 1.0;
        if (a > b) {
          std::swap(a, b);
          s = -1.0;
        }
        auto it = eid.find({a, b});
        if (it == eid.end()) throw Error(BEM_E_INVALID, "gap edge is not a mesh edge");
        col[it->second] = c2(s * x.amp.re / kEta0, s * x.amp.im / kEta0);
      }
      BEM_HIP(hipMemcpyAsync(B + e * ne, col.data(), sizeof(double2) * ne, hipMemcpyHostToDevice, st));
      BEM_HIP(hipStreamSynchronize(st));
    } else {
      throw Error(BEM_E_INVALID, "unknown excitation kind");
    }
  }
  if (!pw.empty()) {
    double* dk = tmp.upload(khat);
    double2* dp = tmp.upload(pol);
    double2* da = tmp.upload(amp);
    double2* Bpw = tmp.alloc<double2>(size_t(ne) * pw.size());
    RhsArgs ra{op.geo, op.nt, op.tp, op.tm, op.ip, op.im, ne, dk, dp, da, op.kbg.real(), op.kbg.imag(),
               1.0 / kEta0, Bpw, ne};
    launch_rhs_planewave(ra, int(pw.size()), st);
    for (size_t i = 0; i < pw.size(); ++i)
      BEM_HIP(hipMemcpyAsync(B + pw[i] * ne, Bpw + i * ne, sizeof(double2) * ne, hipMemcpyDeviceToDevice, st));
  }
}

// Outputs of R solutions xs (N x R, ldx): H = a / (j k0), E = eta0 e, rho = -B x3 / c0
// (excitation e of the batch at column e of every output).
void write_outputs(OpObj& op, DevArena& tmp, const double2* xs, int64_t ldx, int R, const bem_solve_opts& opts,
                   bem_c64* Hout, bem_c64* Eout, bem_c64* rhoout, hipStream_t st) {
  const int64_t ne = op.ne, nt = op.nt;
  double2* o1 = tmp.alloc<double2>(size_t(ne) * R);
  double2* o3 = tmp.alloc<double2>(size_t(nt) * R);
  auto put = [&](bem_c64* dst, const double2* src, int64_t len) {
    if (!dst) return;
    BEM_HIP(hipMemcpyAsync(dst, src, sizeof(double2) * len * R,
                           opts.out_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    BEM_HIP(hipStreamSynchronize(st));
  };
  launch_axpby(ne, c2(0.0, -1.0 / op.k0), xs, c2(0.0), nullptr, o1, st, R, ldx, 0, ne);
  put(Hout, o1, ne);
  launch_axpby(ne, c2(kEta0), xs + ne, c2(0.0), nullptr, o1, st, R, ldx, 0, ne);
  put(Eout, o1, ne);
  launch_expand_charge(xs + 2 * ne, o3, op.obj_tri_d, op.nobj, c2(-1.0 / kC0), st, R, ldx, nt);
  put(rhoout, o3, nt);
  tmp.release(o1);
  tmp.release(o3);
}

// True float64 relative residuals ||b - A x|| / ||b|| of R columns.
std::vector<double> true_residuals(BGmres& w, const BApplyFn& A64, const double2* b, const double2* x, int64_t ld,
                                   int R, hipStream_t st) {
  w.norms(b, ld, R, st);
  std::vector<double> bn(R);
  for (int c = 0; c < R; ++c) bn[c] = w.h_nrm[c].x;
  A64(x, ld, w.T, w.ldv, R);
  launch_axpby(w.n, c2(1.0), b, c2(-1.0), w.T, w.T, st, R, ld, w.ldv, w.ldv);
  w.norms(w.T, w.ldv, R, st);
  std::vector<double> rel(R);
  for (int c = 0; c < R; ++c) rel[c] = bn[c] > 0 ? w.h_nrm[c].x / bn[c] : 0.0;
  return rel;
}

constexpr int kMaxBatch = 256;
// largest system (unknowns) whose step products are replayed from captured graphs
constexpr int64_t kGraphMaxN = 65536;

}  // namespace

size_t estimate_request_bytes(int64_t nt, int64_t nobj, int precision, int restart, int64_t nexc, int formulation) {
  const double ne = 1.5 * double(nt), no = double(std::max<int64_t>(nobj, 1));
  const double nq = double(nt) - no, N = 2 * ne + nq, neq = ne + nq;
  // bytes per dense entry: float64 + float32 copy while assembling (BEM_FP32 and BEM_MIXED), then
  // the float32 copy alone (BEM_FP32) or both (BEM_MIXED)
  const double per_fill = precision == BEM_FP64 ? 16.0 : 24.0;
  const double per = precision == BEM_FP64 ? 16.0 : (precision == BEM_FP32 ? 8.0 : 24.0);
  const bool eaefie = formulation == BEM_FORM_EAEFIE;
  // per object L^A, K~ (and K~_l), L^phi; all pairs L^A_l, L^phi_l (and K~_m)
  const double entries = ((eaefie ? 2 : 3) * ne * ne + double(nt) * nt) / no + (eaefie ? 2 : 1) * ne * ne +
                         double(nt) * nt;
  const double dense = per * entries, dense_fill = per_fill * entries;
  const double fill_scratch = 16.0 * 9.0 * double(nt) * double(fill_chunk_triangles(nt, 3 * nt));
  // augmented inverse (not for the eAEFIE) + Sigma_P^-1 (formed in float64 before the drop)
  const double inv_entries = (eaefie ? 0.0 : (neq * neq) / no) + (nq * nq) / no;
  const double inner = per * inv_entries;
  const double R = double(std::min<int64_t>(std::max<int64_t>(nexc, 1), kMaxBatch));
  const double ldN = double(pad64(int64_t(N)));
  const double m = restart;
  const double solve = 16.0 * R * (ldN * (m + 1 + 3 + 4) + double(kWorkFields) * pad64(int64_t(neq)) +
                                   2.0 * (m + 1) * (m + 2)) +
                       double(gemm_workspace_bytes(int64_t(std::max(ne, double(nt))), int64_t(R))) +
                       16.0 * (ne * (nexc + 1) + 2 * 64.0 * neq);
  const double assembly = std::max(dense_fill + fill_scratch, dense_fill + per_fill * inv_entries);
  return size_t(std::max(assembly, dense + inner + solve) + 64.0 * 1024 * 1024);
}

constexpr int kMaxAutoRestart = 1000;

int auto_restart(int64_t N, int64_t nexc) {
  // the longest cycle (at most 1000 steps, at least 100) whose Krylov basis of the batch stays
  // under kAutoKrylovBytes: restarts discard the Krylov space, and the hard (electrically large,
  // high-contrast) problems converge in far fewer steps with long cycles
  const double per_step = 16.0 * double(std::min<int64_t>(std::max<int64_t>(nexc, 1), kMaxBatch)) * double(pad64(N));
  const double m = std::floor(kAutoKrylovBytes / per_step) - 1.0;
  return int(std::max(100.0, std::min(double(kMaxAutoRestart), m)));
}

int solve_op(OpObj& op, const bem_excitation* exc, int64_t nexc, const bem_solve_opts& opts_in, bem_c64* Hout,
             bem_c64* Eout, bem_c64* rhoout, bem_solve_info* info, hipStream_t st) {
  auto tstart = std::chrono::steady_clock::now();
  if (nexc <= 0 || !exc) throw Error(BEM_E_INVALID, "no excitation");
  if (!(opts_in.tol > 0) || opts_in.maxit <= 0) throw Error(BEM_E_INVALID, "invalid solve options");
  bem_solve_opts opts = opts_in;
  if (opts.restart <= 0) opts.restart = auto_restart(op.N, nexc);
  const int64_t ne = op.ne, nt = op.nt, N = op.N;
  DevArena tmp(op.ctx);
  tmp.set_stream(st);
  double2* Bexc = tmp.alloc<double2>(size_t(ne) * nexc);
  build_rhs(op, tmp, exc, nexc, Bexc, st);
  const double inner = opts.inner_tol > 0 ? opts.inner_tol : 0.1 * opts.tol;
  const double inner32 = std::max(inner, 1e-7);
  // Mixed precision: a sweep runs float64 products until the estimated residual is sqrt(tol)
  // of ||b||, then float32 products (relaxed products of gmres_batched).  With float32 products
  // from the first step the true residual stalls near the float32 operator's error times the
  // solution's size (1.4e-4 on the 5120-triangle sphere, against 1e-6 estimated), and every
  // refinement sweep restarts the Krylov space; scaled by sqrt(tol) that error is below tol.
  // (switching earlier costs iterations: from tol^(1/3) the serving mix needed 22% more steps)
  const double relax_global = std::sqrt(opts.tol);
  const int sweeps = opts.max_refine > 0 ? opts.max_refine : (op.precision != BEM_FP64 ? 5 : 3);
  bem_solve_info inf{};
  int status = BEM_OK;
  op.max_inner_iters = 0;

  // batch width: as many excitations as fit a quarter of the remaining budget
  int Rb = int(std::min<int64_t>(nexc, kMaxBatch));
  {
    auto est = [&](int R) {
      const double ldN = double(pad64(N)), m = opts.restart;
      // basis, work columns, Hessenberg matrices (as finished and rotated)
      return 16.0 * R * (ldN * (m + 1 + 3 + 5) + double(kWorkFields) * work_ld(op) + 2.0 * (m + 1) * (m + 2)) +
             double(gemm_workspace_bytes(std::max(ne, nt), R));
    };
    size_t avail;
    {
      std::lock_guard<std::mutex> g(op.ctx->mu);
      avail = op.ctx->budget > op.ctx->used ? op.ctx->budget - op.ctx->used : 0;
    }
    while (Rb > 1 && est(Rb) > 0.5 * double(avail)) Rb = (Rb + 1) / 2;
  }
  const int64_t ldN = pad64(N);
  while (Rb > 1 && BGmres::pinned_bytes(Rb) > kPinnedBytes - kPinnedScalars * sizeof(double)) Rb = (Rb + 1) / 2;
  BGmres bw(tmp, N, opts.restart, Rb, op.pinned + kPinnedScalars);
  WorkView wv = batch_views(op, tmp, Rb);
  double2* bfull = tmp.alloc<double2>(size_t(Rb) * ldN);
  double2* xs = tmp.alloc<double2>(size_t(Rb) * ldN);
  double2* rr = tmp.alloc<double2>(size_t(Rb) * ldN);  // refinement residuals (compacted)
  double2* dd = tmp.alloc<double2>(size_t(Rb) * ldN);  // refinement corrections (compacted)
  int* ref_idx = tmp.alloc<int>(Rb);                     // refinement's active columns
  auto with_R = [&wv](int R) {
    WorkView v = wv;
    v.R = R;
    return v;
  };
  BApplyFn A64 = [&](const double2* x, int64_t ldx, double2* y, int64_t ldy, int R) {
    final_cols(op, with_R(R), x, ldx, y, ldy, false, inner, st);
  };
  BApplyFn A32 = [&](const double2* x, int64_t ldx, double2* y, int64_t ldy, int R) {
    final_cols(op, with_R(R), x, ldx, y, ldy, true, inner32, st);
  };
  BApplyFn P64 = [&](const double2* x, int64_t ldx, double2* y, int64_t ldy, int R) {
    if (ldx != ldy) throw Error(BEM_E_INVALID, "preconditioner needs equal strides");
    precond_cols(op, with_R(R), x, y, ldx, false, st);
  };
  const BApplyFn* Pm64 = op.precond ? &P64 : nullptr;

  // Mixed precision pays only while the float32 products stay close to the float64 ones on
  // vectors shaped like the solution: once per solve, z = P b (b the first excitation's
  // right-hand side, P the preconditioner, an approximate inverse) is multiplied in both
  // precisions, and float64 products are used throughout when ||A32 z - A64 z|| / ||A64 z||
  // exceeds kFp32ProbeTol.  Random vectors do not show it: for small conductors at low
  // frequency the equivalent current cancels the physical one to many digits, so float32
  // products of solution-like vectors lose them all, and float32 steps make no progress.
  // (BEM_FP32: both products read the float32 entries; A64 takes them in float64 arithmetic)
  bool fp32_ok = op.precision != BEM_FP64;
  bool probed = false;
  // Arnoldi step products replayed from captured graphs: where the chain has no host step (no
  // nested GMRES, no serving combiner, no kernel timer) and the operator is small enough for
  // launch overhead to matter.  BEM_GRAPH=0 turns it off.
  const char* genv = std::getenv("BEM_GRAPH");
  const bool graphs = !(genv && std::strcmp(genv, "0") == 0) && !op.comb && !Profiler::get().enabled() &&
                      (op.formulation == BEM_FORM_EAEFIE || op.inner_mode != BEM_INNER_GMRES) && N <= kGraphMaxN;
  for (int64_t e0 = 0; e0 < nexc; e0 += Rb) {
    const int R = int(std::min<int64_t>(Rb, nexc - e0));
    launch_axpby(N, c2(0.0), nullptr, c2(0.0), nullptr, bfull, st, R, 0, 0, ldN);
    BEM_HIP(hipMemcpy2DAsync(bfull, sizeof(double2) * ldN, Bexc + e0 * ne, sizeof(double2) * ne,
                             sizeof(double2) * ne, R, hipMemcpyDeviceToDevice, st));
    std::vector<char> conv(R, 0);
    if (fp32_ok && !probed) {
      probed = true;
      if (op.precond) P64(bfull, ldN, dd, ldN, 1);
      else BEM_HIP(hipMemcpyAsync(dd, bfull, sizeof(double2) * N, hipMemcpyDeviceToDevice, st));
      A64(dd, ldN, rr, ldN, 1);
      const double dev = true_residuals(bw, A32, rr, dd, ldN, 1, st)[0];
      inf.n_products += 2;
      fp32_ok = dev <= kFp32ProbeTol;
      if (verbose()) std::fprintf(stderr, "[bem] float32 product deviation %.3e%s\n", dev, fp32_ok ? "" : ": float64 products");
    }
    // One refinement loop for both precisions.  Every sweep solves A d = r for the active
    // columns with GMRES (in mixed precision float64 products until the residual is small,
    // float32 products after; float64 products otherwise), then x += d and the float64
    // residual r = b - A x is recomputed; a column leaves once ||r|| <= tol ||b||.  A mixed
    // sweep that does not halve the residual of every active column, or that does not reach
    // its target within three restart cycles, switches the remaining sweeps to float64
    // products (float32 too inaccurate for this operator); the sweeps after the first correct
    // the Arnoldi estimate drifting from the true residual.
    launch_axpby(N, c2(0.0), nullptr, c2(0.0), nullptr, xs, st, R, 0, 0, ldN);
    bw.norms(bfull, ldN, R, st);
    std::vector<double> bn(R), rel(R, 1.0);
    std::vector<int> active;
    for (int c = 0; c < R; ++c) {
      bn[c] = bw.h_nrm[c].x;
      if (bn[c] > 0) active.push_back(c);
      else {
        conv[c] = 1;
        rel[c] = 0.0;
      }
    }
    bool use32 = fp32_ok;
    int left = opts.maxit;
    auto upload_active = [&]() {
      BEM_HIP(hipStreamSynchronize(st));
      BEM_HIP(hipMemcpyAsync(ref_idx, active.data(), sizeof(int) * active.size(), hipMemcpyHostToDevice, st));
      BEM_HIP(hipStreamSynchronize(st));
    };
    for (int s = 0; s < sweeps && left > 0 && !active.empty(); ++s) {
      const int Rc = int(active.size());
      const int* didx = ref_idx;
      upload_active();
      // compacted residual: r = b - A64 x (x = 0 on the first sweep)
      launch_gather_cols(bfull, ldN, rr, ldN, didx, N, Rc, st);
      if (s > 0) {
        launch_gather_cols(xs, ldN, dd, ldN, didx, N, Rc, st);
        A64(dd, ldN, bw.T, bw.ldv, Rc);
        ++inf.n_products;
        launch_axpby(N, c2(1.0), rr, c2(-1.0), bw.T, rr, st, Rc, ldN, bw.ldv, ldN);
      }
      BEM_HIP(hipStreamSynchronize(st));
      // GMRES target relative to ||r||: every sweep aims at what the tolerance still needs,
      // tol ||b|| (half of it, for margin); a mixed sweep reduces by at least 4x (so one that
      // does not halve the true residual has met float32's limit).  Its switch to float32
      // products is relative to ||r|| too.
      double gtol = use32 ? 0.25 : 1.0, rmax = 0.0;
      for (int c = 0; c < Rc; ++c) {
        gtol = std::min(gtol, 0.5 * opts.tol / std::max(rel[active[c]], 1e-300));
        rmax = std::max(rmax, rel[active[c]]);
      }
      gtol = std::max(gtol, 1e-15);
      // (BEM_FP32 the same: its float64-arithmetic products on the float32 entries until then;
      // float32 arithmetic from the first step costs more iterations in the later sweeps than it
      // saves - 45% more on the serving mix)
      const double relax = relax_global / std::max(rmax, 1e-300);
      // a mixed sweep gets at most three restart cycles (600 steps at least): one that cannot
      // reach its target in that budget works on products too inaccurate in float32
      const int budget = use32 ? std::min(left, std::max(3 * opts.restart, 600)) : left;
      // (the preconditioner stays float64: the solution update applies it to V y, so the steps
      // must have applied the same one)
      BResult g = use32 ? gmres_batched(bw, A64, rr, ldN, dd, ldN, Rc, gtol, budget, st, Pm64, &A32, Pm64, relax,
                                        graphs)
                        : gmres_batched(bw, A64, rr, ldN, dd, ldN, Rc, gtol, budget, st, Pm64, nullptr, nullptr, 0.0,
                                        graphs);
      bool sweep_failed = false;
      for (int c = 0; c < Rc; ++c) sweep_failed |= !g.converged[c];
      int most = 0;
      for (int c = 0; c < Rc; ++c) {
        inf.outer_iters += g.iters[c];
        most = std::max(most, g.iters[c]);
      }
      left -= most;
      inf.n_products += g.products;
      inf.graph_steps += g.graph_steps;
      if (s > 0 || use32) ++inf.refine_steps;
      // x += d ; float64 residual of the updated columns
      launch_scatter_cols(dd, ldN, xs, ldN, didx, N, Rc, 1, st);
      launch_gather_cols(xs, ldN, dd, ldN, didx, N, Rc, st);
      launch_gather_cols(bfull, ldN, rr, ldN, didx, N, Rc, st);
      std::vector<double> r = true_residuals(bw, A64, rr, dd, ldN, Rc, st);
      ++inf.n_products;
      if (verbose())
        std::fprintf(stderr, "[bem] sweep %d %s: target %.2e, %d steps, true residual %.3e\n", s,
                     use32 ? "mixed" : "float64", gtol, most, *std::max_element(r.begin(), r.end()));
      bool stalled = false;
      std::vector<int> next;
      for (int c = 0; c < Rc; ++c) {
        if (r[c] > 0.5 * rel[active[c]]) stalled = true;
        rel[active[c]] = r[c];
        if (r[c] <= opts.tol) conv[active[c]] = 1;
        else next.push_back(active[c]);
      }
      active.swap(next);
      // A sweep that ran out of steps on an automatic cycle shortened by the basis budget: the
      // next sweeps get a longer one (up to 1000 steps, the basis within a quarter of the
      // context's free budget and, when serving, within what the other admitted requests leave),
      // in the same precision.  Restarted GMRES can stall on a short cycle where a long one
      // converges (a 14700-triangle ellipsoid at k0 a = 9.35 with 53 plane waves: 1e-3 after
      // 3000 steps of 159-step cycles, 1e-6 after 535 steps of one cycle).
      bool grown = false;
      if (sweep_failed && !active.empty() && opts_in.restart <= 0 && bw.m < kMaxAutoRestart) {
        size_t avail;
        {
          std::lock_guard<std::mutex> g(op.ctx->mu);
          avail = op.ctx->budget > op.ctx->used ? op.ctx->budget - op.ctx->used : 0;
        }
        // per step: a basis vector, two projection rows and the Hessenberg entries per column
        const double per_step =
            16.0 * double(Rb) * (double(ldN) + 2.0 * double(bkry_chunks(N)) + 4.0 * (kMaxAutoRestart + 2));
        int m2 = int(std::min(double(kMaxAutoRestart), std::floor(0.25 * double(avail) / per_step) - 1.0));
        while (m2 >= bw.m + bw.m / 2 && op.reserve && !op.reserve(size_t(per_step * double(m2 - bw.m))))
          m2 = bw.m + (m2 - bw.m) / 2;
        if (m2 >= bw.m + bw.m / 2) {
          if (verbose()) std::fprintf(stderr, "[bem] sweep ran out on %d-step cycles: %d-step cycles from here on\n",
                                      bw.m, m2);
          bw.grow(tmp, m2);
          opts.restart = m2;
          grown = true;
          ++inf.cycle_growths;
        }
      }
      if (use32 && (stalled || sweep_failed) && !active.empty() && !grown) {
        use32 = false;
        if (verbose()) std::fprintf(stderr, "[bem] mixed sweep stalled: float64 products from here on\n");
      }
    }
    for (int c = 0; c < R; ++c) inf.rel_residual = std::max(inf.rel_residual, rel[c]);
    for (int c = 0; c < R; ++c)
      if (!conv[c]) status = BEM_E_NOT_CONVERGED;
    write_outputs(op, tmp, xs, ldN, R, opts, Hout ? Hout + e0 * ne : nullptr, Eout ? Eout + e0 * ne : nullptr,
                  rhoout ? rhoout + e0 * nt : nullptr, st);
  }
  inf.inner_iters_max = op.max_inner_iters;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tstart).count();
  if (info) *info = inf;
  return status;
}

}  // namespace bem
