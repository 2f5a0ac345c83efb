// Host-side mesh topology for libbem: validation, RWG edge table, vertex fans, near pairs and
// the Buffa-Christiansen dual-cell data read by the K~ fill.
//
// Readings of the paper (Sec. II-B): RWG functions are area-normalised (unit flux from T+ into
// T-), so the continuity equation uses the signed incidence matrix D; one charge per object
// (its last triangle) is eliminated for neutrality; BC functions follow the standard
// combinatorial flux pattern on the barycentric refinement (flux 1/2 through each half of the
// dual edge, every sub-triangle of the source cell emitting 1/(2N), of the sink cell absorbing
// 1/(2N)).
#include <algorithm>
#include <thread>
#include <array>
#include <cmath>
#include <unordered_map>

#include "internal.h"

namespace bem {

namespace {

inline uint64_t key2(int32_t a, int32_t b) {
  return (uint64_t(uint32_t(a)) << 32) | uint32_t(b);
}

void fail(const std::string& m) { throw Error(BEM_E_MESH, m); }

}  // namespace

// Object o repeats an earlier object p when its triangles, in order, are p's triangles moved by
// one translation with a one-to-one vertex correspondence, and its edges have the same local
// table (T+, T-, free vertices).  Every object-local operator of o is then p's (Sec. II-F,
// repeated objects): the integrands depend on differences of positions only.
static bool translated_copy(const Mesh& m, int64_t p, int64_t o) {
  const int64_t tp0 = m.obj_tri[p], to0 = m.obj_tri[o], nto = m.obj_tri[o + 1] - to0;
  const int64_t ep0 = m.obj_edge[p], eo0 = m.obj_edge[o], neo = m.obj_edge[o + 1] - eo0;
  if (m.obj_tri[p + 1] - tp0 != nto || m.obj_edge[p + 1] - ep0 != neo) return false;
  for (int64_t k = 0; k < neo; ++k) {
    if (m.tp[ep0 + k] - tp0 != m.tp[eo0 + k] - to0 || m.tm[ep0 + k] - tp0 != m.tm[eo0 + k] - to0 ||
        m.ip[ep0 + k] != m.ip[eo0 + k] || m.im[ep0 + k] != m.im[eo0 + k])
      return false;
  }
  const double* x = m.xyz.data();
  const int32_t a0 = m.tri[3 * tp0], b0 = m.tri[3 * to0];
  const double tr[3] = {x[3 * b0] - x[3 * a0], x[3 * b0 + 1] - x[3 * a0 + 1], x[3 * b0 + 2] - x[3 * a0 + 2]};
  double ext = 0;
  for (int64_t k = 0; k < nto; ++k) ext = std::max(ext, m.hmax[tp0 + k]);
  const double tol = 1e-12 * (ext * double(nto) + std::fabs(tr[0]) + std::fabs(tr[1]) + std::fabs(tr[2]) +
                              std::fabs(x[3 * a0]) + std::fabs(x[3 * a0 + 1]) + std::fabs(x[3 * a0 + 2]));
  std::unordered_map<int32_t, int32_t> fwd, bwd;
  for (int64_t k = 0; k < 3 * nto; ++k) {
    const int32_t a = m.tri[3 * tp0 + k], b = m.tri[3 * to0 + k];
    auto f = fwd.emplace(a, b);
    auto g = bwd.emplace(b, a);
    if (f.first->second != b || g.first->second != a) return false;
    for (int c = 0; c < 3; ++c)
      if (std::fabs(x[3 * b + c] - x[3 * a + c] - tr[c]) > tol) return false;
  }
  return true;
}

static void find_translated_copies(Mesh& m) {
  m.geo_proto.assign(m.nobj, 0);
  std::vector<int64_t> protos;
  for (int64_t o = 0; o < m.nobj; ++o) {
    m.geo_proto[o] = int32_t(o);
    for (int64_t p : protos)
      if (translated_copy(m, p, o)) {
        m.geo_proto[o] = int32_t(p);
        break;
      }
    if (m.geo_proto[o] == o) protos.push_back(o);
  }
}

std::unique_ptr<Mesh> build_mesh(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                                 const int32_t* obj) {
  if (!xyz || !tri || nv <= 0 || nt <= 0) throw Error(BEM_E_INVALID, "empty mesh");
  if (nt > (int64_t(1) << 30) || nv > (int64_t(1) << 30)) throw Error(BEM_E_INVALID, "mesh too large");
  auto m = std::make_unique<Mesh>();
  m->nv = nv;
  m->nt = nt;
  m->xyz.assign(xyz, xyz + 3 * nv);
  m->tri.assign(tri, tri + 3 * nt);
  m->obj.assign(nt, 0);
  if (obj) m->obj.assign(obj, obj + nt);
  for (double x : m->xyz)
    if (!std::isfinite(x)) throw Error(BEM_E_NUMERIC, "non-finite vertex coordinate");
  // objects: contiguous, non-decreasing, ids 0..nobj-1
  if (m->obj[0] != 0) fail("object ids must start at 0");
  m->obj_tri.push_back(0);
  for (int64_t t = 1; t < nt; ++t) {
    if (m->obj[t] == m->obj[t - 1]) continue;
    if (m->obj[t] != m->obj[t - 1] + 1) fail("object ids must be contiguous and non-decreasing");
    m->obj_tri.push_back(t);
  }
  m->obj_tri.push_back(nt);
  m->nobj = int64_t(m->obj_tri.size()) - 1;

  // geometry
  m->area.resize(nt);
  m->normal.resize(3 * nt);
  m->centroid.resize(3 * nt);
  m->hmax.resize(nt);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* v = &m->tri[3 * t];
    for (int i = 0; i < 3; ++i)
      if (v[i] < 0 || v[i] >= nv) fail("triangle vertex index out of range");
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) fail("triangle with repeated vertex");
    const double* a = &m->xyz[3 * v[0]];
    const double* b = &m->xyz[3 * v[1]];
    const double* c = &m->xyz[3 * v[2]];
    double ab[3], ac[3], bc[3], cr[3];
    for (int k = 0; k < 3; ++k) {
      ab[k] = b[k] - a[k];
      ac[k] = c[k] - a[k];
      bc[k] = c[k] - b[k];
    }
    cr[0] = ab[1] * ac[2] - ab[2] * ac[1];
    cr[1] = ab[2] * ac[0] - ab[0] * ac[2];
    cr[2] = ab[0] * ac[1] - ab[1] * ac[0];
    double dbl = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    double lab = std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
    double lac = std::sqrt(ac[0] * ac[0] + ac[1] * ac[1] + ac[2] * ac[2]);
    double lbc = std::sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
    double h = std::max(lab, std::max(lac, lbc));
    if (!(dbl > 1e-12 * h * h)) fail("degenerate (zero-area) triangle " + std::to_string(t));
    m->area[t] = 0.5 * dbl;
    m->hmax[t] = h;
    for (int k = 0; k < 3; ++k) {
      m->normal[3 * t + k] = cr[k] / dbl;
      m->centroid[3 * t + k] = (a[k] + b[k] + c[k]) / 3.0;
    }
  }

  // edges: a forward occurrence (from < to) creates the edge, owned by T+ (library order)
  std::unordered_map<uint64_t, int32_t> eid;
  eid.reserve(size_t(3 * nt));
  m->tri_edge.assign(3 * nt, -1);
  m->tri_sign.assign(3 * nt, 0);
  for (int64_t t = 0; t < nt; ++t) {
    for (int i = 0; i < 3; ++i) {
      int32_t from = m->tri[3 * t + (i + 1) % 3], to = m->tri[3 * t + (i + 2) % 3];
      if (from < to) {
        auto ins = eid.emplace(key2(from, to), int32_t(m->ev.size() / 2));
        if (!ins.second) fail("edge traversed twice in the same direction (inconsistent orientation or non-manifold)");
        m->ev.push_back(from);
        m->ev.push_back(to);
        m->tp.push_back(int32_t(t));
        m->ip.push_back(int8_t(i));
        m->tri_edge[3 * t + i] = ins.first->second;
        m->tri_sign[3 * t + i] = 1;
      }
    }
  }
  m->ne = int64_t(m->ev.size() / 2);
  m->tm.assign(m->ne, -1);
  m->im.assign(m->ne, -1);
  for (int64_t t = 0; t < nt; ++t) {
    for (int i = 0; i < 3; ++i) {
      int32_t from = m->tri[3 * t + (i + 1) % 3], to = m->tri[3 * t + (i + 2) % 3];
      if (from > to) {
        auto it = eid.find(key2(to, from));
        if (it == eid.end()) fail("edge without a matching opposite traversal (open surface or inconsistent orientation)");
        int32_t n = it->second;
        if (m->tm[n] != -1) fail("edge shared by more than two triangles");
        m->tm[n] = int32_t(t);
        m->im[n] = int8_t(i);
        m->tri_edge[3 * t + i] = n;
        m->tri_sign[3 * t + i] = -1;
      }
    }
  }
  for (int64_t n = 0; n < m->ne; ++n) {
    if (m->tm[n] < 0) fail("open surface: edge with a single triangle");
    if (m->obj[m->tp[n]] != m->obj[m->tm[n]]) fail("objects share an edge (junction)");
  }
  // edges are grouped by object because they are ordered by T+
  m->obj_edge.assign(m->nobj + 1, 0);
  for (int64_t n = 0; n < m->ne; ++n) m->obj_edge[m->obj[m->tp[n]] + 1]++;
  for (int64_t o = 0; o < m->nobj; ++o) m->obj_edge[o + 1] += m->obj_edge[o];
  find_translated_copies(*m);

  // outward orientation: positive enclosed volume per object
  for (int64_t o = 0; o < m->nobj; ++o) {
    double vol = 0;
    for (int64_t t = m->obj_tri[o]; t < m->obj_tri[o + 1]; ++t) {
      const double* a = &m->xyz[3 * m->tri[3 * t]];
      const double* b = &m->xyz[3 * m->tri[3 * t + 1]];
      const double* c = &m->xyz[3 * m->tri[3 * t + 2]];
      vol += a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
             a[2] * (b[0] * c[1] - b[1] * c[0]);
    }
    if (!(vol > 0)) fail("object " + std::to_string(o) + " is inward-oriented (non-positive volume)");
  }

  // vertex fans.  In a counter-clockwise triangle (v, a, b) the triangle lies between the
  // edges (v, a) and (v, b); chaining a -> b around v must give a single cycle.
  std::vector<int64_t> cnt(nv + 1, 0);
  for (int64_t t = 0; t < nt; ++t)
    for (int i = 0; i < 3; ++i) cnt[m->tri[3 * t + i] + 1]++;
  for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
  std::vector<int32_t> arc_a(3 * nt), arc_b(3 * nt), arc_t(3 * nt);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
      for (int i = 0; i < 3; ++i) {
        int32_t v = m->tri[3 * t + i];
        int64_t p = fill[v]++;
        arc_a[p] = m->tri[3 * t + (i + 1) % 3];
        arc_b[p] = m->tri[3 * t + (i + 2) % 3];
        arc_t[p] = int32_t(t);
      }
  }
  m->vptr = cnt;
  m->vedge.assign(cnt[nv], -1);
  m->vtri.assign(cnt[nv], -1);
  for (int64_t v = 0; v < nv; ++v) {
    int64_t b0 = cnt[v], n = cnt[v + 1] - cnt[v];
    if (n == 0) continue;  // unused vertex
    if (n < 3) fail("vertex with fewer than three triangles");
    m->max_valence = std::max<int>(m->max_valence, int(n));
    // start at the first arc; follow a -> b
    int64_t cur = b0;
    for (int64_t k = 0; k < n; ++k) {
      int32_t a = arc_a[cur];
      auto it = eid.find(a < v ? key2(a, int32_t(v)) : key2(int32_t(v), a));
      m->vedge[b0 + k] = it->second;
      m->vtri[b0 + k] = arc_t[cur];
      int32_t nb = arc_b[cur];
      int64_t nxt = -1;
      for (int64_t p = b0; p < b0 + n; ++p)
        if (arc_a[p] == nb) {
          if (nxt != -1) fail("non-manifold vertex");
          nxt = p;
        }
      if (nxt == -1) fail("non-manifold vertex (open fan)");
      cur = nxt;
      if (k + 1 < n && cur == b0) fail("non-manifold vertex (several fans)");
    }
    if (cur != b0) fail("non-manifold vertex");
  }
  if (m->max_valence > kMaxValence)
    fail("vertex valence above " + std::to_string(kMaxValence) + " is not supported");

  // near pairs: shared vertex, or centroid distance below kNearFactor * max(h_T, h_T')
  double hall = 0, lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t t = 0; t < nt; ++t) {
    hall = std::max(hall, m->hmax[t]);
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], m->centroid[3 * t + k]);
      hi[k] = std::max(hi[k], m->centroid[3 * t + k]);
    }
  }
  double cell = kNearFactor * hall;
  int64_t gdim[3];
  for (int k = 0; k < 3; ++k) gdim[k] = std::max<int64_t>(1, std::min<int64_t>(1024, int64_t((hi[k] - lo[k]) / cell) + 1));
  auto gidx = [&](int64_t t, int k) {
    int64_t g = int64_t((m->centroid[3 * t + k] - lo[k]) / cell);
    return std::min<int64_t>(std::max<int64_t>(g, 0), gdim[k] - 1);
  };
  std::unordered_map<int64_t, std::vector<int32_t>> grid;
  for (int64_t t = 0; t < nt; ++t)
    grid[(gidx(t, 0) * gdim[1] + gidx(t, 1)) * gdim[2] + gidx(t, 2)].push_back(int32_t(t));
  // (triangle ranges on several host threads: graded meshes have hundreds of near pairs per
  // triangle; each range's lists are concatenated in order, so the result does not depend on
  // the thread count)
  m->near_ptr.assign(nt + 1, 0);
  const int nthr = int(std::max<int64_t>(1, std::min<int64_t>({int64_t(std::thread::hardware_concurrency()), 16,
                                                               nt / 2048 + 1})));
  std::vector<std::vector<int32_t>> part_idx(nthr);
  auto near_range = [&](int w) {
    const int64_t ta = nt * w / nthr, tb = nt * (w + 1) / nthr;
    std::vector<int32_t> cand;
    std::vector<int32_t>& out = part_idx[w];
    for (int64_t t = ta; t < tb; ++t) {
      cand.clear();
      int64_t g0 = gidx(t, 0), g1 = gidx(t, 1), g2 = gidx(t, 2);
      for (int64_t a = std::max<int64_t>(0, g0 - 1); a <= std::min(gdim[0] - 1, g0 + 1); ++a)
        for (int64_t b = std::max<int64_t>(0, g1 - 1); b <= std::min(gdim[1] - 1, g1 + 1); ++b)
          for (int64_t c = std::max<int64_t>(0, g2 - 1); c <= std::min(gdim[2] - 1, g2 + 1); ++c) {
            auto it = grid.find((a * gdim[1] + b) * gdim[2] + c);
            if (it == grid.end()) continue;
            for (int32_t s : it->second) {
              double dx = m->centroid[3 * t] - m->centroid[3 * s];
              double dy = m->centroid[3 * t + 1] - m->centroid[3 * s + 1];
              double dz = m->centroid[3 * t + 2] - m->centroid[3 * s + 2];
              double d = std::sqrt(dx * dx + dy * dy + dz * dz);
              if (d < kNearFactor * std::max(m->hmax[t], m->hmax[s])) cand.push_back(s);
            }
          }
      for (int i = 0; i < 3; ++i) {
        int32_t v = m->tri[3 * t + i];
        for (int64_t p = m->vptr[v]; p < m->vptr[v + 1]; ++p) cand.push_back(m->vtri[p]);
      }
      std::sort(cand.begin(), cand.end());
      cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
      out.insert(out.end(), cand.begin(), cand.end());
      m->near_ptr[t + 1] = int64_t(cand.size());
    }
  };
  {
    std::vector<std::thread> pool;
    for (int w = 1; w < nthr; ++w) pool.emplace_back(near_range, w);
    near_range(0);
    for (auto& th : pool) th.join();
  }
  for (int64_t t = 0; t < nt; ++t) m->near_ptr[t + 1] += m->near_ptr[t];
  m->near_idx.reserve(size_t(m->near_ptr[nt]));
  for (auto& p : part_idx) m->near_idx.insert(m->near_idx.end(), p.begin(), p.end());
  return m;
}

CellData build_cells(const Mesh& m) {
  CellData cd;
  cd.ncell = m.nv;
  int maxv = m.max_valence <= 8 ? 8 : kMaxValence;
  cd.maxv = maxv;
  const int64_t nc = cd.ncell;
  const int ns = 2 * maxv;
  cd.nval.assign(nc, 0);
  cd.vpos.assign(3 * nc, 0.0);
  cd.sub_m.assign(size_t(ns) * nc * 3, 0.0);
  cd.sub_c.assign(size_t(ns) * nc * 3, 0.0);
  cd.sub_area.assign(size_t(ns) * nc, 0.0);
  cd.sub_parent.assign(size_t(ns) * nc, -1);
  cd.alpha.assign(size_t(maxv) * nc, 0.0);
  cd.beta.assign(size_t(maxv) * ns * nc * 3, 0.0);
  cd.col0.assign(nc, -1);
  cd.colS.assign(m.ne, -1);
  cd.colT.assign(m.ne, -1);
  // cells of every object (a vertex belongs to the object of its triangles), object-local columns
  std::vector<int32_t> vobj(nc, -1);
  for (int64_t t = 0; t < m.nt; ++t)
    for (int i = 0; i < 3; ++i) vobj[m.tri[3 * t + i]] = m.obj[t];
  cd.obj_cell_ptr.assign(m.nobj + 1, 0);
  cd.obj_ncol.assign(m.nobj, 0);
  for (int64_t v = 0; v < nc; ++v)
    if (vobj[v] >= 0) cd.obj_cell_ptr[vobj[v] + 1]++;
  for (int64_t o = 0; o < m.nobj; ++o) cd.obj_cell_ptr[o + 1] += cd.obj_cell_ptr[o];
  cd.obj_cells.assign(cd.obj_cell_ptr[m.nobj], -1);
  {
    std::vector<int64_t> fill(cd.obj_cell_ptr.begin(), cd.obj_cell_ptr.end() - 1);
    for (int64_t v = 0; v < nc; ++v) {
      if (vobj[v] < 0) continue;
      cd.obj_cells[fill[vobj[v]]++] = int32_t(v);
      cd.col0[v] = cd.obj_ncol[vobj[v]];
      cd.obj_ncol[vobj[v]] += m.vptr[v + 1] - m.vptr[v];
    }
  }
  auto SUB = [&](int s, int64_t v) { return size_t(s) * nc + v; };
  for (int64_t v = 0; v < nc; ++v) {
    const int64_t b0 = m.vptr[v];
    const int N = int(m.vptr[v + 1] - b0);
    cd.nval[v] = N;
    const double* pv = &m.xyz[3 * v];
    for (int k = 0; k < 3; ++k) cd.vpos[3 * v + k] = pv[k];
    if (N == 0) continue;
    // sub-triangles in cyclic order: slot 2k in T_k next to E_k, slot 2k+1 in T_k next to E_{k+1}
    std::vector<std::array<double, 3>> M(N), Cc(N);
    for (int k = 0; k < N; ++k) {
      int32_t e = m.vedge[b0 + k];
      int32_t t = m.vtri[b0 + k];
      for (int c = 0; c < 3; ++c) {
        M[k][c] = 0.5 * (m.xyz[3 * m.ev[2 * e] + c] + m.xyz[3 * m.ev[2 * e + 1] + c]) - pv[c];
        Cc[k][c] = m.centroid[3 * t + c] - pv[c];
      }
    }
    auto cross_norm = [](const std::array<double, 3>& a, const std::array<double, 3>& b) {
      double x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
      return std::sqrt(x * x + y * y + z * z);
    };
    for (int k = 0; k < N; ++k) {
      int32_t t = m.vtri[b0 + k];
      for (int h = 0; h < 2; ++h) {
        int s = 2 * k + h;
        const auto& mm = h == 0 ? M[k] : M[(k + 1) % N];
        for (int c = 0; c < 3; ++c) {
          cd.sub_m[3 * SUB(s, v) + c] = mm[c];
          cd.sub_c[3 * SUB(s, v) + c] = Cc[k][c];
        }
        cd.sub_area[SUB(s, v)] = 0.5 * cross_norm(mm, Cc[k]);
        cd.sub_parent[SUB(s, v)] = t;
      }
    }
    // BC functions of the N incident edges
    for (int b = 0; b < N; ++b) {
      int32_t n = m.vedge[b0 + b];
      const double sigma = (m.ev[2 * n] == v) ? 1.0 : -1.0;  // source cell of va, sink cell of vb
      cd.alpha[size_t(b) * nc + v] = sigma / (2.0 * N);
      if (sigma > 0) cd.colS[n] = cd.col0[v] + b; else cd.colT[n] = cd.col0[v] + b;
      // flux F_i from t_i into t_{i+1}, i = 1..2N-1; F_0 = F_2N = 0
      auto F = [&](int i) { return (i <= 0 || i >= 2 * N) ? 0.0 : sigma * double(i - N) / (2.0 * N); };
      for (int i = 1; i <= 2 * N; ++i) {
        int s = (2 * b + i - 1) % (2 * N);
        int k = s / 2;
        // vertex opposite the edge shared with the previous / next sub-triangle
        const auto& q_prev = (s % 2 == 0) ? Cc[k] : M[(k + 1) % N];
        const auto& q_next = (s % 2 == 0) ? M[k] : Cc[k];
        double out_prev = -F(i - 1), out_next = F(i);
        for (int c = 0; c < 3; ++c)
          cd.beta[(((size_t(b) * ns) + s) * nc + v) * 3 + c] = out_prev * q_prev[c] + out_next * q_next[c];
        // the outer (dual half-edge) flux multiplies the vertex v itself, i.e. 0 in cell coordinates
      }
    }
  }
  for (int64_t n = 0; n < m.ne; ++n)
    if (cd.colS[n] < 0 || cd.colT[n] < 0) throw Error(BEM_E_MESH, "internal: BC cell columns missing");
  return cd;
}

void near_cells(const Mesh& m, std::vector<int64_t>& ptr, std::vector<int32_t>& idx) {
  // triangle ranges on several host threads, concatenated in order (as the near pairs)
  ptr.assign(m.nt + 1, 0);
  idx.clear();
  const int nthr = int(std::max<int64_t>(1, std::min<int64_t>({int64_t(std::thread::hardware_concurrency()), 16,
                                                               m.nt / 2048 + 1})));
  std::vector<std::vector<int32_t>> part(nthr);
  auto range = [&](int w) {
    const int64_t ta = m.nt * w / nthr, tb = m.nt * (w + 1) / nthr;
    std::vector<int32_t> c;
    std::vector<int64_t> stamp(m.nv, -1);  // last triangle that listed the vertex
    for (int64_t t = ta; t < tb; ++t) {
      c.clear();
      for (int64_t p = m.near_ptr[t]; p < m.near_ptr[t + 1]; ++p) {
        int32_t s = m.near_idx[p];
        for (int i = 0; i < 3; ++i) {
          const int32_t v = m.tri[3 * s + i];
          if (stamp[v] != t) {
            stamp[v] = t;
            c.push_back(v);
          }
        }
      }
      std::sort(c.begin(), c.end());
      part[w].insert(part[w].end(), c.begin(), c.end());
      ptr[t + 1] = int64_t(c.size());
    }
  };
  {
    std::vector<std::thread> pool;
    for (int w = 1; w < nthr; ++w) pool.emplace_back(range, w);
    range(0);
    for (auto& th : pool) th.join();
  }
  for (int64_t t = 0; t < m.nt; ++t) ptr[t + 1] += ptr[t];
  idx.reserve(size_t(ptr[m.nt]));
  for (auto& q : part) idx.insert(idx.end(), q.begin(), q.end());
}

}  // namespace bem
