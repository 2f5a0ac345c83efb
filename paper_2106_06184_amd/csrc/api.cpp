// C ABI of libbem: argument checks, handle tables, status codes and error messages.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "ctx.h"
#include "dense.h"
#include "linalg.h"
#include "prof.h"
#include "serve.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const bem::Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(BEM_E_NOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(BEM_E_INVALID, e.what());
  }
}

void need_device(bem_ctx* c) {
  auto* ctx = reinterpret_cast<bem::Ctx*>(c);
  if (ctx->device < 0) throw bem::Error(BEM_E_DEVICE, "host-only context (created with device = -1)");
  BEM_HIP(hipSetDevice(ctx->device));
}

bem::Ctx* C(bem_ctx* c) {
  if (!c) throw bem::Error(BEM_E_INVALID, "null context");
  return reinterpret_cast<bem::Ctx*>(c);
}

bem::MeshObj& mesh_of(bem::Ctx* ctx, bem_mesh_h h) {
  auto it = ctx->meshes.find(h);
  if (it == ctx->meshes.end()) throw bem::Error(BEM_E_INVALID, "unknown mesh handle");
  return *it->second;
}

bem::OpObj& op_of(bem::Ctx* ctx, bem_op_h h) {
  auto it = ctx->ops.find(h);
  if (it == ctx->ops.end()) throw bem::Error(BEM_E_INVALID, "unknown operator handle");
  return *it->second;
}

}  // namespace

namespace bem {
Ctx::~Ctx() {
  server.reset();
  ops.clear();
  meshes.clear();
  if (pinned) (void)hipHostFree(pinned);
  if (stream) (void)hipStreamDestroy(stream);
  for (auto& kv : cache) (void)hipFree(kv.second);
  cache.clear();
}
}  // namespace bem

extern "C" {

int bem_create(int device, size_t hbm_budget_bytes, bem_ctx** out) {
  return guarded([&]() -> int {
    if (!out) return fail(BEM_E_INVALID, "null output pointer");
    auto ctx = std::make_unique<bem::Ctx>();
    ctx->device = device;
    if (device >= 0) {
      int n = 0;
      if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
        (void)hipGetLastError();
        return fail(BEM_E_DEVICE, "no such HIP device");
      }
      BEM_HIP(hipSetDevice(device));
      bem::noalloc_scratch_init(device);  // device address of the fixed inversion workspace
      BEM_HIP(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      BEM_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), bem::kPinnedBytes, hipHostMallocDefault));
      size_t fr = 0, tot = 0;
      BEM_HIP(hipMemGetInfo(&fr, &tot));
      // the default leaves the HIP runtime its own room (scratch of the queues, kernel
      // arguments, other libraries): the block cache keeps freed blocks up to the budget, and a
      // budget of all free memory has starved the runtime of queue resources
      const size_t headroom = std::max<size_t>(size_t(4) << 30, tot / 32);
      ctx->budget = hbm_budget_bytes ? hbm_budget_bytes : (fr > 2 * headroom ? fr - headroom : fr / 2);
    } else {
      ctx->budget = hbm_budget_bytes;
    }
    *out = reinterpret_cast<bem_ctx*>(ctx.release());
    return BEM_OK;
  });
}

void bem_destroy(bem_ctx* c) {
  if (!c) return;
  auto* ctx = reinterpret_cast<bem::Ctx*>(c);
  if (ctx->device >= 0) (void)hipSetDevice(ctx->device);
  delete ctx;
}

const char* bem_last_error(const bem_ctx*) { return g_err.c_str(); }

int bem_mesh_load(bem_ctx* c, const double* xyz, int64_t nv, const int32_t* tri, int64_t nt, const int32_t* obj,
                  bem_mesh_h* out) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (!out) return fail(BEM_E_INVALID, "null output pointer");
    auto mo = std::make_unique<bem::MeshObj>();
    mo->mesh = bem::build_mesh(xyz, nv, tri, nt, obj);
    const uint64_t h = ctx->next_handle++;
    ctx->meshes[h] = std::move(mo);
    *out = h;
    return BEM_OK;
  });
}

int bem_mesh_info(bem_ctx* c, bem_mesh_h h, int64_t* n_tri, int64_t* n_edge, int64_t* n_obj, int64_t* n_unknowns) {
  return guarded([&]() -> int {
    const bem::Mesh& m = *mesh_of(C(c), h).mesh;
    if (n_tri) *n_tri = m.nt;
    if (n_edge) *n_edge = m.ne;
    if (n_obj) *n_obj = m.nobj;
    if (n_unknowns) *n_unknowns = 2 * m.ne + m.nt - m.nobj;
    return BEM_OK;
  });
}

int bem_edge_table(bem_ctx* c, bem_mesh_h h, int32_t* va, int32_t* vb, int32_t* tplus, int32_t* tminus) {
  return guarded([&]() -> int {
    const bem::Mesh& m = *mesh_of(C(c), h).mesh;
    for (int64_t n = 0; n < m.ne; ++n) {
      if (va) va[n] = m.ev[2 * n];
      if (vb) vb[n] = m.ev[2 * n + 1];
      if (tplus) tplus[n] = m.tp[n];
      if (tminus) tminus[n] = m.tm[n];
    }
    return BEM_OK;
  });
}

int bem_near_pairs(bem_ctx* c, bem_mesh_h h, int64_t* ptr, int32_t* idx) {
  return guarded([&]() -> int {
    const bem::Mesh& m = *mesh_of(C(c), h).mesh;
    if (!ptr) return fail(BEM_E_INVALID, "null ptr");
    std::memcpy(ptr, m.near_ptr.data(), sizeof(int64_t) * m.near_ptr.size());
    if (idx) std::memcpy(idx, m.near_idx.data(), sizeof(int32_t) * m.near_idx.size());
    return BEM_OK;
  });
}

int bem_far_field(bem_ctx* c, bem_op_h h, const bem_c64* H, const bem_c64* E, int64_t nexc, const double* rhat,
                  int64_t ndir, bem_c64* N, double* rcs) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    bem::OpObj& op = op_of(ctx, h);
    need_device(c);
    bem::far_field(op, H, E, nexc, rhat, ndir, N, rcs, op.stream);
    return BEM_OK;
  });
}

int bem_near_field(bem_ctx* c, bem_op_h h, const bem_c64* H, const bem_c64* E, const bem_c64* rho, int64_t nexc,
                   const bem_excitation* exc, const double* points, int64_t npts, bem_c64* E_out, bem_c64* H_out) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    bem::OpObj& op = op_of(ctx, h);
    need_device(c);
    bem::near_field(op, H, E, rho, nexc, exc, points, npts, E_out, H_out, op.stream);
    return BEM_OK;
  });
}

int bem_mesh_copies(bem_ctx* c, bem_mesh_h h, int32_t* proto) {
  return guarded([&]() -> int {
    const bem::Mesh& m = *mesh_of(C(c), h).mesh;
    if (!proto) return fail(BEM_E_INVALID, "null proto");
    std::memcpy(proto, m.geo_proto.data(), sizeof(int32_t) * m.geo_proto.size());
    return BEM_OK;
  });
}

int bem_assemble(bem_ctx* c, bem_mesh_h h, const bem_problem* prob, bem_op_h* out) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (!prob || !out) return fail(BEM_E_INVALID, "null argument");
    bem::MeshObj& mo = mesh_of(ctx, h);
    need_device(c);
    auto op = std::make_unique<bem::OpObj>(ctx);
    bem::assemble_op(*op, mo, *prob);
    const uint64_t id = ctx->next_handle++;
    ctx->ops[id] = std::move(op);
    *out = id;
    return BEM_OK;
  });
}

int bem_apply(bem_ctx* c, bem_op_h h, int block, const void* x, void* y, int64_t nrhs, void* stream) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    bem::OpObj& op = op_of(ctx, h);
    need_device(c);
    if (!x || !y || nrhs < 0) return fail(BEM_E_INVALID, "invalid vectors");
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
    int64_t rows, cols;
    switch (block) {
      case BEM_BLOCK_FINAL: rows = cols = op.N; break;
      case BEM_BLOCK_LPHI_INT:
      case BEM_BLOCK_LPHI_BG: rows = cols = op.nt; break;
      case BEM_BLOCK_MEQ: rows = cols = op.Neq; break;
      case BEM_BLOCK_LA_INT:
      case BEM_BLOCK_K_INT:
      case BEM_BLOCK_LA_BG:
      case BEM_BLOCK_K_BG:
      case BEM_BLOCK_K_M:
      case BEM_BLOCK_IX: rows = cols = op.ne; break;
      default: return fail(BEM_E_INVALID, "unknown block");
    }
    if (op.precision == BEM_FP32) {
      // float32 vectors: widened into float64 work columns, products on the float32 blocks,
      // results rounded back (chunks of up to 256 columns)
      const float2* xp = static_cast<const float2*>(x);
      float2* yp = static_cast<float2*>(y);
      bem::DevArena tmp(ctx);
      tmp.set_stream(st);
      const int64_t cb = std::min<int64_t>(256, nrhs);
      double2* xw = tmp.alloc<double2>(size_t(cols) * cb);
      double2* yw = tmp.alloc<double2>(size_t(rows) * cb);
      for (int64_t r0 = 0; r0 < nrhs; r0 += 256) {
        const int64_t nr = std::min<int64_t>(256, nrhs - r0);
        bem::launch_cast_f64(xp + r0 * cols, nr, cols, cols, xw, cols, st);
        bem::apply_block(op, block, xw, yw, nr, st);
        bem::launch_cast_f32(yw, nr, rows, rows, yp + r0 * rows, rows, st);
      }
      BEM_HIP(hipStreamSynchronize(st));
      return BEM_OK;
    }
    const double2* xp = static_cast<const double2*>(x);
    double2* yp = static_cast<double2*>(y);
    // columns go through the matrix-core products in chunks of up to 256
    for (int64_t r0 = 0; r0 < nrhs; r0 += 256)
      bem::apply_block(op, block, xp + r0 * cols, yp + r0 * rows, std::min<int64_t>(256, nrhs - r0), st);
    return BEM_OK;
  });
}

int bem_dense_invert(bem_ctx* c, void* A, int64_t n, int64_t ld, void* stream, double* health) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    need_device(c);
    if (!A || n < 0 || ld < n) return fail(BEM_E_INVALID, "invalid matrix");
    if (n == 0) return BEM_OK;
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
    bem::DevArena mem(ctx);
    mem.set_stream(st);
    bem::DenseScratch ws = bem::dense_scratch_at(mem.alloc<double2>(bem::dense_scratch_elems(n)), n);
    bem::dense_invert(static_cast<double2*>(A), n, ld, ws, st);
    const bem::DenseHealth h = bem::dense_health(ws, st);
    if (health) {
      health[0] = h.min_pivot_ratio;
      health[1] = h.probe_error;
    }
    if (!bem::dense_health_ok(h)) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "elimination without pivoting broke down: smallest pivot ratio %.3e, probe error %.3e",
                    h.min_pivot_ratio, h.probe_error);
      return fail(BEM_E_NUMERIC, msg);
    }
    return BEM_OK;
  });
}

int bem_dense_invert_noalloc(bem_ctx* c, void* A, int64_t n, int64_t ld, void* stream, double* health) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    need_device(c);
    if (!A || n < 0 || ld < n) return fail(BEM_E_INVALID, "invalid matrix");
    if (n == 0) return BEM_OK;
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : ctx->stream;
    bem::DenseHealth h{};
    bem::dense_invert_noalloc(ctx->device, static_cast<double2*>(A), n, ld, &h, st);
    if (health) {
      health[0] = h.min_pivot_ratio;
      health[1] = h.probe_error;
    }
    if (!bem::dense_health_ok(h)) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "elimination without pivoting broke down: smallest pivot ratio %.3e, probe error %.3e",
                    h.min_pivot_ratio, h.probe_error);
      return fail(BEM_E_NUMERIC, msg);
    }
    return BEM_OK;
  });
}

int bem_block_export(bem_ctx* c, bem_op_h h, int block, bem_c64* host_dst) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    bem::OpObj& op = op_of(ctx, h);
    need_device(c);
    if (!host_dst) return fail(BEM_E_INVALID, "null destination");
    bem::export_block(op, block, host_dst);
    return BEM_OK;
  });
}

int bem_set_inner_tol(bem_ctx* c, bem_op_h h, double tol) {
  return guarded([&]() -> int {
    bem::OpObj& op = op_of(C(c), h);
    if (!(tol > 0)) return fail(BEM_E_INVALID, "tolerance must be positive");
    op.inner_tol = tol;
    return BEM_OK;
  });
}

int bem_solve(bem_ctx* c, bem_op_h h, const bem_excitation* exc, int64_t nexc, const bem_solve_opts* opts, bem_c64* H,
              bem_c64* E, bem_c64* rho, bem_solve_info* info) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    bem::OpObj& op = op_of(ctx, h);
    need_device(c);
    if (!opts) return fail(BEM_E_INVALID, "null options");
    int st = bem::solve_op(op, exc, nexc, *opts, H, E, rho, info, ctx->stream);
    if (st == BEM_E_NOT_CONVERGED) g_err = "GMRES did not reach the tolerance within maxit";
    return st;
  });
}

int bem_release(bem_ctx* c, uint64_t h) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (ctx->device >= 0) BEM_HIP(hipSetDevice(ctx->device));
    if (ctx->ops.erase(h)) return BEM_OK;
    if (ctx->meshes.count(h)) {
      for (auto& kv : ctx->ops)
        if (kv.second->m == ctx->meshes[h]->mesh.get())
          return fail(BEM_E_INVALID, "mesh still used by an operator");
      ctx->meshes.erase(h);
      return BEM_OK;
    }
    return fail(BEM_E_INVALID, "unknown handle");
  });
}

int bem_memory_in_use(bem_ctx* c, size_t* bytes) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (!bytes) return fail(BEM_E_INVALID, "null output");
    std::lock_guard<std::mutex> g(ctx->mu);
    *bytes = ctx->used;
    return BEM_OK;
  });
}

int bem_op_stats_get(bem_ctx* c, bem_op_h h, bem_op_stats* out) {
  return guarded([&]() -> int {
    bem::OpObj& op = op_of(C(c), h);
    if (!out) return fail(BEM_E_INVALID, "null output");
    out->fill_seconds = op.fill_seconds;
    out->fill_bytes = op.fill_bytes;
    out->kernel_evals = op.kernel_evals;
    out->device_bytes = double(op.mem.bytes());
    int64_t filled = 0;
    for (int64_t o = 0; o < op.nobj; ++o) filled += op.mat_rep[o] == o ? 1 : 0;
    out->interiors_filled = double(filled);
    out->inverse_min_pivot_ratio = op.inv_min_pivot;
    out->inverse_probe_error = op.inv_probe_err;
    return BEM_OK;
  });
}

int bem_profile_enable(int on) {
  return guarded([&]() -> int {
    bem::Profiler::get().enable(on != 0);
    return BEM_OK;
  });
}

int bem_profile_read(int cls, int64_t* launches, double* ms, double* bytes, double* work) {
  return guarded([&]() -> int {
    if (cls < 0 || cls >= bem::KC_COUNT) return fail(BEM_E_INVALID, "unknown kernel class");
    bem::ClassStats s = bem::Profiler::get().read(cls);
    if (launches) *launches = s.launches;
    if (ms) *ms = s.ms;
    if (bytes) *bytes = s.bytes;
    if (work) *work = s.work;
    return BEM_OK;
  });
}

int bem_submit(bem_ctx* c, const bem_request* req, bem_ticket* out) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    need_device(c);
    if (!req || !out) return fail(BEM_E_INVALID, "null argument");
    if (!ctx->server) ctx->server = std::make_unique<bem::Server>(ctx);
    *out = ctx->server->submit(*req);
    return BEM_OK;
  });
}

int bem_poll(bem_ctx* c, bem_ticket t, bem_solve_info* info) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (!ctx->server) return fail(BEM_E_INVALID, "unknown ticket");
    std::string msg;
    int st = ctx->server->poll(t, info, &msg);
    if (st < 0) g_err = msg;
    return st;
  });
}

int bem_drain(bem_ctx* c) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    if (ctx->server) ctx->server->drain();
    return BEM_OK;
  });
}

int bem_serve_stats(bem_ctx* c, int64_t* launches, int64_t* products) {
  return guarded([&]() -> int {
    bem::Ctx* ctx = C(c);
    int64_t l = 0, p = 0;
    if (ctx->server) ctx->server->combiner_stats(&l, &p);
    if (launches) *launches = l;
    if (products) *products = p;
    return BEM_OK;
  });
}

}  // extern "C"
