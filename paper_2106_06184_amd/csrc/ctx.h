// Context, device memory accounting and the assembled operator object.
#pragma once

#include <functional>
#include <map>
#include <mutex>

#include "fill.h"
#include "internal.h"
#include "linalg.h"

namespace bem {

class Server;

// Pinned host staging per stream owner (context or serving slot): the first 64 doubles hold
// convergence scalars; the rest stages the per-column Krylov scalars and index lists.
constexpr size_t kPinnedBytes = 64 * 1024;
// largest half-row scratch of one fill chunk
constexpr size_t kFillScratchBytes = size_t(4) << 30;
int64_t fill_chunk_triangles(int64_t nt, int64_t row_len);
constexpr size_t kPinnedScalars = 64;
constexpr int kInnerNone = -1;  // operator without an equivalent-configuration solve

struct Ctx {
  int device = -1;
  size_t budget = 0;
  size_t used = 0;
  hipStream_t stream = nullptr;
  uint64_t next_handle = 1;
  std::map<uint64_t, std::unique_ptr<struct MeshObj>> meshes;
  std::map<uint64_t, std::unique_ptr<struct OpObj>> ops;
  double* pinned = nullptr;  // small pinned host buffer for convergence scalars
  std::unique_ptr<Server> server;
  std::mutex mu;             // guards `used` and the block cache (the serving threads allocate too)
  // Device blocks released by finished work, kept for reuse (hipMalloc / hipFree of the
  // multi-GB dense blocks cost milliseconds and synchronise the device).  `used` counts
  // blocks in use, `cached` the idle ones; both count against the budget, and idle blocks
  // are freed when a new allocation would not fit otherwise.
  std::multimap<size_t, void*> cache;
  size_t cached = 0;
  ~Ctx();
};

// Device allocations owned by one object; released (and un-accounted) on destruction.
class DevArena {
 public:
  explicit DevArena(Ctx* c) : ctx_(c) {}
  DevArena(const DevArena&) = delete;
  ~DevArena();
  void* raw(size_t bytes);
  template <class T>
  T* alloc(size_t n) {
    return static_cast<T*>(raw(sizeof(T) * (n ? n : 1)));
  }
  // Copies v to a new device buffer, ordered on the arena's stream and complete on return (the
  // kernels that read it may run on that stream, which does not synchronise with the null
  // stream).
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) {
      BEM_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, stream_));
      BEM_HIP(hipStreamSynchronize(stream_));
    }
    return p;
  }
  void set_stream(hipStream_t st) { stream_ = st; }
  hipStream_t stream() const { return stream_; }
  void release(void* p);
  bool owns(const void* p) const {
    for (const auto& b : blocks_)
      if (b.first == p) return true;
    return false;
  }
  size_t bytes() const { return total_; }

 private:
  Ctx* ctx_;
  hipStream_t stream_ = nullptr;
  std::vector<std::pair<void*, size_t>> blocks_;
  size_t total_ = 0;
};

struct MeshObj {
  std::unique_ptr<Mesh> mesh;
  std::unique_ptr<CellData> cells;  // built on first assemble
};

// Dense block: float64 storage, optional float32 copy, padded leading dimension.
struct Dense {
  double2* d64 = nullptr;
  float2* d32 = nullptr;
  int64_t rows = 0, cols = 0, ld = 0;
};

struct GmresWork;

// Groups the small dense products of concurrently solving requests into shared launches.
class ProductCombiner {
 public:
  virtual ~ProductCombiner() = default;
  // Runs the descriptors after the work already enqueued on st and before the work enqueued on
  // st after the call returns (possibly inside one grouped launch with other requests').
  virtual void run(const std::vector<GemvDesc>& ds, hipStream_t st) = 0;
};

struct OpObj {
  Ctx* ctx;
  const Mesh* m;
  const CellData* cells;
  DevArena mem;
  // problem
  double freq = 0, k0 = 0;
  std::vector<cd> epsc, kint;
  std::vector<double> mur;
  cd eps_bg = 1.0, kbg = 0.0;
  double mu_bg = 1.0;
  int precision = BEM_FP64;
  // sizes
  int64_t ne = 0, nt = 0, nq = 0, nobj = 0, N = 0, Neq = 0;
  // device tables
  double* geo = nullptr;
  int32_t *tp = nullptr, *tm = nullptr, *tri_edge = nullptr, *kept = nullptr;
  int8_t *ip = nullptr, *im = nullptr, *tri_sign = nullptr;
  int64_t* obj_tri_d = nullptr;
  int64_t* ix_ptr = nullptr;
  int32_t* ix_idx = nullptr;
  double* ix_val = nullptr;
  double2* eps_inv_edge = nullptr;  // 1/eps_c of the object of every edge
  // host copies of the per-object ranges
  std::vector<int64_t> obj_tri, obj_edge, obj_q;
  // dense blocks
  std::vector<Dense> LA_int, Lphi_int, K_int, K_bg;  // per object (block-diagonal operators)
  Dense LA_bg, Lphi_bg;                              // all pairs (background coupling)
  int formulation = BEM_FORM_SLDM;
  // repeated objects: geo_rep[o] = the object whose background-wavenumber blocks o shares
  // (a translated copy), mat_rep[o] = the object whose interior blocks it shares (a translated
  // copy with the same material); o itself when it owns them
  std::vector<int64_t> geo_rep, mat_rep;
  Dense Km;  // eAEFIE: K~ at k_l over all pairs (K_bg[o] are then views of its diagonal blocks)
  // nested solve and preconditioners
  int inner_mode = BEM_INNER_GMRES;  // kInnerNone for the eAEFIE (no equivalent configuration)
  bool precond = false;
  std::vector<Dense> Minv;           // per object: inverse of M_eq (direct inner solve)
  std::vector<Dense> SigP, SigEq;    // per object: inverses of the charge Schur complements
  double2* pcW = nullptr;            // per edge: inverse of the 2x2 diagonal block of P (4 entries)
  double2* lam_bg = nullptr;         // per triangle: diag L^phi_l
  double2* lam_int = nullptr;        // per triangle: diag L^phi (object wavenumber)
  double2* eq_d = nullptr;           // per edge: 1 / (mu_l diag L^A_l)
  // solver settings and work
  double inner_tol = 1e-12;
  int inner_restart = 200, inner_maxit = 4000;
  int last_inner_iters = 0, max_inner_iters = 0;
  double fill_seconds = 0, fill_bytes = 0, kernel_evals = 0;
  double inv_min_pivot = HUGE_VAL, inv_probe_err = 0;  // worst health of the dense inversions
  std::unique_ptr<GmresWork> inner_ws, outer_ws;
  double2* work = nullptr;  // vector workspace
  int64_t work_len = 0;
  ProductCombiner* comb = nullptr;  // set by the serving loop
  // set by the serving loop: adds bytes to the request's admitted reservation, false when they
  // do not fit next to the other admitted requests (memory a solve takes beyond its estimate)
  std::function<bool(size_t)> reserve;
  hipStream_t stream = nullptr;  // stream of the operator's work
  double* pinned = nullptr;      // pinned host scalars for convergence checks

  explicit OpObj(Ctx* c) : ctx(c), m(nullptr), cells(nullptr), mem(c), stream(c->stream), pinned(c->pinned) {}
  ~OpObj();
};

using ApplyFn = std::function<void(const double2* x, double2* y)>;

struct GmresResult {
  int iters = 0;
  double relres = 0;  // estimated (Arnoldi) relative residual
  bool converged = false;
};

struct GmresWork {
  int64_t n = 0, ldv = 0;
  int m = 0;
  double2 *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *h2 = nullptr;
  double2 *z = nullptr, *z2 = nullptr;  // preconditioned-vector temporaries
  double2* nrm = nullptr;
  double* res = nullptr;
  KrylovScratch ks{};
  const char* tag = nullptr;  // progress label (BEM_VERBOSE)
};

std::unique_ptr<GmresWork> make_gmres_work(DevArena& mem, int64_t n, int m);
// Right-preconditioner-free restarted GMRES (CGS2 Arnoldi, complex Givens, float64) on `st`.
// x holds the initial guess (zeroed when x_zero) and receives the solution.
// M (optional) is a right preconditioner: GMRES runs on A M and returns x = M u.
GmresResult gmres(GmresWork& w, double* pinned, const ApplyFn& A, const double2* b, double2* x, bool x_zero,
                  double tol, int maxit, hipStream_t st, const ApplyFn* M = nullptr);
void apply_precond(OpObj& op, const double2* r, double2* x, bool fp32, hipStream_t st);
void apply_precond_eq(OpObj& op, const double2* r, double2* x, bool fp32, hipStream_t st);

// Operator construction and application.
void assemble_op(OpObj& op, MeshObj& mo, const bem_problem& prob);
// y = A x for `block`, nrhs columns (leading dimensions = the block's size); nrhs > 1 runs the
// dense products on matrix cores.
void apply_block(OpObj& op, int block, const double2* x, double2* y, int64_t nrhs, hipStream_t st);
void apply_meq(OpObj& op, const double2* x, double2* y, bool fp32, hipStream_t st);
void apply_final(OpObj& op, const double2* x, double2* y, bool fp32, double inner_tol, hipStream_t st);
void export_block(OpObj& op, int block, bem_c64* host);
// Far field of nexc solutions (host H, E): N per (solution, direction) and the bistatic RCS.
void far_field(OpObj& op, const bem_c64* H, const bem_c64* E, int64_t nexc, const double* rhat, int64_t ndir,
               bem_c64* N, double* rcs, hipStream_t st);
void near_field(OpObj& op, const bem_c64* H, const bem_c64* E, const bem_c64* rho, int64_t nexc,
                const bem_excitation* exc, const double* pts, int64_t npts, bem_c64* Eout, bem_c64* Hout,
                hipStream_t st);
// Upper bound of the device bytes of one request (assembly peak or solve peak), for admission.
size_t estimate_request_bytes(int64_t nt, int64_t nobj, int precision, int restart, int64_t nexc,
                              int formulation = BEM_FORM_SLDM);
// GMRES restart chosen when bem_solve_opts.restart <= 0 (N final unknowns, nexc excitations).
constexpr double kAutoKrylovBytes = 8.0e9;
int auto_restart(int64_t N, int64_t nexc);
int solve_op(OpObj& op, const bem_excitation* exc, int64_t nexc, const bem_solve_opts& opts, bem_c64* H, bem_c64* E,
             bem_c64* rho, bem_solve_info* info, hipStream_t st);

}  // namespace bem
