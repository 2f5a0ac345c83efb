/*
 * bem.h - C ABI of the MI355X dense single-layer dual-mesh BEM library (libbem.so).
 *
 * The library assembles and applies the Galerkin operators of the single-layer
 * dual-mesh boundary element method for penetrable objects (Sharma & Triverio,
 * Sec. II) on one AMD Instinct MI355X (gfx950) and solves the final system
 * (eq. finalsystem) with GMRES, the equivalent-configuration system
 * (eq. AEFIEeqvdis) being solved on the fly for every product (Sec. III).
 *
 * Conventions
 *  - Every call returns a status code (BEM_OK = 0, negative on error); no
 *    exception or signal crosses the ABI.  bem_last_error() describes the last
 *    failure on the calling thread.
 *  - Handles are opaque 64-bit integers owned by the context; bem_release()
 *    frees them.  The library owns every device-resident operator and every
 *    Krylov state; the caller owns all buffers it passes in.
 *  - Complex numbers are interleaved (re, im) pairs: bem_c64 for float64,
 *    two floats for float32.
 *  - Time dependence e^{+j omega t}; G = e^{-jkR}/(4 pi R) (eq. hgf);
 *    eps_c = eps_r - j sigma/(omega eps0) (eq. epsrc); mu0 = 4 pi 1e-7 H/m.
 *  - Unknown ordering of the final system: [a; e; x3] with a = jk0 H (one per
 *    edge, RWG), e = E/eta0 (one per edge, Buffa-Christiansen), x3 = -c0 rho'
 *    (one per triangle minus one per object; each object's highest-index
 *    triangle carries minus the sum of its other charges).
 *  - Edges are numbered by the library (bem_edge_table gives their vertex
 *    pairs); triangles and vertices keep the caller's numbering.
 *  - A context is not thread-safe: calls on one context must not overlap, except
 *    bem_poll, which may be called from any thread.
 */
#ifndef BEM_H
#define BEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_ctx bem_ctx;
typedef uint64_t bem_mesh_h;
typedef uint64_t bem_op_h;
typedef uint64_t bem_ticket;
typedef struct { double re, im; } bem_c64;

enum {
  BEM_OK = 0,
  BEM_PENDING = 1,
  BEM_E_INVALID = -1,       /* bad argument, unknown handle, wrong state */
  BEM_E_MESH = -2,          /* mesh not closed / not 2-manifold / not outward / degenerate */
  BEM_E_NOMEM = -3,         /* over the context's HBM budget, or allocation failure */
  BEM_E_NOT_CONVERGED = -4, /* iteration limit reached; best iterate written */
  BEM_E_DEVICE = -5,        /* HIP runtime error, or a device call on a host-only context */
  BEM_E_NUMERIC = -6        /* NaN/Inf in an input or in a residual */
};

/* Precision of an operator (bem_problem.precision).
 * BEM_FP64: float64 blocks and products.
 * BEM_FP32: the fill runs in float64 and is rounded once to float32; only the float32 blocks
 *   (and float32 copies of the nested-solve and preconditioner inverses) are kept, a third of the
 *   float64-plus-float32 memory; every product reads float32 storage, and bem_solve refines in
 *   float64 vectors: its GMRES sweeps and residuals r = b - A x use the float32 operator, so the
 *   solution converges to that of the float32-rounded operator (its difference from the float64
 *   one is the rounding times the condition number).  bem_apply takes and returns float32 vectors.
 * BEM_MIXED: float64 blocks plus float32 copies; float32 products in the late steps of each
 *   refinement sweep, float64 residuals (see bem_problem.precision). */
enum { BEM_FP64 = 0, BEM_FP32 = 1, BEM_MIXED = 2 };

/* Dense operator blocks addressable through bem_apply / bem_block_export. */
enum {
  BEM_BLOCK_FINAL = 0,    /* the final system of eq. finalsystem, (N x N), N = 2 NE + NQ */
  BEM_BLOCK_LA_INT = 1,   /* L^(A) at the object wavenumber k (eq. opLAhgf), NE x NE, block-diagonal */
  BEM_BLOCK_LPHI_INT = 2, /* L^(phi) at k (eq. opLphihgf), NT x NT, block-diagonal */
  BEM_BLOCK_K_INT = 3,    /* K~ at k (eq. opKhgf) on BC sources, NE x NE, block-diagonal */
  BEM_BLOCK_LA_BG = 4,    /* L^(A) at the background wavenumber k_l, NE x NE, all pairs */
  BEM_BLOCK_LPHI_BG = 5,  /* L^(phi) at k_l, NT x NT, all pairs */
  BEM_BLOCK_K_BG = 6,     /* K~ at k_l, NE x NE, block-diagonal */
  BEM_BLOCK_IX = 7,       /* Gram matrix I_x (BC tested with n x RWG), NE x NE, sparse */
  BEM_BLOCK_MEQ = 8,      /* equivalent-configuration matrix of eq. AEFIEeqvdis, (NE+NQ)^2 */
  BEM_BLOCK_MEQ_INV = 9,  /* its device inverse (direct nested solve only), (NE+NQ)^2,
                             block-diagonal; ordering [edges; kept charges] per object */
  BEM_BLOCK_K_M = 10      /* K~ at k_l over every object pair, NE x NE (eAEFIE formulation only) */
};

/* Context.  device >= 0 selects a HIP device; device = -1 gives a host-only
 * context on which mesh loading, validation and the mesh queries work but
 * assemble/apply/solve return BEM_E_DEVICE.  hbm_budget_bytes = 0 means the
 * free device memory less a reserve for the HIP runtime (1/32 of the device, at
 * least 4 GiB).  Errors: BEM_E_DEVICE (no such device). */
int bem_create(int device, size_t hbm_budget_bytes, bem_ctx** out);
void bem_destroy(bem_ctx* ctx);
/* Message of the last failing call on this thread; valid until the next call. */
const char* bem_last_error(const bem_ctx* ctx);

/* Load a closed triangle mesh (Sec. II: objects with closed surfaces and outward
 * normal).  xyz: nv*3 float64 (m), host; tri: nt*3 int32, counter-clockwise about
 * the outward normal, host; obj: nt int32 object ids 0..n_obj-1, non-decreasing
 * along the triangle list (each object contiguous), or NULL for one object.
 * Everything is copied.  BEM_E_MESH if a surface is open, non-manifold,
 * inconsistently or inward oriented, has a degenerate triangle, or objects
 * share an edge (junctions are not supported, Sec. II-E). */
int bem_mesh_load(bem_ctx* ctx, const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                  const int32_t* obj, bem_mesh_h* out);
/* Sizes: triangles, edges (RWG and BC functions), objects and final unknowns
 * N = 2 NE + NT - n_obj. */
int bem_mesh_info(bem_ctx* ctx, bem_mesh_h mesh, int64_t* n_tri, int64_t* n_edge, int64_t* n_obj,
                  int64_t* n_unknowns);
/* Edge table in the library's order (host buffers of NE entries each, any may be
 * NULL): vertex pair va < vb, T+ (triangle traversing va -> vb counter-
 * clockwise) and T-.  The RWG of an edge flows from T+ into T- with unit flux;
 * its BC function flows from the dual cell of va into that of vb. */
int bem_edge_table(bem_ctx* ctx, bem_mesh_h mesh, int32_t* va, int32_t* vb, int32_t* tplus,
                   int32_t* tminus);
/* Near-pair structure used by the singular quadrature: for each triangle T the
 * sorted list of triangles T' sharing a vertex with T or whose centroid lies
 * closer than (2 - 2e-9) * max(longest edge of T, of T').  ptr: NT+1 int64, idx:
 * ptr[NT] int32 (call once with idx = NULL to size it).  Host buffers. */
int bem_near_pairs(bem_ctx* ctx, bem_mesh_h mesh, int64_t* ptr, int32_t* idx);
/* Repeated objects (Sec. II-F): proto[o] (host, n_obj int32) = the first object of which
 * object o is a translated copy (its triangles, in order, are that object's moved by one
 * translation, to 1e-12 of the coordinates, with a one-to-one vertex correspondence, and its
 * edge table has the same local T+, T- and free vertices), or o itself.  Assembly shares the
 * object-local blocks of such copies unless bem_problem.no_reuse is set. */
int bem_mesh_copies(bem_ctx* ctx, bem_mesh_h mesh, int32_t* proto);

typedef struct { bem_c64 eps_r; double mu_r, sigma; } bem_material;

/* How the equivalent-configuration system (eq. AEFIEeqvdis) is solved inside every product
 * (Sec. III): directly (its inverse is formed once per assembly; the paper's route for small
 * objects) or by nested GMRES (its route for large objects).  DIRECT inverts the augmented
 * (NE_o + NQ_o)^2 matrix of each object.  SCHUR uses that the right-hand side has no charge
 * part: the second row gives w = k0^-2 F D u, and substituting it leaves
 * S u = r with S = mu_l L^A_l - (eps_l k0^2)^-1 D^T L^phi_l D (NE_o x NE_o; exact because the
 * charges of D u sum to zero on each object), so only S is inverted.  Its conditioning grows
 * like (k_l h)^-2, h the longest edge, so AUTO takes SCHUR when |k_l| h >= 0.01 and
 * NE_o <= 32768, else DIRECT while NE_o + NQ_o <= 16384, else GMRES. */
enum { BEM_INNER_AUTO = 0, BEM_INNER_GMRES = 1, BEM_INNER_DIRECT = 2, BEM_INNER_SCHUR = 3 };

/* Formulation of the final system.  SLDM: eq. finalsystem, the external problem uses only
 * single-layer operators and C1, C2 come from the equivalent configuration (eqs. C1, C2).
 * EAEFIE: the comparison formulation of Sec. II-F on the same homogeneous background, with C1
 * and C2 replaced by the external double-layer operator K~_m over every object pair and zero;
 * in the sign convention of the unknowns [jk0 H; E / eta0; -c0 rho] used here C1 = I_x/2 - K~_m
 * (the printed K~_m - I_x/2 goes with the printed sign of the middle block), so for a single
 * object both give the same matrix.  No equivalent-configuration solve is made (inner_mode is
 * ignored); K~_m (NE x NE) replaces the per-object K~_l blocks and nested-solve inverses. */
enum { BEM_FORM_SLDM = 0, BEM_FORM_EAEFIE = 1 };

typedef struct {
  double freq_hz;
  bem_c64 eps_bg;               /* background (homogeneous layer l) relative permittivity */
  double mu_bg;
  const bem_material* obj;      /* n_obj materials, host */
  int64_t n_obj;
  int precision;                /* BEM_FP64, BEM_FP32 (float32 blocks only, see above), or
                                   BEM_MIXED: float32 copies of the dense blocks;
                                   each refinement sweep runs float64 products until GMRES's
                                   residual estimate is sqrt(tol), float32 products after (first
                                   restart cycle only), float64 residual refinement; float64
                                   products throughout when a float32 probe deviates > 1e-4 */
  int inner_mode;               /* BEM_INNER_* */
  int precond;                  /* 1: block preconditioner of eq. pcext for the final system
                                   (and its equivalent-configuration counterpart for the nested
                                   GMRES), built at assembly; 0: none */
  int formulation;              /* BEM_FORM_* (0: eq. finalsystem) */
  int no_reuse;                 /* 0: an object that is a translated copy of an earlier one
                                   (same triangles in the same order moved by one translation,
                                   same edge table) shares that object's object-local blocks
                                   and their inverses (Sec. II-F, repeated objects): K~_l and
                                   the equivalent-configuration inverse for any material, and
                                   L^A, L^phi, K~ and the preconditioner's charge Schur inverse
                                   when the materials are equal too; 1: every object is filled
                                   and inverted separately */
} bem_problem;

/* Fill every dense block on the device: L^A, L^phi and K~ at the object
 * wavenumbers (interior, eq. AEFIEintdis) and at the background wavenumber
 * (eqs. AEFIEeqvdis and AEFIEextdis), the sparse D, F, B and I_x, and, with
 * BEM_MIXED, their float32 copies.  Runs synchronously on the context's
 * stream.  BEM_E_NOMEM if the blocks exceed the HBM budget; BEM_E_NUMERIC if a
 * dense inversion of the nested solve or of the preconditioner breaks down (see
 * bem_op_stats). */
int bem_assemble(bem_ctx* ctx, bem_mesh_h mesh, const bem_problem* prob, bem_op_h* out);

/* y = A x for `block` (see above), nrhs columns.  x, y: device pointers, column-
 * major, leading dimension = the block's row/column count, complex float64 (two
 * floats per entry when the operator was assembled with BEM_FP32);
 * stream: a hipStream_t or NULL for the context's stream (the call is
 * asynchronous on it, except BEM_BLOCK_FINAL, whose inner solve synchronises).
 * BEM_BLOCK_FINAL applies eq. finalsystem with the equivalent-configuration
 * solve (eq. AEFIEeqvdis) done by GMRES to the relative tolerance set by
 * bem_set_inner_tol (default 1e-12). */
int bem_apply(bem_ctx* ctx, bem_op_h op, int block, const void* x, void* y, int64_t nrhs, void* stream);
/* In-place inverse of a dense complex matrix on the device by the library's blocked
 * Gauss-Jordan elimination without pivoting: the routine that forms the direct nested-solve
 * inverses (M_eq^-1 of eq. AEFIEeqvdis, or its charge-eliminated S^-1) and the inverses of the
 * preconditioner's charge Schur complements (eq. pcext; Sec. III).  A: device pointer, n x n
 * row-major complex float64 (bem_c64 layout), leading dimension ld >= n elements; the caller
 * owns it and should equilibrate it (no scaling is done here).  stream: a hipStream_t or NULL
 * for the context's stream; the call waits for it.  The library allocates a workspace of about
 * 8 KiB per row for the call.  health (host, 2 doubles, may be NULL): the smallest pivot relative
 * to the largest entry of its 64 x 64 diagonal block, and the relative error
 * |A^-1 (A x) - x| / |x| of a fixed probe vector x.  BEM_E_NUMERIC when a pivot ratio is below
 * 1e-12, the probe error above 1e-6, or either is NaN: elimination without pivoting has broken
 * down and A holds no usable inverse.  BEM_E_INVALID for n < 0, ld < n or a null A. */
int bem_dense_invert(bem_ctx* ctx, void* A, int64_t n, int64_t ld, void* stream, double* health);

/* bem_dense_invert for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same elimination, checks, arguments
 * and status codes, but the workspace is a fixed device array of the library (one per GPU, about
 * 17 MB, held until the process ends), so the call allocates nothing.  n is limited to 2048 rows
 * (BEM_E_INVALID above).  Every call on one GPU uses that GPU's array: calls that overlap on one
 * GPU (from any context or thread) race and must not be made. */
int bem_dense_invert_noalloc(bem_ctx* ctx, void* A, int64_t n, int64_t ld, void* stream, double* health);

/* Copy a dense block (blocks 1..7) into a host buffer, row-major complex
 * float64, rows x cols as documented above (block-diagonal blocks include
 * their zero off-diagonal parts); a BEM_FP32 operator's float32 entries are
 * widened. */
int bem_block_export(bem_ctx* ctx, bem_op_h op, int block, bem_c64* host_dst);
int bem_set_inner_tol(bem_ctx* ctx, bem_op_h op, double tol);

/* Far field of solutions (Sec. II-C: outside the objects the scattered field is the one the
 * differential current J_delta = J - J_eq radiates in the background, J_eq being the current
 * of the equivalent configuration, eq. AEFIEeqvdis, for the same E):
 *   N(rhat) = int J_delta(r') exp(+j k_l rhat . r') dS'   (7-point rule on every triangle)
 * for ndir unit directions rhat (host, 3 doubles each) and nexc solutions H, E as bem_solve
 * returns them (host, column-major NE x nexc).  Outputs (host, either may be NULL): N, 3
 * complex per (solution, direction), laid out [exc][dir][xyz]; rcs, the bistatic radar
 * cross-section |k_l eta_l|^2 / (4 pi) |N_perp|^2 in m^2 per unit incident amplitude,
 * [exc][dir].  The equivalent solve runs in float64 (nested GMRES to the operator's inner
 * tolerance).  Not concurrently with bem_solve on the same operator.  BEM_E_INVALID for the
 * eAEFIE formulation (no equivalent configuration) or non-unit directions. */
int bem_far_field(bem_ctx* ctx, bem_op_h op, const bem_c64* H, const bem_c64* E, int64_t nexc,
                  const double* rhat, int64_t ndir, bem_c64* N, double* rcs);

enum { BEM_EXC_PLANE_WAVE = 0, BEM_EXC_DELTA_GAP = 1 };
typedef struct {
  int kind;
  double khat[3];               /* plane wave: unit propagation direction */
  bem_c64 pol[3];               /* plane wave: polarisation (orthogonal to khat) */
  bem_c64 amp;                  /* plane wave: E0 (V/m); delta gap: voltage (V) */
  const int32_t* gap_edges;     /* delta gap: 2*n_gap vertex pairs (host), gap across each edge */
  int64_t n_gap;
} bem_excitation;

/* Near field of solutions at exterior points (Sec. II-C, eqs. diffsources and diffsourcesdis;
 * the probe-line observable of Sec. IV-D): outside the objects the scattered field is the one
 * that the differential current J_delta = J - J_eq and charge rho_delta = rho - rho_eq radiate
 * in the background (k_l, eps_l, mu_l), J_eq and rho_eq being those of the equivalent
 * configuration (eq. AEFIEeqvdis, same E; solved in float64 to the operator's inner tolerance):
 *   E = -j omega mu A - grad Phi,  H = curl A,  A = int G J_delta dS',  Phi = (1/eps) int G rho_delta dS'
 * per triangle by the 7-point rule on the fill's source split; for a point within two longest
 * edges of a triangle's centroid the static parts of G and grad G in closed form and the
 * bounded remainders on at least 16 pieces.  Inputs (host): H, E (NE x nexc) and rho
 * (NT x nexc) as bem_solve returns them, column-major; npts points, 3 doubles each, which must
 * lie outside every object and off the surface (inside an object the sum is not that
 * object's field; on the surface it is singular).  exc: NULL for the scattered field only, or
 * the nexc plane waves of the solve to add the incident field (E0 pol e^{-j k_l khat . r},
 * H = khat x E / eta_l): the total field.  Outputs (host, either may be NULL): E_out, H_out,
 * 3 complex per (solution, point), laid out [exc][point][xyz], in V/m and A/m.  npts = 0
 * returns at once.  Not concurrently with bem_solve on the same operator.  BEM_E_INVALID for
 * the eAEFIE formulation, a delta-gap excitation with exc given, or a non-finite point. */
int bem_near_field(bem_ctx* ctx, bem_op_h op, const bem_c64* H, const bem_c64* E, const bem_c64* rho, int64_t nexc,
                   const bem_excitation* exc, const double* points, int64_t npts, bem_c64* E_out, bem_c64* H_out);

typedef struct {
  double tol;                   /* relative residual ||b - A x|| / ||b|| in float64 */
  int restart;                  /* GMRES restart length; <= 0: automatic, the longest cycle (100 to
                                   1000 steps) whose Krylov basis for the batch of excitations
                                   stays under 8 GB, lengthened (up to 1000 steps, the basis
                                   within a quarter of the free budget) for the later sweeps when
                                   a sweep runs out of steps */
  int maxit;                    /* total outer iteration limit */
  double inner_tol;             /* relative tolerance of the equivalent-configuration solve;
                                   <= 0 selects 0.1 * tol */
  int max_refine;               /* BEM_MIXED: maximum refinement sweeps */
  int out_device;               /* 1: H, E, rho are device pointers; 0: host */
} bem_solve_opts;

typedef struct {
  int outer_iters;              /* total outer GMRES iterations (all sweeps) */
  int inner_iters_max;          /* largest inner GMRES iteration count of one product */
  int refine_steps;             /* float64 residual evaluations (BEM_MIXED) */
  int n_products;               /* applications of the final system */
  double rel_residual;          /* final float64 relative residual (worst excitation) */
  double seconds;
  int graph_steps;              /* Arnoldi steps whose product was replayed from a captured HIP
                                   graph (small operators without a nested GMRES; BEM_GRAPH=0
                                   in the environment turns the capture off) */
  int cycle_growths;            /* times the automatic restart cycle was lengthened */
} bem_solve_info;

/* Solve eq. finalsystem for nexc excitations (right-hand side of eq.
 * AEFIEextdis: b_m = eta0^-1 int f_m . E_inc).  Outputs, column-major with nexc
 * columns: H (NE x nexc) coefficients of n x H on RWG functions, E (NE x nexc)
 * coefficients of n x E on BC functions, rho (NT x nexc) charge density
 * coefficients on area-normalised pulses (the full, un-reduced vector).  Any
 * output may be NULL.  On BEM_E_NOT_CONVERGED the best iterate is written. */
int bem_solve(bem_ctx* ctx, bem_op_h op, const bem_excitation* exc, int64_t nexc,
              const bem_solve_opts* opts, bem_c64* H, bem_c64* E, bem_c64* rho, bem_solve_info* info);

/* Asynchronous serving (continuous batching).  A request carries its own mesh,
 * problem, excitations and options; all arrays are copied at submit time except
 * the output buffers (host), which must stay valid until bem_poll returns
 * something other than BEM_PENDING.  Requests are admitted while their
 * estimated device footprint fits the HBM budget; admitted requests progress
 * together and share batched product launches.  A request that runs out of
 * device memory while others are solving is queued again at the head and rerun
 * alone (at most twice) before BEM_E_NOMEM is reported for it. */
typedef struct {
  const double* xyz; int64_t nv;
  const int32_t* tri; int64_t nt;
  const int32_t* obj;
  bem_problem prob;
  const bem_excitation* exc; int64_t nexc;
  bem_solve_opts opts;
  bem_c64* H; bem_c64* E; bem_c64* rho;   /* host outputs, as for bem_solve */
} bem_request;
int bem_submit(bem_ctx* ctx, const bem_request* req, bem_ticket* out);
/* BEM_PENDING while queued or running; otherwise the request's final status
 * (its outputs are then written) and info is filled.  The ticket is retired
 * when a final status is returned. */
int bem_poll(bem_ctx* ctx, bem_ticket ticket, bem_solve_info* info);
/* Block until no submitted request is pending. */
int bem_drain(bem_ctx* ctx);
/* Serving counters since the first bem_submit: grouped launches issued by the product
 * combiner, and the product requests they carried (> launches when requests shared a launch).
 * Both outputs may be NULL. */
int bem_serve_stats(bem_ctx* ctx, int64_t* combined_launches, int64_t* combined_products);

/* Statistics of an assembled operator: device time of the whole fill (all wavenumbers, near
 * corrections and gathers), bytes of the float64 dense blocks written, Green's-function and
 * gradient evaluations of the quadrature, device bytes held by the operator, the number of
 * objects whose interior blocks (L^A, L^phi, K~ at the object wavenumber) were filled (the
 * others share a translated copy's, see bem_problem.no_reuse), and the worst health of the
 * operator's dense inversions (nested-solve inverses and the preconditioner's charge Schur
 * complements; blocked Gauss-Jordan without pivoting): the smallest pivot relative to the
 * largest entry of its 64 x 64 diagonal block (+inf when nothing was inverted) and the largest
 * relative error |A^-1 (A x) - x| / |x| of a fixed probe vector x.  bem_assemble fails with
 * BEM_E_NUMERIC when a pivot ratio is below 1e-12 or a probe error above 1e-6. */
typedef struct {
  double fill_seconds;
  double fill_bytes;
  double kernel_evals;
  double device_bytes;
  double interiors_filled;
  double inverse_min_pivot_ratio;
  double inverse_probe_error;
} bem_op_stats;
int bem_op_stats_get(bem_ctx* ctx, bem_op_h op, bem_op_stats* out);

/* Opt-in kernel timing (all contexts of the process).  When enabled, HIP events are recorded
 * on the launch stream around every fill, gather and dense-product launch made by a caller's
 * thread (the serving loop's requests are not timed: they overlap on the device), together
 * with the launch's algorithmic bytes and work.  Enabling clears the counters.  Classes: 0 float64
 * products, 1 float32 products, 2 L fill, 3 K~ fill, 4 near corrections, 5 gathers, 6 float32
 * matrix-core products (several excitations), 7 Gauss-Jordan panel updates of the dense inversions,
 * 8 float64 matrix-core products.  bem_profile_read waits for the recorded events. */
int bem_profile_enable(int on);
int bem_profile_read(int kernel_class, int64_t* launches, double* ms, double* bytes, double* work);

/* Free a mesh or operator handle and its device memory. */
int bem_release(bem_ctx* ctx, uint64_t handle);
/* Device bytes currently held by the context. */
int bem_memory_in_use(bem_ctx* ctx, size_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
