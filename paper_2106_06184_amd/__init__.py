"""Python binding of libbem (MI355X dense single-layer dual-mesh BEM).

Argument marshalling only: every computation runs in libbem.so (HIP kernels for gfx950 and
the C++ host code behind the C ABI of include/bem.h).  The function names are those of the
C ABI.  Device vectors are passed as raw pointers (e.g. torch tensors' data_ptr()).

Loading fails loudly when the library has not been built (python -m paper_2106_06184_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

# BEM_LIB selects another build of the library (e.g. one made with other compiler flags).
_LIB_PATH = Path(os.environ["BEM_LIB"]) if os.environ.get("BEM_LIB") else Path(__file__).resolve().parent / "libbem.so"

BEM_OK, BEM_PENDING = 0, 1
BEM_E_INVALID, BEM_E_MESH, BEM_E_NOMEM, BEM_E_NOT_CONVERGED, BEM_E_DEVICE, BEM_E_NUMERIC = -1, -2, -3, -4, -5, -6
BEM_FP64, BEM_FP32, BEM_MIXED = 0, 1, 2
(BEM_BLOCK_FINAL, BEM_BLOCK_LA_INT, BEM_BLOCK_LPHI_INT, BEM_BLOCK_K_INT, BEM_BLOCK_LA_BG,
 BEM_BLOCK_LPHI_BG, BEM_BLOCK_K_BG, BEM_BLOCK_IX, BEM_BLOCK_MEQ, BEM_BLOCK_MEQ_INV, BEM_BLOCK_K_M) = range(11)
BEM_EXC_PLANE_WAVE, BEM_EXC_DELTA_GAP = 0, 1

SYMBOLS = ["bem_create", "bem_destroy", "bem_last_error", "bem_mesh_load", "bem_mesh_info", "bem_edge_table",
           "bem_near_pairs", "bem_mesh_copies", "bem_far_field", "bem_near_field", "bem_assemble", "bem_apply", "bem_dense_invert",
           "bem_dense_invert_noalloc",
           "bem_block_export", "bem_set_inner_tol", "bem_solve",
           "bem_submit", "bem_poll", "bem_drain", "bem_release", "bem_memory_in_use", "bem_op_stats_get",
           "bem_profile_enable", "bem_profile_read", "bem_serve_stats"]
(KC_GEMV_F64, KC_GEMV_F32, KC_FILL_L, KC_FILL_K, KC_FILL_NEAR, KC_GATHER, KC_GEMM_F32, KC_DENSE_INV,
 KC_GEMM_F64) = range(9)
KC_NAMES = ["gemv_f64", "gemv_f32", "fill_L", "fill_K", "fill_near", "gather", "gemm_f32_mfma", "dense_inv_update",
            "gemm_f64_mfma"]


class bem_op_stats(C.Structure):
    _fields_ = [("fill_seconds", C.c_double), ("fill_bytes", C.c_double), ("kernel_evals", C.c_double),
                ("device_bytes", C.c_double), ("interiors_filled", C.c_double),
                ("inverse_min_pivot_ratio", C.c_double), ("inverse_probe_error", C.c_double)]


class c64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class bem_material(C.Structure):
    _fields_ = [("eps_r", c64), ("mu_r", C.c_double), ("sigma", C.c_double)]


BEM_INNER_AUTO, BEM_INNER_GMRES, BEM_INNER_DIRECT, BEM_INNER_SCHUR = 0, 1, 2, 3
BEM_FORM_SLDM, BEM_FORM_EAEFIE = 0, 1


class bem_problem(C.Structure):
    _fields_ = [("freq_hz", C.c_double), ("eps_bg", c64), ("mu_bg", C.c_double),
                ("obj", C.POINTER(bem_material)), ("n_obj", C.c_int64), ("precision", C.c_int),
                ("inner_mode", C.c_int), ("precond", C.c_int), ("formulation", C.c_int),
                ("no_reuse", C.c_int)]


class bem_excitation(C.Structure):
    _fields_ = [("kind", C.c_int), ("khat", C.c_double * 3), ("pol", c64 * 3), ("amp", c64),
                ("gap_edges", C.POINTER(C.c_int32)), ("n_gap", C.c_int64)]


class bem_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("inner_tol", C.c_double),
                ("max_refine", C.c_int), ("out_device", C.c_int)]


class bem_solve_info(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters_max", C.c_int), ("refine_steps", C.c_int),
                ("n_products", C.c_int), ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("graph_steps", C.c_int), ("cycle_growths", C.c_int)]


class bem_request(C.Structure):
    _fields_ = [("xyz", C.POINTER(C.c_double)), ("nv", C.c_int64), ("tri", C.POINTER(C.c_int32)),
                ("nt", C.c_int64), ("obj", C.POINTER(C.c_int32)), ("prob", bem_problem),
                ("exc", C.POINTER(bem_excitation)), ("nexc", C.c_int64), ("opts", bem_solve_opts),
                ("H", C.POINTER(c64)), ("E", C.POINTER(c64)), ("rho", C.POINTER(c64))]


_lib = None


def lib() -> C.CDLL:
    """The loaded libbem.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_2106_06184_amd.build`")
        L = C.CDLL(str(_LIB_PATH))
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "bem_create": (C.c_int, [C.c_int, C.c_size_t, C.POINTER(P)]),
            "bem_destroy": (None, [P]),
            "bem_last_error": (C.c_char_p, [P]),
            "bem_mesh_load": (C.c_int, [P, C.POINTER(D), I64, C.POINTER(I32), I64, C.POINTER(I32), C.POINTER(C.c_uint64)]),
            "bem_mesh_info": (C.c_int, [P, C.c_uint64, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
            "bem_edge_table": (C.c_int, [P, C.c_uint64, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]),
            "bem_near_pairs": (C.c_int, [P, C.c_uint64, C.POINTER(I64), C.POINTER(I32)]),
            "bem_mesh_copies": (C.c_int, [P, C.c_uint64, C.POINTER(I32)]),
            "bem_far_field": (C.c_int, [P, C.c_uint64, C.POINTER(c64), C.POINTER(c64), C.c_int64,
                                        C.POINTER(C.c_double), C.c_int64, C.POINTER(c64), C.POINTER(C.c_double)]),
            "bem_near_field": (C.c_int, [P, C.c_uint64, C.POINTER(c64), C.POINTER(c64), C.POINTER(c64), C.c_int64,
                                         C.POINTER(bem_excitation), C.POINTER(C.c_double), C.c_int64,
                                         C.POINTER(c64), C.POINTER(c64)]),
            "bem_assemble": (C.c_int, [P, C.c_uint64, C.POINTER(bem_problem), C.POINTER(C.c_uint64)]),
            "bem_apply": (C.c_int, [P, C.c_uint64, C.c_int, P, P, I64, P]),
            "bem_dense_invert": (C.c_int, [P, P, I64, I64, P, C.POINTER(D)]),
            "bem_dense_invert_noalloc": (C.c_int, [P, P, I64, I64, P, C.POINTER(D)]),
            "bem_block_export": (C.c_int, [P, C.c_uint64, C.c_int, C.POINTER(c64)]),
            "bem_set_inner_tol": (C.c_int, [P, C.c_uint64, D]),
            "bem_solve": (C.c_int, [P, C.c_uint64, C.POINTER(bem_excitation), I64, C.POINTER(bem_solve_opts),
                                    C.POINTER(c64), C.POINTER(c64), C.POINTER(c64), C.POINTER(bem_solve_info)]),
            "bem_submit": (C.c_int, [P, C.POINTER(bem_request), C.POINTER(C.c_uint64)]),
            "bem_serve_stats": (C.c_int, [P, C.POINTER(I64), C.POINTER(I64)]),
            "bem_poll": (C.c_int, [P, C.c_uint64, C.POINTER(bem_solve_info)]),
            "bem_drain": (C.c_int, [P]),
            "bem_release": (C.c_int, [P, C.c_uint64]),
            "bem_memory_in_use": (C.c_int, [P, C.POINTER(C.c_size_t)]),
            "bem_op_stats_get": (C.c_int, [P, C.c_uint64, C.POINTER(bem_op_stats)]),
            "bem_profile_enable": (C.c_int, [C.c_int]),
            "bem_profile_read": (C.c_int, [C.c_int, C.POINTER(I64), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class BemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libbem status {code}: {msg}")
        self.code = code


def _check(ctx, rc: int, allow=(BEM_OK,)) -> int:
    if rc not in allow:
        raise BemError(rc, lib().bem_last_error(ctx).decode())
    return rc


# ------------------------------------------------------------- marshalling helpers

def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _cptr(a):
    return a.ctypes.data_as(C.POINTER(c64)) if a is not None else None


def bem_create(device: int = 0, budget: int = 0):
    p = C.c_void_p()
    _check(None, lib().bem_create(device, budget, C.byref(p)))
    return p


def bem_destroy(ctx) -> None:
    lib().bem_destroy(ctx)


def bem_last_error(ctx) -> str:
    return lib().bem_last_error(ctx).decode()


def bem_mesh_load(ctx, xyz, tri, obj=None) -> int:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    o = np.ascontiguousarray(obj, dtype=np.int32) if obj is not None else None
    h = C.c_uint64()
    _check(ctx, lib().bem_mesh_load(ctx, _dptr(xyz), len(xyz), _iptr(tri), len(tri),
                                    _iptr(o) if o is not None else None, C.byref(h)))
    return h.value


def bem_mesh_info(ctx, mesh: int) -> dict:
    v = [C.c_int64() for _ in range(4)]
    _check(ctx, lib().bem_mesh_info(ctx, mesh, *[C.byref(x) for x in v]))
    return dict(n_tri=v[0].value, n_edge=v[1].value, n_obj=v[2].value, n_unknowns=v[3].value)


def bem_edge_table(ctx, mesh: int):
    ne = bem_mesh_info(ctx, mesh)["n_edge"]
    out = [np.zeros(ne, np.int32) for _ in range(4)]
    _check(ctx, lib().bem_edge_table(ctx, mesh, *[_iptr(a) for a in out]))
    return out  # va, vb, tplus, tminus


def bem_far_field(ctx, op: int, H, E, rhat):
    """Far-field vector N[exc, dir, xyz] and bistatic RCS[exc, dir] (m^2 per unit amplitude) of
    solutions H, E (NE x nexc) in the unit directions rhat (ndir x 3)."""
    H = np.ascontiguousarray(np.asarray(H, np.complex128).reshape(H.shape[0], -1).T)
    E = np.ascontiguousarray(np.asarray(E, np.complex128).reshape(E.shape[0], -1).T)
    rhat = np.ascontiguousarray(np.atleast_2d(np.asarray(rhat, np.float64)))
    nexc, ndir = H.shape[0], rhat.shape[0]
    N = np.zeros((nexc, ndir, 3), np.complex128)
    rcs = np.zeros((nexc, ndir), np.float64)
    cp = lambda a: a.ctypes.data_as(C.POINTER(c64))
    _check(ctx, lib().bem_far_field(ctx, op, cp(H), cp(E), nexc, rhat.ctypes.data_as(C.POINTER(C.c_double)), ndir,
                                    cp(N), rcs.ctypes.data_as(C.POINTER(C.c_double))))
    return N, rcs


def bem_near_field(ctx, op: int, H, E, rho, points, exc=None):
    """Near field E[exc, point, xyz], H[exc, point, xyz] (V/m, A/m) of solutions H, E (NE x nexc)
    and rho (NT x nexc) at exterior points (npts x 3): the scattered field, or the total field
    when `exc` holds the solve's plane waves."""
    H = np.ascontiguousarray(np.asarray(H, np.complex128).reshape(H.shape[0], -1).T)
    E = np.ascontiguousarray(np.asarray(E, np.complex128).reshape(E.shape[0], -1).T)
    rho = np.ascontiguousarray(np.asarray(rho, np.complex128).reshape(rho.shape[0], -1).T)
    pts = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, 3))
    nexc, npts = H.shape[0], pts.shape[0]
    Eo = np.zeros((nexc, npts, 3), np.complex128)
    Ho = np.zeros((nexc, npts, 3), np.complex128)
    cp = lambda a: a.ctypes.data_as(C.POINTER(c64))
    _check(ctx, lib().bem_near_field(ctx, op, cp(H), cp(E), cp(rho), nexc, exc,
                                     pts.ctypes.data_as(C.POINTER(C.c_double)), npts, cp(Eo), cp(Ho)))
    return Eo, Ho


def bem_mesh_copies(ctx, mesh: int) -> np.ndarray:
    """proto[o]: the first object of which object o is a translated copy, or o."""
    out = np.zeros(bem_mesh_info(ctx, mesh)["n_obj"], np.int32)
    _check(ctx, lib().bem_mesh_copies(ctx, mesh, _iptr(out)))
    return out


def bem_near_pairs(ctx, mesh: int):
    nt = bem_mesh_info(ctx, mesh)["n_tri"]
    ptr = np.zeros(nt + 1, np.int64)
    _check(ctx, lib().bem_near_pairs(ctx, mesh, ptr.ctypes.data_as(C.POINTER(C.c_int64)), None))
    idx = np.zeros(int(ptr[-1]), np.int32)
    _check(ctx, lib().bem_near_pairs(ctx, mesh, ptr.ctypes.data_as(C.POINTER(C.c_int64)), _iptr(idx)))
    return ptr, idx


def make_problem(freq_hz, eps_r, mu_r, sigma, eps_bg=1.0, mu_bg=1.0, precision=BEM_FP64,
                 inner_mode=BEM_INNER_AUTO, precond=1, formulation=BEM_FORM_SLDM, reuse=True):
    mats = (bem_material * len(eps_r))()
    for i, (e, m, s) in enumerate(zip(eps_r, mu_r, sigma)):
        mats[i] = bem_material(c64(complex(e).real, complex(e).imag), float(m), float(s))
    p = bem_problem(float(freq_hz), c64(complex(eps_bg).real, complex(eps_bg).imag), float(mu_bg),
                    C.cast(mats, C.POINTER(bem_material)), len(eps_r), int(precision), int(inner_mode), int(precond),
                    int(formulation), 0 if reuse else 1)
    p._keep = mats
    return p


def bem_assemble(ctx, mesh: int, prob: bem_problem) -> int:
    h = C.c_uint64()
    _check(ctx, lib().bem_assemble(ctx, mesh, C.byref(prob), C.byref(h)))
    return h.value


def bem_apply(ctx, op: int, block: int, x_ptr: int, y_ptr: int, nrhs: int = 1, stream: int | None = None) -> None:
    _check(ctx, lib().bem_apply(ctx, op, block, C.c_void_p(x_ptr), C.c_void_p(y_ptr), nrhs,
                                C.c_void_p(stream) if stream else None))


def bem_dense_invert(ctx, a_ptr: int, n: int, ld: int, stream=None):
    """In-place device inverse of the n x n complex matrix at a_ptr (row-major, leading dimension
    ld).  Returns (status, (min_pivot_ratio, probe_error)); raises on errors other than
    BEM_E_NUMERIC (the breakdown status, returned so that callers can inspect the health)."""
    h = np.zeros(2, np.float64)
    rc = lib().bem_dense_invert(ctx, C.c_void_p(a_ptr), int(n), int(ld), C.c_void_p(stream) if stream else None,
                                h.ctypes.data_as(C.POINTER(C.c_double)))
    _check(ctx, rc, allow=(BEM_OK, BEM_E_NUMERIC))
    return rc, (float(h[0]), float(h[1]))


def bem_dense_invert_noalloc(ctx, a_ptr: int, n: int, ld: int, stream=None):
    """bem_dense_invert on the library's fixed workspace (allocates nothing; n <= 2048)."""
    h = np.zeros(2, np.float64)
    rc = lib().bem_dense_invert_noalloc(ctx, C.c_void_p(a_ptr), int(n), int(ld),
                                        C.c_void_p(stream) if stream else None, h.ctypes.data_as(C.POINTER(C.c_double)))
    _check(ctx, rc, allow=(BEM_OK, BEM_E_NUMERIC))
    return rc, (float(h[0]), float(h[1]))


def bem_block_export(ctx, op: int, block: int, rows: int, cols: int) -> np.ndarray:
    out = np.zeros((rows, cols), np.complex128)
    _check(ctx, lib().bem_block_export(ctx, op, block, _cptr(out)))
    return out


def bem_set_inner_tol(ctx, op: int, tol: float) -> None:
    _check(ctx, lib().bem_set_inner_tol(ctx, op, float(tol)))


def plane_waves(khat, pol, amp=1.0):
    khat = np.atleast_2d(np.asarray(khat, np.float64))
    pol = np.atleast_2d(np.asarray(pol, np.complex128))
    arr = (bem_excitation * len(khat))()
    for i in range(len(khat)):
        e = arr[i]
        e.kind = BEM_EXC_PLANE_WAVE
        for k in range(3):
            e.khat[k] = khat[i, k]
            e.pol[k] = c64(pol[i, k].real, pol[i, k].imag)
        e.amp = c64(complex(amp).real, complex(amp).imag)
    return arr


def delta_gaps(ports, volts=1.0):
    """Voltage-gap excitations: ports is a list of (n_gap, 2) arrays of vertex pairs (a, b),
    one array per excitation; the field across each listed edge drives the RWG of the directed
    pair with `volts` (complex)."""
    arr = (bem_excitation * len(ports))()
    keep = []
    for i, pairs in enumerate(ports):
        pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
        keep.append(pairs)
        e = arr[i]
        e.kind = BEM_EXC_DELTA_GAP
        e.amp = c64(complex(volts).real, complex(volts).imag)
        e.gap_edges = _iptr(pairs)
        e.n_gap = len(pairs)
    arr._keep = keep
    return arr


def solve_opts(tol=1e-8, restart=50, maxit=2000, inner_tol=0.0, max_refine=0, out_device=0):
    return bem_solve_opts(tol, restart, maxit, inner_tol, max_refine, out_device)


def bem_solve(ctx, op: int, exc, opts: bem_solve_opts, n_edge: int, n_tri: int):
    """Returns (status, H[ne, nexc], E[ne, nexc], rho[nt, nexc], info) with host outputs."""
    n = len(exc)
    H = np.zeros((n, n_edge), np.complex128)
    E = np.zeros((n, n_edge), np.complex128)
    rho = np.zeros((n, n_tri), np.complex128)
    info = bem_solve_info()
    rc = lib().bem_solve(ctx, op, exc, n, C.byref(opts), _cptr(H), _cptr(E), _cptr(rho), C.byref(info))
    _check(ctx, rc, allow=(BEM_OK, BEM_E_NOT_CONVERGED))
    return rc, H.T, E.T, rho.T, info


class Request:
    """A serving request with its own copies of the inputs and host output arrays (H, E: n_edge x
    nexc; rho: n_tri x nexc, read after bem_poll returns a final status)."""

    def __init__(self, xyz, tri, obj, prob: bem_problem, exc, opts: bem_solve_opts):
        self.xyz = np.ascontiguousarray(xyz, np.float64)
        self.tri = np.ascontiguousarray(tri, np.int32)
        self.obj = None if obj is None else np.ascontiguousarray(obj, np.int32)
        self.prob, self.exc, self.opts = prob, exc, opts
        nt = len(self.tri)
        ne = 3 * nt // 2
        n = len(exc)
        self._H = np.zeros((n, ne), np.complex128)
        self._E = np.zeros((n, ne), np.complex128)
        self._rho = np.zeros((n, nt), np.complex128)
        self.c = bem_request(self.xyz.ctypes.data_as(C.POINTER(C.c_double)), len(self.xyz),
                             _iptr(self.tri), nt, _iptr(self.obj) if self.obj is not None else None,
                             prob, C.cast(exc, C.POINTER(bem_excitation)), n, opts,
                             _cptr(self._H), _cptr(self._E), _cptr(self._rho))

    @property
    def H(self):
        return self._H.T

    @property
    def E(self):
        return self._E.T

    @property
    def rho(self):
        return self._rho.T


def bem_submit(ctx, req) -> int:
    if isinstance(req, Request):
        req = req.c
    t = C.c_uint64()
    _check(ctx, lib().bem_submit(ctx, C.byref(req), C.byref(t)))
    return t.value


def bem_poll(ctx, ticket: int):
    info = bem_solve_info()
    rc = lib().bem_poll(ctx, ticket, C.byref(info))
    if rc < 0 and rc != BEM_E_NOT_CONVERGED:
        raise BemError(rc, bem_last_error(ctx))
    return rc, info


def bem_drain(ctx) -> None:
    _check(ctx, lib().bem_drain(ctx))


def bem_serve_stats(ctx) -> tuple[int, int]:
    """(grouped launches of the serving combiner, product requests they carried)."""
    a, b = C.c_int64(), C.c_int64()
    _check(ctx, lib().bem_serve_stats(ctx, C.byref(a), C.byref(b)))
    return a.value, b.value


def bem_release(ctx, handle: int) -> None:
    _check(ctx, lib().bem_release(ctx, handle))


def bem_op_stats_get(ctx, op: int) -> dict:
    s = bem_op_stats()
    _check(ctx, lib().bem_op_stats_get(ctx, op, C.byref(s)))
    return {f: getattr(s, f) for f, _ in bem_op_stats._fields_}


def bem_profile_enable(on: bool) -> None:
    _check(None, lib().bem_profile_enable(1 if on else 0))


def bem_profile_read(kernel_class: int) -> dict:
    n, ms, by, wk = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
    _check(None, lib().bem_profile_read(kernel_class, C.byref(n), C.byref(ms), C.byref(by), C.byref(wk)))
    return dict(launches=n.value, ms=ms.value, bytes=by.value, work=wk.value)


def bem_memory_in_use(ctx) -> int:
    v = C.c_size_t()
    _check(ctx, lib().bem_memory_in_use(ctx, C.byref(v)))
    return v.value
