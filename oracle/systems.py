"""Discrete systems of the single-layer dual-mesh formulation and their dense solves (oracle).

Unknowns (Sec. II-B..E): a = jk0 H, e = eta0^-1 E, q = c0 rho' (reduced charges),
a_eq = jk0 H_eq, q_eq = c0 rho'_eq.  L^A_m = mu_l L^A_l and L^phi_m = eps_l^-1 L^phi_l
for a homogeneous background (the layered Green's function is not used).

augmented system (plain definition; eqs. AEFIEintdis, AEFIEeqvdis, AEFIEextdis
with eq. diffsourcesdis substituted), rows
  (I)  mu_r L^A a - eps_c^-1 D^T L^phi B q - (K~ + I_x/2) e                 = 0
  (I2) F D a - k0^2 q                                                    = 0
  (Q)  mu_l L^A_l a_eq - eps_l^-1 D^T L^phi_l B q_eq - (K~_l + I_x/2) e     = 0
  (Q2) F D a_eq - k0^2 q_eq                                              = 0
  (X)  L^A_m (a - a_eq) - D^T L^phi_m B (q - q_eq) + I_x e                = b
The continuity row of eq. AEFIEextdis is (I2) - (Q2) and is not repeated.
For several disjoint objects every block of (I), (I2), (Q), (Q2) is block-
diagonal over objects (eq. Aobj) with each object's material; (X) couples them.

final system (eq. finalsystem) with explicit Y = M_eq^-1 [K_l; 0] (eq. Yeqdef),
unknowns [a; e; -q]:
  [ L^A_m   C1   D^T L^phi_m B       ]
  [ mu_r L^A   -K   eps_c^-1 D^T L^phi B ]
  [ F D     C2   k0^2 I            ]
  C1 = I_x - (L^A_m Y11 - D^T L^phi_m B Y21),  C2 = -(F D Y11 - k0^2 Y21)
Readings: the middle block is -K (eliminating row (I) with x3 = -q gives -K;
the printed +K does not follow from eq. AEFIEintdis), and C1 uses L^phi_m as in
eq. AEFIEextdis (the printed L^phi_l differs from it by eps_l).

eAEFIE counterpart (Sec. II-F): the same matrix with C1 and C2 replaced by the external
double-layer operator of the background medium over every object pair, K~_m, and zero:
  C1 = I_x/2 - K~_m,  C2 = 0   (same unknowns [a; e; -q], no equivalent problem)
Reading: the comparison prints C1 = K~_m - I_x/2.  For one object on a homogeneous background
the exact Y of eq. Yeqdef gives the proposed C1 = I_x - K_l = I_x/2 - K~_l and C2 = 0 in the
sign convention of the unknowns above, i.e. the two formulations coincide; the printed sign
belongs to the opposite sign of the E column that also prints +K in the middle block.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import constants as C
from . import mesh as M
from . import operators as O
from . import quadrature as Q


@dataclass
class Problem:
    freq_hz: float
    eps_r: list            # per object
    mu_r: list
    sigma: list
    eps_bg: complex = 1.0
    mu_bg: float = 1.0


@dataclass
class Operators:
    topo: M.Topology
    bary: M.Barycentric
    D: np.ndarray
    B: np.ndarray
    F: np.ndarray
    Ix: np.ndarray
    LA_int: np.ndarray      # block-diagonal, per-object interior wavenumber
    Lphi_int: np.ndarray
    K_int: np.ndarray
    LA_bg: np.ndarray       # full, background wavenumber
    Lphi_bg: np.ndarray
    K_bg: np.ndarray        # block-diagonal, background wavenumber
    K_m: np.ndarray         # full (every object pair), background wavenumber
    k0: float
    k_int: list
    k_bg: complex
    epsc: list
    mu_r: list
    eps_bg: complex
    mu_bg: float


def assemble(xyz, tri, obj, prob: Problem) -> Operators:
    topo = M.build_topology(xyz, tri, obj)
    bary = M.buffa_christiansen(topo)
    bcdata = O.bc_on_subtriangles(bary)
    near = O.near_pairs(topo)
    D = M.incidence_D(topo).toarray()
    B, F, _ = M.charge_maps(topo)
    B, F = B.toarray(), F.toarray()
    Ix = O.gram_Ix(topo, bary, bcdata)
    k0 = C.k0_of(prob.freq_hz)
    epsc = [C.eps_c(e, s, prob.freq_hz) for e, s in zip(prob.eps_r, prob.sigma)]
    k_int = [C.wavenumber(k0, ec, mu) for ec, mu in zip(epsc, prob.mu_r)]
    k_bg = C.wavenumber(k0, prob.eps_bg, prob.mu_bg)
    nt, ne = len(topo.tri), len(topo.edges)
    same_e = topo.edge_obj[:, None] == topo.edge_obj[None, :]
    same_t = topo.obj[:, None] == topo.obj[None, :]
    LA_int = np.zeros((ne, ne), complex)
    Lphi_int = np.zeros((nt, nt), complex)
    K_int = np.zeros((ne, ne), complex)
    cache = {}
    for o in range(topo.n_obj):
        k = k_int[o]
        if k not in cache:
            LA, Lp = O.fill_L(topo, k, near)
            K = O.fill_K(topo, bary, k, near, bcdata)
            cache[k] = (LA, Lp, K)
        LA, Lp, K = cache[k]
        me = (topo.edge_obj == o)[:, None] & same_e
        mt = (topo.obj == o)[:, None] & same_t
        LA_int[me] = LA[me]
        Lphi_int[mt] = Lp[mt]
        K_int[me] = K[me]
    if k_bg in cache:
        LA_bg, Lphi_bg, Kb = cache[k_bg]
    else:
        LA_bg, Lphi_bg = O.fill_L(topo, k_bg, near)
        Kb = O.fill_K(topo, bary, k_bg, near, bcdata)
    K_bg = np.where(same_e, Kb, 0.0)
    return Operators(topo, bary, D, B, F, Ix, LA_int, Lphi_int, K_int, LA_bg, Lphi_bg, K_bg, Kb,
                     k0, k_int, k_bg, epsc, list(prob.mu_r), complex(prob.eps_bg), float(prob.mu_bg))


def _per_edge(ops: Operators, vals):
    return np.asarray(vals)[ops.topo.edge_obj]


def _per_tri(ops: Operators, vals):
    return np.asarray(vals)[ops.topo.obj]


def rhs(ops: Operators, khat, pol, E0=1.0):
    return O.rhs_plane_wave(ops.topo, ops.k_bg, khat, pol, E0)


def augmented_matrix(ops: Operators):
    ne = len(ops.topo.edges)
    nq = ops.B.shape[1]
    D, B, F = ops.D, ops.B, ops.F
    mu_e = _per_edge(ops, ops.mu_r)[:, None]
    inv_eps_e = (1.0 / _per_edge(ops, ops.epsc))[:, None]
    same_e = ops.topo.edge_obj[:, None] == ops.topo.edge_obj[None, :]
    same_t = ops.topo.obj[:, None] == ops.topo.obj[None, :]
    LA_l_bd = np.where(same_e, ops.LA_bg, 0.0)
    Lphi_l_bd = np.where(same_t, ops.Lphi_bg, 0.0)
    Kint = ops.K_int + 0.5 * ops.Ix
    Kbg = ops.K_bg + 0.5 * ops.Ix
    k02 = ops.k0 ** 2
    Iq = np.eye(nq)
    Z_ee = np.zeros((ne, ne))
    Z_eq = np.zeros((ne, nq))
    Z_qe = np.zeros((nq, ne))
    Z_qq = np.zeros((nq, nq))
    mu_l, eps_l = ops.mu_bg, ops.eps_bg
    rows = [
        [mu_e * ops.LA_int, -Kint, -inv_eps_e * (D.T @ ops.Lphi_int @ B), Z_ee, Z_eq],
        [F @ D, Z_qe, -k02 * Iq, Z_qe, Z_qq],
        [Z_ee, -Kbg, Z_eq, mu_l * LA_l_bd, -(1 / eps_l) * (D.T @ Lphi_l_bd @ B)],
        [Z_qe, Z_qe, Z_qq, F @ D, -k02 * Iq],
        [mu_l * ops.LA_bg, ops.Ix, -(1 / eps_l) * (D.T @ ops.Lphi_bg @ B),
         -mu_l * ops.LA_bg, (1 / eps_l) * (D.T @ ops.Lphi_bg @ B)],
    ]
    return np.block(rows)


@dataclass
class Solution:
    a: np.ndarray       # jk0 H
    e: np.ndarray       # eta0^-1 E
    q: np.ndarray       # c0 rho' (reduced)
    a_eq: np.ndarray
    q_eq: np.ndarray

    def H(self, k0):
        return self.a / (1j * k0)

    def E(self):
        return self.e * C.ETA0

    def rho(self, B):
        return (B @ self.q) / C.C0


def solve_augmented(ops: Operators, b):
    ne = len(ops.topo.edges)
    nq = ops.B.shape[1]
    A = augmented_matrix(ops)
    b = np.atleast_2d(np.asarray(b).T).T if np.ndim(b) == 1 else np.asarray(b)
    rhs_full = np.zeros((A.shape[0], b.shape[1]), complex)
    rhs_full[3 * ne + 2 * nq - ne:] = 0.0
    rhs_full[ne + nq + ne + nq:] = b
    x = sla.lu_solve(sla.lu_factor(A), rhs_full)
    sl = np.cumsum([0, ne, ne, nq, ne, nq])
    parts = [x[sl[i]:sl[i + 1]] for i in range(5)]
    sols = [Solution(*(p[:, c] for p in parts)) for c in range(b.shape[1])]
    return sols if len(sols) > 1 else sols[0]


def equivalent_matrix_object(ops: Operators, o: int):
    """M_eq of eq. AEFIEeqvdis for object o, with its edge / kept-charge index sets."""
    e_idx = np.nonzero(ops.topo.edge_obj == o)[0]
    t_idx = np.nonzero(ops.topo.obj == o)[0]
    q_idx = np.nonzero(np.abs(ops.B[t_idx]).sum(axis=0) > 0)[0]
    D = ops.D[np.ix_(t_idx, e_idx)]
    B = ops.B[np.ix_(t_idx, q_idx)]
    F = ops.F[np.ix_(q_idx, t_idx)]
    LA = ops.LA_bg[np.ix_(e_idx, e_idx)]
    Lp = ops.Lphi_bg[np.ix_(t_idx, t_idx)]
    nq = len(q_idx)
    Meq = np.block([[ops.mu_bg * LA, -(1 / ops.eps_bg) * (D.T @ Lp @ B)],
                    [F @ D, -ops.k0 ** 2 * np.eye(nq)]])
    return Meq, e_idx, q_idx


def admittance_Y(ops: Operators):
    """Y11 (NE x NE) and Y21 (NQ x NE) of eq. Yeqdef, block-diagonal over objects."""
    ne = len(ops.topo.edges)
    nq = ops.B.shape[1]
    Kl = ops.K_bg + 0.5 * ops.Ix
    Y11 = np.zeros((ne, ne), complex)
    Y21 = np.zeros((nq, ne), complex)
    for o in range(ops.topo.n_obj):
        Meq, e_idx, q_idx = equivalent_matrix_object(ops, o)
        rhs_ = np.zeros((Meq.shape[0], len(e_idx)), complex)
        rhs_[:len(e_idx)] = Kl[np.ix_(e_idx, e_idx)]
        Y = sla.lu_solve(sla.lu_factor(Meq), rhs_)
        Y11[np.ix_(e_idx, e_idx)] = Y[:len(e_idx)]
        Y21[np.ix_(q_idx, e_idx)] = Y[len(e_idx):]
    return Y11, Y21


def final_matrix(ops: Operators, Y=None):
    """The matrix of eq. finalsystem (readings in the module docstring)."""
    D, B, F = ops.D, ops.B, ops.F
    nq = B.shape[1]
    Y11, Y21 = Y if Y is not None else admittance_Y(ops)
    LAm = ops.mu_bg * ops.LA_bg
    Lpm = (1 / ops.eps_bg) * ops.Lphi_bg
    C1 = ops.Ix - (LAm @ Y11 - D.T @ Lpm @ B @ Y21)
    C2 = -(F @ D @ Y11 - ops.k0 ** 2 * Y21)
    mu_e = _per_edge(ops, ops.mu_r)[:, None]
    inv_eps_e = (1.0 / _per_edge(ops, ops.epsc))[:, None]
    Kfull = ops.K_int + 0.5 * ops.Ix
    return np.block([
        [LAm, C1, D.T @ Lpm @ B],
        [mu_e * ops.LA_int, -Kfull, inv_eps_e * (D.T @ ops.Lphi_int @ B)],
        [F @ D, C2, ops.k0 ** 2 * np.eye(nq)],
    ])


def solve_final(ops: Operators, b, Y=None):
    """Solve eq. finalsystem by LU; a_eq, q_eq follow from Y (eq. invAEFIEeqvdis)."""
    ne = len(ops.topo.edges)
    nq = ops.B.shape[1]
    Y11, Y21 = Y if Y is not None else admittance_Y(ops)
    A = final_matrix(ops, (Y11, Y21))
    rhs_full = np.zeros(A.shape[0], complex)
    rhs_full[:ne] = b
    x = sla.lu_solve(sla.lu_factor(A), rhs_full)
    a, e, x3 = x[:ne], x[ne:2 * ne], x[2 * ne:]
    return Solution(a, e, -x3, Y11 @ e, Y21 @ e)


def final_matrix_eaefie(ops: Operators):
    """The eAEFIE counterpart of eq. finalsystem (Sec. II-F; reading in the module docstring):
    C1 = I_x/2 - K~_m with K~_m over every object pair at the background wavenumber, C2 = 0."""
    D, B, F = ops.D, ops.B, ops.F
    nq = B.shape[1]
    ne = len(ops.topo.edges)
    LAm = ops.mu_bg * ops.LA_bg
    Lpm = (1 / ops.eps_bg) * ops.Lphi_bg
    mu_e = _per_edge(ops, ops.mu_r)[:, None]
    inv_eps_e = (1.0 / _per_edge(ops, ops.epsc))[:, None]
    Kfull = ops.K_int + 0.5 * ops.Ix
    return np.block([
        [LAm, 0.5 * ops.Ix - ops.K_m, D.T @ Lpm @ B],
        [mu_e * ops.LA_int, -Kfull, inv_eps_e * (D.T @ ops.Lphi_int @ B)],
        [F @ D, np.zeros((nq, ne)), ops.k0 ** 2 * np.eye(nq)],
    ])


def solve_final_eaefie(ops: Operators, b):
    """Solve the eAEFIE system by LU; returns (a, e, q) of the physical unknowns."""
    ne = len(ops.topo.edges)
    A = final_matrix_eaefie(ops)
    b = np.asarray(b)
    r = np.zeros((A.shape[0],) + b.shape[1:], complex)
    r[:ne] = b
    x = sla.lu_solve(sla.lu_factor(A), r)
    return x[:ne], x[ne:2 * ne], -x[2 * ne:]


def solve_reduced_single(ops: Operators, b):
    """Single object only: (X) + (Q) eliminates a_eq, q_eq exactly, leaving
    [mu_l L^A_l, -(K~_l - I_x/2), -eps_l^-1 D^T L^phi_l B] in row 1 plus (I), (I2)."""
    assert ops.topo.n_obj == 1
    ne = len(ops.topo.edges)
    nq = ops.B.shape[1]
    D, B, F = ops.D, ops.B, ops.F
    mu_r, epsc = ops.mu_r[0], ops.epsc[0]
    A = np.block([
        [ops.mu_bg * ops.LA_bg, -(ops.K_bg - 0.5 * ops.Ix), -(1 / ops.eps_bg) * (D.T @ ops.Lphi_bg @ B)],
        [mu_r * ops.LA_int, -(ops.K_int + 0.5 * ops.Ix), -(1 / epsc) * (D.T @ ops.Lphi_int @ B)],
        [F @ D, np.zeros((nq, ne)), -ops.k0 ** 2 * np.eye(nq)],
    ])
    r = np.zeros(A.shape[0], complex)
    r[:ne] = b
    x = sla.lu_solve(sla.lu_factor(A), r)
    return x[:ne], x[ne:2 * ne], x[2 * ne:]


# ---------------------------------------------------------------- far field

def far_field_N(ops: Operators, jdelta, rhat):
    """N(rhat) = int J_delta(r') exp(+j k_l rhat . r') dS' (Q7 per triangle)."""
    topo = ops.topo
    V = O.tri_vertices(topo)
    bq, wq = Q.q7()
    pts = Q.points(V, bq)                                    # (NT, 7, 3)
    rhat = np.atleast_2d(rhat)
    ph = np.exp(1j * ops.k_bg * np.einsum("dc,tkc->dtk", rhat, pts))   # (Nd, NT, 7)
    N = np.zeros((len(rhat), 3), complex)
    for i in range(3):
        f = topo.tri_signs[:, i][:, None, None] * (pts - V[:, i][:, None, :]) / (2 * topo.area[:, None, None])
        coef = jdelta[topo.tri_edges[:, i]]                  # (NT,)
        N += np.einsum("t,dtk,tkc,k->dc", coef * topo.area, ph, f, wq)
    return N


def rcs(ops: Operators, sol: Solution, rhat, E0=1.0):
    """Bistatic radar cross-section (m^2) of J_delta = (a - a_eq)/(jk0) radiating in the
    background: sigma = (k_l eta_l)^2 / (4 pi) |N_perp|^2 / |E0|^2."""
    jdelta = (sol.a - sol.a_eq) / (1j * ops.k0)
    N = far_field_N(ops, jdelta, rhat)
    rhat = np.atleast_2d(rhat)
    Nperp = N - np.einsum("dc,dc->d", N, rhat)[:, None] * rhat
    eta_l = C.ETA0 * np.sqrt(ops.mu_bg / ops.eps_bg)
    return (abs(ops.k_bg * eta_l) ** 2) / (4 * math.pi) * np.sum(np.abs(Nperp) ** 2, axis=1) / abs(E0) ** 2
