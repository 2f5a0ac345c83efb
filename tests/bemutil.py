"""Test helpers: map the library's edge numbering onto the oracle's and back.

Both sides number triangles like the caller; edges are matched by their vertex pair.
"""
from __future__ import annotations

import numpy as np


def edge_perm(lib_va, lib_vb, oracle_edges) -> np.ndarray:
    """perm[i] = oracle index of library edge i."""
    key = {(int(a), int(b)): i for i, (a, b) in enumerate(oracle_edges)}
    return np.array([key[(int(a), int(b))] for a, b in zip(lib_va, lib_vb)], dtype=np.int64)


def final_perm(perm: np.ndarray, ne: int, nq: int) -> np.ndarray:
    """Permutation of the final unknowns [a; e; x3] from library to oracle order."""
    return np.concatenate([perm, ne + perm, 2 * ne + np.arange(nq)])


def meq_perm(perm: np.ndarray, ne: int, nq: int) -> np.ndarray:
    return np.concatenate([perm, ne + np.arange(nq)])


def rel(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
