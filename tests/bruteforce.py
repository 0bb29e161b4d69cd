"""Brute-force full-grid references used to pin the oracle (tiny grids only).

Everything here is written independently of ``oracle/``: dense 1-D operator matrices
built entry by entry, separable operators as explicit Kronecker products on the full
grid, CP tensors reconstructed with einsum, and least-squares problems handed to
``numpy.linalg.lstsq``.
"""
from __future__ import annotations

import string
from functools import reduce
from typing import List, Sequence

import numpy as np


def dense_op(op) -> np.ndarray:
    n = op.n
    M = np.zeros((n, n))
    if op.kind == "identity":
        for i in range(n):
            M[i, i] = 1.0
    elif op.kind == "diag":
        for i in range(n):
            M[i, i] = op.data[i]
    elif op.kind == "band":
        h = op.half_bw
        for i in range(n):
            for j in range(2 * h + 1):
                M[i, (i + j - h) % n] += op.data[j, i]
    elif op.kind == "rank1":
        for i in range(n):
            for j in range(n):
                M[i, j] = op.data[0, i] * op.data[1, j]
    else:
        raise ValueError(op.kind)
    return M


def full_operator(L) -> np.ndarray:
    """Dense (prod n_k) x (prod n_k) matrix of sum_e coef_e kron_k E_k^e, acting on the
    C-order flattening of the full tensor."""
    total = None
    for e in range(L.n_terms):
        mats = [dense_op(L.ops[k][L.op_index[e, k]]) for k in range(L.d)]
        t = L.coef[e] * reduce(np.kron, mats)
        total = t if total is None else total + t
    return total


def cp_full(U: Sequence[np.ndarray]) -> np.ndarray:
    d = len(U)
    letters = string.ascii_lowercase[:d]
    spec = ",".join(c + "z" for c in letters) + "->" + letters
    return np.einsum(spec, *U)


def jacobian(U: Sequence[np.ndarray], q: int) -> np.ndarray:
    """J_q with vec_C(f) = J_q vec_F(U_q) for f = sum_l prod_k U_k[:, l]."""
    n, r = U[q].shape
    cols = []
    for l in range(r):
        for i in range(n):
            parts = []
            for k, u in enumerate(U):
                if k == q:
                    e = np.zeros(n)
                    e[i] = 1.0
                    parts.append(e)
                else:
                    parts.append(u[:, l])
            cols.append(reduce(np.kron, parts))
    return np.stack(cols, axis=1)


def lstsq_update(A, B, U: List[np.ndarray], V: Sequence[np.ndarray], q: int, source=None) -> np.ndarray:
    """argmin_{U_q} ||A f(U) - B f_n (- c)|| by dense least squares on the full grid."""
    Af = full_operator(A)
    g = full_operator(B) @ cp_full(V).reshape(-1)
    if source is not None:
        g = g + cp_full(source).reshape(-1)
    J = jacobian(U, q)
    x, *_ = np.linalg.lstsq(Af @ J, g, rcond=None)
    n, r = U[q].shape
    return x.reshape((n, r), order="F")


def full_step(A, B, f: np.ndarray) -> np.ndarray:
    """Exact full-grid implicit step A f_{n+1} = B f_n."""
    g = full_operator(B) @ f.reshape(-1)
    return np.linalg.solve(full_operator(A), g).reshape(f.shape)
