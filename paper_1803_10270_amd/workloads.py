"""Seeded synthetic inputs for the implicit CP-ALS time step.

This module only *describes* problems: grids, the 1-D finite-difference
operators that make up a separable operator (Section 3, eq. (Lz) and eq. (BLs)),
and initial conditions in canonical (CP) form (Section 2.1, eq. (functional-SSE)).
It performs none of the solver's arithmetic, so both the FP64 CPU oracle and the
GPU library consume exactly the same inputs.

Conventions
-----------
* A CP tensor is a list of ``d`` factor panels ``U[k]`` of shape ``(n_k, r)``
  (float64).  Column ``l`` of every panel together forms the l-th separable term.
* A 1-D operator (``Op1D``) is one of
    - ``identity``
    - ``diag``   : ``data`` has shape ``(n,)``; O = diag(data)
    - ``band``   : periodic band with half bandwidth ``h``; ``data`` has shape
                   ``(2h+1, n)`` with ``O[i, (i + j - h) mod n] = data[j, i]``
    - ``rank1``  : ``data`` has shape ``(2, n)``; O = outer(data[0], data[1])
* A separable operator (``SepOperator``) is ``sum_e coef[e] * kron_k ops[k][op_index[e, k]]``
  where ``ops[k]`` lists the distinct 1-D operators of dimension k (the "map of
  unique one-dimensional integrals" of Section 3.1).
* Grid: ``x_j = lo + (hi - lo) * j / n``, j = 0..n-1 (periodic, endpoint excluded).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PAD_SEED_OFFSET = 1_000_000


@dataclass
class Op1D:
    kind: str
    n: int
    data: Optional[np.ndarray] = None
    half_bw: int = 0

    def __post_init__(self):
        assert self.kind in ("identity", "diag", "band", "rank1"), self.kind
        if self.kind == "diag":
            assert self.data.shape == (self.n,)
        elif self.kind == "band":
            assert self.data.shape == (2 * self.half_bw + 1, self.n)
        elif self.kind == "rank1":
            assert self.data.shape == (2, self.n)


@dataclass
class SepOperator:
    coef: np.ndarray            # (T,) float64
    op_index: np.ndarray        # (T, d) int32 into ops[k]
    ops: List[List[Op1D]]       # per dimension: distinct 1-D operators

    @property
    def d(self) -> int:
        return len(self.ops)

    @property
    def n_terms(self) -> int:
        return int(self.coef.shape[0])

    def dims(self) -> List[int]:
        return [self.ops[k][0].n for k in range(self.d)]


@dataclass
class Problem:
    """One implicit step problem family: A f_{n+1} = B f_n, repeated n_steps times."""
    name: str
    A: SepOperator
    B: SepOperator
    f0: List[np.ndarray]        # initial condition, CP factors (n_k, r0)
    guess: List[np.ndarray]     # first-step initial guess, padded to the rank cap
    rank_cap: int
    dt: float
    n_steps: int
    tol: float
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------------------------
# grids and 1-D operators (operator entries are problem inputs)
# ----------------------------------------------------------------------------------

def grid(n: int, lo: float = -np.pi, hi: float = np.pi) -> np.ndarray:
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / n


def op_identity(n: int) -> Op1D:
    return Op1D("identity", n)


def op_central_diff(n: int, length: float = 2 * np.pi) -> Op1D:
    """Second-order periodic central difference (u_{j+1} - u_{j-1}) / (2h)."""
    h = length / n
    data = np.zeros((3, n))
    data[0, :] = -1.0 / (2.0 * h)
    data[2, :] = 1.0 / (2.0 * h)
    return Op1D("band", n, data, 1)


def op_diag(values: np.ndarray) -> Op1D:
    v = np.asarray(values, dtype=np.float64)
    return Op1D("diag", v.shape[0], v.copy())


def op_rank1(m: np.ndarray, w: np.ndarray) -> Op1D:
    return Op1D("rank1", m.shape[0], np.stack([m, w]).astype(np.float64))


def identity_operator(dims: List[int]) -> SepOperator:
    return SepOperator(np.ones(1), np.zeros((1, len(dims)), np.int32),
                       [[op_identity(n)] for n in dims])


# ----------------------------------------------------------------------------------
# initial conditions
# ----------------------------------------------------------------------------------

def periodic_gaussian(x: np.ndarray, c: float, w: float, length: float = 2 * np.pi) -> np.ndarray:
    """Sum over three periodic images of exp(-(x - c)^2 / (2 w^2))."""
    g = np.zeros_like(x)
    for p in (-1, 0, 1):
        g += np.exp(-((x - c + length * p) ** 2) / (2.0 * w * w))
    return g


def gaussian_mixture(rng: np.random.Generator, d: int, n: int, terms: int) -> List[np.ndarray]:
    x = grid(n)
    U = [np.zeros((n, terms)) for _ in range(d)]
    for l in range(terms):
        c = rng.uniform(-1.0, 1.0, size=d)
        w = rng.uniform(0.3, 0.6, size=d)
        for k in range(d):
            U[k][:, l] = periodic_gaussian(x, c[k], w[k])
    return U


def pad_rank(U: List[np.ndarray], cap: int, seed: int) -> List[np.ndarray]:
    """Fixed-rank initial guess: extra columns are seeded unit directions with a zero
    factor in dimension 0, so the represented tensor is unchanged (a "small random
    perturbation" of the previous solution with zero amplitude, Section 3.1)."""
    r0 = U[0].shape[1]
    if r0 >= cap:
        return [u.copy() for u in U]
    rng = np.random.default_rng(seed + PAD_SEED_OFFSET)
    out = []
    for k, u in enumerate(U):
        n = u.shape[0]
        extra = rng.standard_normal((n, cap - r0))
        extra /= np.linalg.norm(extra, axis=0, keepdims=True)
        if k == 0:
            extra[:] = 0.0
        out.append(np.concatenate([u, extra], axis=1))
    return out


# ----------------------------------------------------------------------------------
# problem families
# ----------------------------------------------------------------------------------

def advection_cn_constant(seed: int = 0, d: int = 6, n: int = 32, dt: float = 1e-3, ic_rank: int = 2,
                          cap: int = 4, n_steps: int = 10, tol: float = 1e-10,
                          velocity: Optional[np.ndarray] = None) -> Problem:
    """u_t + sum_i a_i du/dx_i = 0 on [-pi, pi)^d, Crank-Nicolson (eq. (CNFDE)):
    A = I + dt/2 sum_i a_i D_i,  B = I - dt/2 sum_i a_i D_i."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=d) if velocity is None else np.asarray(velocity, float)
    f0 = gaussian_mixture(rng, d, n, ic_rank)
    ops = [[op_identity(n), op_central_diff(n)] for _ in range(d)]
    idx = np.zeros((d + 1, d), np.int32)
    for i in range(d):
        idx[i + 1, i] = 1
    A = SepOperator(np.concatenate([[1.0], 0.5 * dt * a]), idx.copy(), ops)
    B = SepOperator(np.concatenate([[1.0], -0.5 * dt * a]), idx.copy(), ops)
    return Problem("advection_cn_constant", A, B, f0, pad_rank(f0, cap, seed), cap, dt, n_steps, tol,
                   {"velocity": a, "seed": seed})


def advection_ie_variable(seed: int = 0, d: int = 6, n: int = 256, dt: float = 1e-3, ic_rank: int = 8,
                          cap: int = 32, n_steps: int = 100, tol: float = 1e-8) -> Problem:
    """u_t + sum_i a_i(x) du/dx_i = 0 with a_i(x) = 1 + 0.5 sin(x_{(i+1) mod d}) (0-based),
    implicit Euler: A = I + dt sum_i (D_i + 0.5 S_{(i+1) mod d} D_i), B = I.
    2d + 1 Kronecker terms; distinct 1-D operators per dimension: {I, D, diag(sin x)}."""
    rng = np.random.default_rng(seed)
    f0 = gaussian_mixture(rng, d, n, ic_rank)
    x = grid(n)
    ops = [[op_identity(n), op_central_diff(n), op_diag(np.sin(x))] for _ in range(d)]
    T = 2 * d + 1
    coef = np.zeros(T)
    idx = np.zeros((T, d), np.int32)
    coef[0] = 1.0
    for i in range(d):
        coef[1 + i] = dt
        idx[1 + i, i] = 1
        coef[1 + d + i] = 0.5 * dt
        idx[1 + d + i, i] = 1
        idx[1 + d + i, (i + 1) % d] = 2
    A = SepOperator(coef, idx, ops)
    B = identity_operator([n] * d)
    return Problem("advection_ie_variable", A, B, f0, pad_rank(f0, cap, seed), cap, dt, n_steps, tol,
                   {"seed": seed})


def advection_ie_constant(seed: int, d: int, n: int, cap: int, ic_rank: int, dt: float = 1e-3,
                          n_steps: int = 20, tol: float = 1e-8) -> Problem:
    """Constant-velocity advection, implicit Euler: A = I + dt sum_i a_i D_i, B = I."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=d)
    f0 = gaussian_mixture(rng, d, n, ic_rank)
    ops = [[op_identity(n), op_central_diff(n)] for _ in range(d)]
    idx = np.zeros((d + 1, d), np.int32)
    for i in range(d):
        idx[i + 1, i] = 1
    A = SepOperator(np.concatenate([[1.0], dt * a]), idx, ops)
    B = identity_operator([n] * d)
    return Problem("advection_ie_constant", A, B, f0, pad_rank(f0, cap, seed), cap, dt, n_steps, tol,
                   {"velocity": a, "seed": seed})


def batched_instances(count: int = 256, base_seed: int = 10_000, n_steps: int = 20) -> List[Problem]:
    """Uneven advection instances: d in {4, 6}, n in {64, 128, 256, 512}, cap in 4..48,
    IC rank in 2..8 (at most cap), constant velocities U(-1, 1), implicit Euler."""
    out = []
    for i in range(count):
        seed = base_seed + i
        rng = np.random.default_rng(seed)
        d = int(rng.choice([4, 6]))
        n = int(rng.choice([64, 128, 256, 512]))
        cap = int(rng.integers(4, 49))
        ic_rank = min(int(rng.integers(2, 9)), cap)
        out.append(advection_ie_constant(seed + 7, d, n, cap, ic_rank, n_steps=n_steps))
    return out


def maxwellian_1d(v: np.ndarray, hv: float) -> np.ndarray:
    """Discrete 1-D Maxwellian (RT = 1) normalised so that hv * sum(m) = 1."""
    m = np.exp(-0.5 * v * v)
    return m / (hv * m.sum())


def kinetic_cn(seed: int = 0, n: int = 128, nu: float = 1.0, dt: float = 0.01, field_rank: int = 16,
               eps: float = 0.1, cap: int = 64, n_steps: int = 50, tol: float = 1e-8,
               vmax: float = 5.0) -> Problem:
    """Linearised kinetic model in 3 space + 3 velocity dimensions (dims 0-2: x, 3-5: v):
    f_t = L f,  L = -sum_i diag(v_i) D_{x_i} - nu I + nu (I_x (x) Pi (x) Pi (x) Pi),
    Pi = m w^T with w = h_v 1 and m the discrete Maxwellian (w^T m = 1): relaxation of f to
    M(v) rho[f], cf. Section 4.2, eqs. (BGK_LIN), (opL) and Table (tab:ordering).
    Crank-Nicolson: A = I - dt/2 L, B = I + dt/2 L (5 terms each)."""
    rng = np.random.default_rng(seed)
    x = grid(n)
    v = grid(n, -vmax, vmax)
    hv = 2 * vmax / n
    m = maxwellian_1d(v, hv)
    w = np.full(n, hv)
    xops = [op_identity(n), op_central_diff(n)]
    vops = [op_identity(n), op_diag(v), op_rank1(m, w)]
    ops = [list(xops) for _ in range(3)] + [list(vops) for _ in range(3)]
    # terms: identity, three transport terms v_i d/dx_i, Maxwellian projection on v
    idx = np.zeros((5, 6), np.int32)
    for i in range(3):
        idx[1 + i, i] = 1
        idx[1 + i, 3 + i] = 1
    idx[4, 3:] = 2
    coefL = np.array([-nu, -1.0, -1.0, -1.0, nu])
    cA = -0.5 * dt * coefL
    cA[0] += 1.0
    cB = 0.5 * dt * coefL
    cB[0] += 1.0
    A = SepOperator(cA, idx.copy(), ops)
    B = SepOperator(cB, idx.copy(), ops)
    # f0 = M(v) (1 + eps * g), g = (1/R) sum of R separable low-frequency trig products
    R = field_rank
    U = [np.zeros((n, R + 1)) for _ in range(6)]
    for k in range(3):
        U[k][:, 0] = 1.0
    for k in range(3, 6):
        U[k][:, 0] = m
    for l in range(R):
        for k in range(6):
            coord = x if k < 3 else v * (np.pi / vmax)
            g = np.zeros(n)
            for f in range(1, 4):
                a, b = rng.standard_normal(2)
                g += a * np.cos(f * coord) + b * np.sin(f * coord)
            g /= np.max(np.abs(g))
            if k >= 3:
                g = g * m
            U[k][:, 1 + l] = g
        U[0][:, 1 + l] *= eps / R
    return Problem("kinetic_cn", A, B, U, pad_rank(U, cap, seed), cap, dt, n_steps, tol,
                   {"nu": nu, "seed": seed, "maxwellian": m, "w": w})


def bgk_linear_cn(seed: int = 0, n: int = 32, nu: float = 1.0, dt: float = 0.01, field_rank: int = 3,
                  eps: float = 0.1, cap: int = 8, n_steps: int = 10, tol: float = 1e-8, vmax: float = 5.0,
                  x_dependent: bool = True) -> Problem:
    """The linearised BGK equation with a fixed equilibrium (Section 4.2, eqs. BGK_LIN, opL):
    f_t = L f + nu f_eq,  L = -sum_i diag(v_i) D_{x_i} - nu I,  f_eq = M(v) (x) 1_x, in 3 space
    + 3 velocity dimensions (dims 0-2: x, 3-5: v).  Crank-Nicolson with the source applied once:
    A f_{n+1} = B f_n + c, A = I - dt/2 L, B = I + dt/2 L (4 terms each), c = dt nu f_eq
    (rank 1, in problem.meta["source"]).  f0 = f_eq + eps M(v) g with g a sum of field_rank
    separable low-frequency trig products (x-independent when x_dependent is False)."""
    rng = np.random.default_rng(seed)
    x = grid(n)
    v = grid(n, -vmax, vmax)
    hv = 2 * vmax / n
    m = maxwellian_1d(v, hv)
    xops = [op_identity(n), op_central_diff(n)]
    vops = [op_identity(n), op_diag(v)]
    ops = [list(xops) for _ in range(3)] + [list(vops) for _ in range(3)]
    idx = np.zeros((4, 6), np.int32)
    for i in range(3):
        idx[1 + i, i] = 1
        idx[1 + i, 3 + i] = 1
    coefL = np.array([-nu, -1.0, -1.0, -1.0])
    cA = -0.5 * dt * coefL
    cA[0] += 1.0
    cB = 0.5 * dt * coefL
    cB[0] += 1.0
    A = SepOperator(cA, idx.copy(), ops)
    B = SepOperator(cB, idx.copy(), ops)
    feq = [np.ones((n, 1)) for _ in range(3)] + [m[:, None].copy() for _ in range(3)]
    source = [f.copy() for f in feq]
    source[0] = source[0] * (dt * nu)
    R = field_rank
    U = [np.concatenate([f, np.zeros((n, R))], axis=1) for f in feq]
    for l in range(R):
        for k in range(6):
            coord = x if k < 3 else v * (np.pi / vmax)
            if k < 3 and not x_dependent:
                g = np.ones(n)
            else:
                g = np.zeros(n)
                for f in range(1, 4):
                    a, b = rng.standard_normal(2)
                    g += a * np.cos(f * coord) + b * np.sin(f * coord)
                g /= np.max(np.abs(g))
            if k >= 3:
                g = g * m
            U[k][:, 1 + l] = g
        U[0][:, 1 + l] *= eps / R
    return Problem("bgk_linear_cn", A, B, U, pad_rank(U, cap, seed), cap, dt, n_steps, tol,
                   {"nu": nu, "seed": seed, "maxwellian": m, "feq": feq, "source": source, "hx": 2 * np.pi / n,
                    "hv": hv})


CD6 = np.array([-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0]) / 60.0   # 6th-order first derivative, offsets -3..3


def op_central_diff6(x: np.ndarray) -> Op1D:
    """Sixth-order periodic central difference on the uniform grid x (band, half width 3)."""
    n = x.size
    h = (x[1] - x[0])
    return Op1D("band", n, np.repeat((CD6 / h)[:, None], n, axis=1), 3)


def op_times_diff6(x: np.ndarray) -> Op1D:
    """diag(x) times the sixth-order central difference (band, half width 3)."""
    n = x.size
    h = (x[1] - x[0])
    return Op1D("band", n, (CD6 / h)[:, None] * x[None, :], 3)


def spiral_generator(C: np.ndarray, x: np.ndarray) -> SepOperator:
    """L f = -sum_{j,k} C_jk z_k d f / d z_j as a separable operator of N^2 terms in the
    ordering of the paper's Table (tab:ordering0): term (j, k) has z_j d/dz_j in dimension j when
    j = k, else d/dz_j in dimension j and z_k in dimension k, coefficient -C_jk.  Distinct
    operators per dimension: [I, D, Z, Z D]."""
    N = C.shape[0]
    n = x.size
    ops = [[op_identity(n), op_central_diff6(x), op_diag(x), op_times_diff6(x)] for _ in range(N)]
    idx = np.zeros((N * N, N), np.int32)
    coef = np.zeros(N * N)
    for j in range(N):
        for k in range(N):
            t = j * N + k
            if j == k:
                idx[t, j] = 3
            else:
                idx[t, j] = 1
                idx[t, k] = 2
            coef[t] = -C[j, k]
    return SepOperator(coef, idx, ops)


def spiral_matrix(seed: int, N: int, decay: float = 0.5) -> np.ndarray:
    """Seeded C = decay I + K with K skew-symmetric (K = (G - G^T)/2, G ~ N(0, 1)): complex
    eigenvalues with real part decay > 0, a stable spiral of the characteristics."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((N, N))
    return decay * np.eye(N) + 0.5 * (G - G.T)


def spiral_advection_cn(seed: int = 0, N: int = 6, n: int = 64, b: float = 6.0, dt: float = 0.01, cap: int = 4,
                        n_steps: int = 10, tol: float = 1e-8) -> Problem:
    """The paper's advection benchmark with a linear velocity field (Section 4.1, eq. PDE-advR):
    f_t + sum_j (C z)_j df/dz_j = 0 on the periodic box [-b, b)^N, f0 = exp(-|z|^2) (rank 1),
    exact solution f0(exp(-t C) z) (eq. solutionF).  Sixth-order central differences;
    Crank-Nicolson A = I - dt/2 L, B = I + dt/2 L with N^2 + 1 terms each."""
    x = grid(n, -b, b)
    C = spiral_matrix(seed, N)
    L = spiral_generator(C, x)
    T = L.n_terms
    idx = np.concatenate([np.zeros((1, N), np.int32), L.op_index], axis=0)
    A = SepOperator(np.concatenate([[1.0], -0.5 * dt * L.coef]), idx.copy(), L.ops)
    B = SepOperator(np.concatenate([[1.0], 0.5 * dt * L.coef]), idx.copy(), L.ops)
    f0 = [np.exp(-x * x)[:, None] for _ in range(N)]
    return Problem("spiral_advection_cn", A, B, f0, pad_rank(f0, cap, seed), cap, dt, n_steps, tol,
                   {"C": C, "L": L, "x": x, "b": b, "terms": T})


def spiral_exact(C: np.ndarray, z: np.ndarray, t: float) -> float:
    """f(z, t) = exp(-|exp(-t C) z|^2) (eq. solutionF with f0 = exp(-|z|^2))."""
    from scipy.linalg import expm
    y = expm(-t * C) @ np.asarray(z, dtype=np.float64)
    return float(np.exp(-y @ y))


def random_factors(rng: np.random.Generator, dims: List[int], r: int) -> List[np.ndarray]:
    return [rng.standard_normal((n, r)) for n in dims]
