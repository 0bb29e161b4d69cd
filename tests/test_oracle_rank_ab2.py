"""Pins of the oracle's residual, adaptive-rank and explicit (AB2) parts.

Each test names what fixes the expected value: exact rational arithmetic, the published
outputs of the SplitMix64 generator, the Eckart-Young theorem, the monotonicity of
alternating minimisation, and full-grid / Fourier solutions of the AB2 recurrence.  None
re-types the oracle's own formulas.
"""
from fractions import Fraction

import numpy as np
import pytest

from bruteforce import cp_full, dense_op, full_operator
from oracle import cpals_oracle as O
from oracle import ddarith as DD
from paper_1803_10270_amd import workloads as W


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- double-double pieces

def test_error_free_transforms_are_exact():
    """TwoSum and TwoProduct return the rounding error exactly (checked in rationals)."""
    rng = np.random.default_rng(0)
    a = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    b = rng.standard_normal(200) * 10.0 ** rng.integers(-8, 8, 200)
    s, e = DD.two_sum(a, b)
    p, f = DD.two_prod(a, b)
    for i in range(200):
        assert Fraction(s[i]) + Fraction(e[i]) == Fraction(a[i]) + Fraction(b[i])
        assert Fraction(p[i]) + Fraction(f[i]) == Fraction(a[i]) * Fraction(b[i])


def exact_norm2(factors):
    """||sum_l prod_k W_k[:, l]||^2 in rational arithmetic on the full grid (tiny sizes)."""
    full = cp_full(factors)   # only for the shape
    dims = full.shape
    Wf = [[[Fraction(x) for x in col] for col in W_.T] for W_ in factors]
    r = factors[0].shape[1]
    tot = Fraction(0)
    for idx in np.ndindex(*dims):
        v = Fraction(0)
        for l in range(r):
            t = Fraction(1)
            for k, i in enumerate(idx):
                t *= Wf[k][l][i]
            v += t
        tot += v * v
    return tot


@pytest.mark.parametrize("log2eps", [-20, -30, -40])
def test_residual_resolves_below_float64_floor(log2eps):
    """rho = ||f - g|| / ||g|| for g = u (x) v + eps w (x) z and f = 3u (x) v/3 (equal to
    u (x) v up to the rounding of v/3): the oracle's double-double residual matches exact
    rational arithmetic; the float64 Gram expansion cannot resolve it (its floor is
    ~1e-8 relative)."""
    rng = np.random.default_rng(-log2eps)
    n, eps = 12, 2.0 ** log2eps
    u, v, w, z = [rng.standard_normal(n) for _ in range(4)]
    f = [3 * u[:, None], (v / 3)[:, None]]
    g = [np.stack([u, eps * w], 1), np.stack([v, z], 1)]
    I = W.identity_operator([n, n])
    diff = [np.concatenate([f[0], -g[0]], 1), np.concatenate([f[1], g[1]], 1)]
    exact = float(exact_norm2(diff) / exact_norm2(g)) ** 0.5
    rho = O.residual(I, I, f, g)
    assert abs(rho - exact) <= 1e-6 * exact
    if log2eps <= -30:   # float64 expansion: wrong by orders of magnitude (or zero)
        X = diff
        H = np.ones((3, 3))
        for x in X:
            H = H * (x.T @ x)
        naive = np.sqrt(max(H.sum(), 0.0) / O.cp_inner(g, g))
        assert abs(naive - exact) > 0.5 * exact


def test_residual_with_operator_matches_rational_full_grid():
    """The residual of an implicit step with dyadic operator entries (so every applied
    value is exact) against the full-grid residual in rational arithmetic."""
    rng = np.random.default_rng(5)
    dims = [4, 3, 4]
    ops = [[W.op_identity(n), W.Op1D("band", n, np.array([[-0.5] * n, [0.0] * n, [0.5] * n]), 1),
            W.op_diag(np.array([0.25 * (i + 1) for i in range(n)]))] for n in dims]
    A = W.SepOperator(np.array([1.0, 0.125, -0.0625, 0.03125]),
                      np.array([[0, 0, 0], [1, 0, 0], [0, 1, 2], [2, 2, 1]], np.int32), ops)
    B = W.identity_operator(dims)
    V = W.random_factors(rng, dims, 2)
    # f: A^{-1} g up to a tiny perturbation, so the residual is small
    g = cp_full(V).reshape(-1)
    Af = full_operator(A)
    U = [np.array(v) for v in V]
    rho = O.residual(A, B, U, V)
    # rational full grid: ||A f - g|| with A's dyadic entries and f's float entries exact
    fvec = [Fraction(x) for x in cp_full(U).reshape(-1)]
    # cp_full rounds; rebuild f exactly from the factors instead
    fvec = []
    for idx in np.ndindex(*dims):
        s = Fraction(0)
        for l in range(U[0].shape[1]):
            t = Fraction(1)
            for k, i in enumerate(idx):
                t *= Fraction(U[k][i, l])
            s += t
        fvec.append(s)
    N = len(fvec)
    Afr = [[Fraction(Af[i, j]) for j in range(N)] for i in range(N)]
    res = [sum(Afr[i][j] * fvec[j] for j in range(N) if Afr[i][j] != 0) - fvec[i] for i in range(N)]
    exact = float(sum(x * x for x in res) / sum(x * x for x in fvec)) ** 0.5
    assert abs(rho - exact) <= 1e-12 * exact
    assert abs(Af @ g - g).max() > 0   # a non-trivial operator


# ---------------------------------------------------------------- growth directions

def test_splitmix64_published_outputs():
    """The generator's first three outputs for seed 0 are the published ones of the
    SplitMix64 reference implementation."""
    assert O.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert O.splitmix64(0, 2) == 0x06C45D188009454F


def test_growth_column_layout():
    """Zero in dimension 0 (the represented tensor is unchanged), values 2u - 1 in [-1, 1)
    elsewhere, distinct for every (step, column, dimension)."""
    n = 64
    assert not O.growth_column(7, 0, 3, 0, n).any()
    cols = [O.growth_column(7, s, l, k, n) for s in (0, 1) for l in (3, 4) for k in (1, 2)]
    for c in cols:
        assert c.min() >= -1.0 and c.max() < 1.0 and abs(c.mean()) < 0.3
    for i in range(len(cols)):
        for j in range(i):
            assert not np.array_equal(cols[i], cols[j])
    u = (O.splitmix64(7, ((0 * 64 + 3) * 8 + 1) << 32) >> 11) * 2.0 ** -53
    assert O.growth_column(7, 0, 3, 1, n)[0] == 2 * u - 1


def test_drop_small_terms_keeps_order():
    rng = np.random.default_rng(3)
    U = W.random_factors(rng, [5, 6, 7], 5)
    U[1][:, 1] *= 1e-16
    U[2][:, 3] = 0.0
    D = O.drop_small_terms(U)
    assert D[0].shape[1] == 3
    for k in range(3):
        assert np.array_equal(D[k], U[k][:, [0, 2, 4]])


# ---------------------------------------------------------------- adaptive rank

def test_adaptive_rank_grows_to_exact_rank():
    """Fitting a rank-3 tensor (A = B = I) from rank 1 with a tolerance far below the
    rank-2 error: the rank grows one term at a time to exactly 3 and the residual, resolved
    in double-double, falls to the rounding level."""
    rng = np.random.default_rng(21)
    dims = [6, 7, 5]
    G = W.random_factors(rng, dims, 3)
    I = W.identity_operator(dims)
    start = [g[:, :1] + 0.1 * rng.standard_normal((g.shape[0], 1)) for g in G]
    U, rep = O.adaptive_step(I, I, G, start, cap=6, tau=1e-10, tol=1e-13, max_sweeps=2000, eps_reg=1e-14,
                             seed=11)
    assert [r for r, _ in rep["log"]] == [1, 2, 3]
    assert rep["final_rank"] == 3
    assert rep["log"][1][1] > 1e-3 and rep["rel_residual"] <= 1e-12
    assert rel(cp_full(U), cp_full(G)) <= 1e-12


def test_adaptive_rank_d2_follows_the_svd():
    """d = 2: the best rank-r fit is the truncated SVD (Eckart-Young), so every logged
    residual equals the singular-value tail and the accepted rank is the first whose tail
    is below tau."""
    rng = np.random.default_rng(4)
    n = 10
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 4.0 ** -np.arange(n)
    G = [Q1 * s, Q2]
    tails = np.sqrt([np.sum(s[r:] ** 2) for r in range(n + 1)]) / np.linalg.norm(s)
    tau = 1e-4
    expect = int(np.argmax(tails <= tau))
    I = W.identity_operator([n, n])
    start = [rng.standard_normal((n, 1)), rng.standard_normal((n, 1))]
    U, rep = O.adaptive_step(I, I, G, start, cap=n, tau=tau, tol=1e-14, max_sweeps=3000, eps_reg=0.0, seed=2)
    assert rep["final_rank"] == expect == 7
    for r, rho in rep["log"]:
        assert abs(rho - tails[r]) <= 1e-6 * tails[r], (r, rho, tails[r])


def test_adaptive_residual_never_increases_with_rank_for_truncation():
    """A = B = I (rank reduction): the appended term is a rank-1 least-squares fit of the
    residual g - f started from a zero first factor, so ||g - (f + t)|| <= ||g - f||, and
    every later update is the exact minimiser over one factor (Section 3.1): the logged
    residual cannot increase with the rank."""
    rng = np.random.default_rng(8)
    dims = [7, 6, 8]
    G = W.random_factors(rng, dims, 6)
    I = W.identity_operator(dims)
    start = [g[:, :1] for g in G]
    U, rep = O.adaptive_step(I, I, G, start, cap=5, tau=1e-14, tol=1e-12, max_sweeps=60, eps_reg=1e-14, seed=5)
    rhos = [rho for _, rho in rep["log"]]
    assert [r for r, _ in rep["log"]] == [1, 2, 3, 4, 5]
    for a, b in zip(rhos, rhos[1:]):
        assert b <= a * (1 + 1e-9)
    assert rhos[-1] < 0.5 * rhos[0]


def test_growth_term_recovers_a_rank_one_residual():
    """When g - f is exactly a rank-1 tensor s (g = f + s, A = B = I), one sweep of the
    rank-1 fit already reproduces s: checked on the full grid."""
    rng = np.random.default_rng(12)
    dims = [5, 6, 4]
    F = W.random_factors(rng, dims, 3)
    S = W.random_factors(rng, dims, 1)
    G = [np.concatenate([f, s], axis=1) for f, s in zip(F, S)]
    I = W.identity_operator(dims)
    t = O.growth_term(I, I, F, G, seed=4, step=0)
    assert rel(cp_full([x[:, None] for x in t]), cp_full(S)) <= 1e-12


def test_growth_term_d2_is_power_iteration():
    """d = 2: a sweep of rank-1 ALS on the residual matrix R is one step of the power
    method, so after three sweeps t_0 t_1^T = u u^T R / (u^T u) with
    u = R (R^T R)^2 t_1^(0) (dense matrices, computed without the CP form)."""
    rng = np.random.default_rng(6)
    n0, n1 = 9, 7
    F = W.random_factors(rng, [n0, n1], 2)
    G = W.random_factors(rng, [n0, n1], 4)
    I = W.identity_operator([n0, n1])
    t = O.growth_term(I, I, F, G, seed=17, step=3)
    Rm = cp_full(G) - cp_full(F)
    t1 = O.growth_column(17, 3, 2, 1, n1)
    u = Rm @ (Rm.T @ (Rm @ (Rm.T @ (Rm @ t1))))
    expect = np.outer(u, u) @ Rm / (u @ u)
    assert rel(np.outer(t[0], t[1]), expect) <= 1e-12


def test_adaptive_replay_reproduces_the_logged_decisions():
    """Replaying the logged final rank follows the same decisions to the same result."""
    p = W.advection_ie_variable(seed=1, d=3, n=8, ic_rank=2, cap=5)
    U, rep = O.adaptive_step(p.A, p.B, p.f0, p.f0, cap=5, tau=5e-5, tol=1e-10, max_sweeps=40, seed=9)
    assert 2 < rep["final_rank"] < 5
    U2, rep2 = O.adaptive_step(p.A, p.B, p.f0, p.f0, cap=5, tau=0.0, tol=1e-10, max_sweeps=40, seed=9,
                               replay_rank=rep["final_rank"])
    assert [r for r, _ in rep2["log"]] == [r for r, _ in rep["log"]]
    for a, b in zip(U, U2):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- explicit AB2 (Section 3.2)

def ab2_dense(Lm, dt, f0, f1, steps):
    fs = [f0, f1]
    for _ in range(steps):
        fs.append(fs[-1] + 0.5 * dt * (Lm @ (3 * fs[-1] - fs[-2])))
    return fs


def test_ab2_d1_is_the_vector_recurrence():
    """d = 1: every CP tensor is one vector, so the rank reductions are exact and the CP
    form reproduces the AB2 recurrence of eq. (AB2_) on the vector."""
    n, dt = 32, 0.05
    rng = np.random.default_rng(6)
    ops = [[W.op_identity(n), W.op_central_diff(n), W.op_diag(rng.uniform(0.5, 1.5, n))]]
    L = W.SepOperator(np.array([-0.3, -1.0, 0.4]), np.array([[0], [1], [2]], np.int32), ops)
    Lm = full_operator(L)
    f0, f1 = rng.standard_normal(n), rng.standard_normal(n)
    ref = ab2_dense(Lm, dt, f0, f1, 5)
    Fp, Fc = [f0[:, None]], [f1[:, None]]
    for s in range(5):
        Fn, rep = O.ab2_step(L, dt, Fp, Fc, cap=1, eps_reg=0.0)
        Fp, Fc = Fc, Fn
        assert rel(cp_full(Fc), ref[s + 2]) <= 1e-13


def test_ab2_single_direction_advection_matches_fourier():
    """u_t + a u_x1 = 0 in d = 3 (central differences): the CP AB2 step keeps the other
    factors and advances each column's first factor by the AB2 recurrence, whose Fourier
    multiplier per mode is known in closed form."""
    n, d, dt, a = 16, 3, 0.02, 0.8
    rng = np.random.default_rng(7)
    ops = [[W.op_central_diff(n)]] + [[W.op_identity(n)] for _ in range(d - 1)]
    L = W.SepOperator(np.array([-a]), np.zeros((1, d), np.int32), ops)
    f0 = W.gaussian_mixture(rng, d, n, 2)
    # first level: the exact semi-discrete solution (Fourier) at t = dt
    m = np.fft.fftfreq(n, 1.0 / n)
    h = 2 * np.pi / n
    lam = -a * 1j * np.sin(m * h) / h          # symbol of -a D
    def evolve(F, mult):
        return [np.real(np.fft.ifft(mult[:, None] * np.fft.fft(F[0], axis=0), axis=0))] + [f.copy() for f in F[1:]]
    f1 = evolve(f0, np.exp(lam * dt))
    # AB2 multipliers: y_{k+2} = y_{k+1} + dt/2 lam (3 y_{k+1} - y_k) mode by mode
    y0, y1 = np.ones(n, complex), np.exp(lam * dt)
    Fp, Fc = f0, f1
    for s in range(6):
        Fn, rep = O.ab2_step(L, dt, Fp, Fc, cap=2, tol=1e-14, eps_reg=0.0)
        y0, y1 = y1, y1 + 0.5 * dt * lam * (3 * y1 - y0)
        ref = evolve(f0, y1)
        assert rel(cp_full(Fn), cp_full(ref)) <= 1e-11
        assert Fn[0].shape[1] == 2
        Fp, Fc = Fc, Fn


def test_ab2_d2_full_rank_matches_full_grid():
    """d = 2 at rank n: CP represents every n x n grid function, every reduction is exact,
    and the CP AB2 step equals the full-grid AB2 step of a two-direction variable
    coefficient operator."""
    n, dt = 8, 0.02
    rng = np.random.default_rng(8)
    x = W.grid(n)
    ops = [[W.op_identity(n), W.op_central_diff(n), W.op_diag(np.sin(x))] for _ in range(2)]
    L = W.SepOperator(np.array([-1.0, -0.7, -0.5]), np.array([[1, 0], [0, 1], [1, 2]], np.int32), ops)
    Lm = full_operator(L)
    F0 = W.random_factors(rng, [n, n], n)
    F1 = W.random_factors(rng, [n, n], n)
    ref = ab2_dense(Lm, dt, cp_full(F0).reshape(-1), cp_full(F1).reshape(-1), 2)
    Fp, Fc = F0, F1
    for s in range(2):
        Fn, rep = O.ab2_step(L, dt, Fp, Fc, cap=n, tol=1e-14, max_sweeps=500, eps_reg=0.0)
        assert rel(cp_full(Fn).reshape(-1), ref[s + 2]) <= 1e-9
        Fp, Fc = Fc, Fn
