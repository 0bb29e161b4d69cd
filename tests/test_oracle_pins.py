"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's formulas:
they compare against full-grid brute force (explicit Kronecker operators, dense least
squares), closed forms (Fourier symbols, exact 1-D solves, SVD truncation) and
invariants (mass, CN norm, steady state, relaxation rate).
"""
import numpy as np
import pytest

from bruteforce import cp_full, dense_op, full_operator, full_step, lstsq_update
from oracle import cpals_oracle as O
from paper_1803_10270_amd import workloads as W


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def mixed_operator(rng, dims, n_terms, with_rank1=True, scale=0.3):
    """Random separable operator whose dimensions carry {I, D, diag, rank-1} operators."""
    ops = []
    for n in dims:
        o = [W.op_identity(n), W.op_central_diff(n), W.op_diag(rng.uniform(-1, 1, n))]
        if with_rank1:
            o.append(W.op_rank1(rng.uniform(0, 1, n), rng.uniform(0, 1, n) / n))
        ops.append(o)
    idx = rng.integers(0, len(ops[0]), size=(n_terms, len(dims))).astype(np.int32)
    idx[0, :] = 0
    coef = np.concatenate([[1.0], scale * rng.uniform(-1, 1, n_terms - 1)])
    return W.SepOperator(coef, idx, ops)


# ----------------------------------------------------------------------------- CP basics

def test_inner_and_norm_bruteforce():
    """Scalar products of canonical tensors reduce to 1-D products (Section 2.2, last
    paragraph): compare with the inner product of the reconstructed full tensors."""
    rng = np.random.default_rng(1)
    X = W.random_factors(rng, [5, 6, 7], 3)
    Y = W.random_factors(rng, [5, 6, 7], 2)
    assert abs(O.cp_inner(X, Y) - np.vdot(cp_full(X), cp_full(Y))) <= 1e-12 * np.linalg.norm(cp_full(X)) * np.linalg.norm(cp_full(Y))
    assert abs(O.cp_norm(X) - np.linalg.norm(cp_full(X))) <= 1e-13 * np.linalg.norm(cp_full(X))
    assert abs(O.full_tensor(X) - cp_full(X)).max() <= 1e-13 * abs(cp_full(X)).max()


def test_apply_operator_bruteforce():
    """Operator application (Section 3.2, item ii) equals the explicit Kronecker-product
    operator of eq. (Lz) acting on the full tensor."""
    rng = np.random.default_rng(2)
    dims = [5, 6, 4]
    L = mixed_operator(rng, dims, 6)
    X = W.random_factors(rng, dims, 3)
    Y = O.cp_apply_operator(L, X)
    assert Y[0].shape == (5, 18)
    ref = (full_operator(L) @ cp_full(X).reshape(-1)).reshape(dims)
    assert rel(cp_full(Y), ref) <= 1e-13


def test_central_difference_fourier_symbol():
    """Periodic central difference on sin(m x): D sin(m x) = sin(m h)/h cos(m x) exactly."""
    n = 32
    x = W.grid(n)
    h = 2 * np.pi / n
    D = O.op_matrix(W.op_central_diff(n))
    for m in (1, 3, 7, 15):
        assert np.allclose(D @ np.sin(m * x), np.sin(m * h) / h * np.cos(m * x), atol=1e-12, rtol=0)


def test_op_matrix_matches_entrywise_definition():
    rng = np.random.default_rng(3)
    for op in (W.op_central_diff(7), W.op_diag(rng.standard_normal(7)), W.op_identity(7),
               W.op_rank1(rng.standard_normal(7), rng.standard_normal(7)),
               W.Op1D("band", 7, rng.standard_normal((5, 7)), 2), W.op_central_diff(2)):
        assert np.array_equal(O.op_matrix(op).toarray(), dense_op(op))


# ------------------------------------------------------------- one dimension update

@pytest.mark.parametrize("dims,r,q", [([8, 8, 8], 3, 0), ([8, 7, 6], 3, 1), ([8, 7, 6], 3, 2),
                                      ([4] * 6, 2, 3)])
def test_update_dim_equals_least_squares(dims, r, q):
    """Each ALS update is the unique minimiser of a convex least-squares problem in U_q
    (eqs. (sequential_min), (ALS2)): compare with dense lstsq on the explicitly formed
    A J_q on the full grid, for operators mixing band, diagonal and rank-1 factors and a
    B-side operator of several terms (eq. (MR))."""
    rng = np.random.default_rng(10 + q + len(dims))
    A = mixed_operator(rng, dims, 5)
    B = mixed_operator(rng, dims, 3)
    U = W.random_factors(rng, dims, r)
    V = W.random_factors(rng, dims, r + 1)
    Unew, delta = O.update_dim(A, B, [u.copy() for u in U], V, q, eps_reg=0.0)
    ref = lstsq_update(A, B, U, V, q)
    assert rel(Unew, ref) <= 1e-10
    # ||Delta f_q|| is the norm of the change of the represented tensor
    U2 = [u.copy() for u in U]
    U2[q] = Unew
    assert abs(delta - np.linalg.norm(cp_full(U2) - cp_full(U))) <= 1e-10 * np.linalg.norm(cp_full(U))


def test_update_dim_with_source_equals_least_squares():
    """Affine source term (eq. (CNFDE1), residual eq. (rRr) with the sign reading
    R = A f_{n+1} - B f_n - dt C)."""
    rng = np.random.default_rng(21)
    dims = [6, 5, 4]
    A = mixed_operator(rng, dims, 4)
    B = mixed_operator(rng, dims, 2)
    U = W.random_factors(rng, dims, 2)
    V = W.random_factors(rng, dims, 2)
    C = W.random_factors(rng, dims, 1)
    Unew, _ = O.update_dim(A, B, [u.copy() for u in U], V, 1, eps_reg=0.0, source=C)
    assert rel(Unew, lstsq_update(A, B, U, V, 1, source=C)) <= 1e-10


# ------------------------------------------------------------------- whole steps

def test_step_d1_is_banded_solve():
    """d = 1, r = 1: the step is the textbook 1-D periodic Crank-Nicolson solve
    u = A^{-1} B v (eq. (CNFDE))."""
    p = W.advection_cn_constant(seed=3, d=1, n=64, dt=0.05, ic_rank=1, cap=1)
    U, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=1e-14, max_sweeps=5, eps_reg=0.0)
    Ad, Bd = full_operator(p.A), full_operator(p.B)
    ref = np.linalg.solve(Ad, Bd @ p.f0[0][:, 0])
    assert rel(U[0][:, 0], ref) <= 1e-12
    assert rep["flags"] == 0


def test_step_d2_full_rank_is_exact():
    """d = 2 with r = n: a rank-n CP tensor represents every n x n matrix, so the minimum
    of eq. (resnorm) is zero and the step equals the dense full-grid solve."""
    n = 12
    rng = np.random.default_rng(4)
    A = mixed_operator(rng, [n, n], 4, with_rank1=False)
    B = mixed_operator(rng, [n, n], 3, with_rank1=False)
    V = W.random_factors(rng, [n, n], 3)
    guess = W.random_factors(rng, [n, n], n)
    U, rep = O.als_step(A, B, V, guess, tol=1e-13, max_sweeps=50, eps_reg=0.0)
    ref = full_step(A, B, cp_full(V))
    assert rel(cp_full(U), ref) <= 1e-9
    assert O.residual(A, B, U, V) <= 1e-9


def test_single_direction_advection_preserves_rank():
    """Velocity along x_1 only: the CN operator is Cayley(a_1 D) on dimension 1 times the
    identity elsewhere, so every column's first factor evolves by the 1-D CN solve and
    the rank is preserved exactly."""
    p = W.advection_cn_constant(seed=5, d=4, n=16, dt=0.05, ic_rank=2, cap=2,
                                velocity=np.array([0.8, 0.0, 0.0, 0.0]))
    U, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=1e-13, max_sweeps=100, eps_reg=0.0)
    n = 16
    D = dense_op(W.op_central_diff(n))
    th = 0.5 * 0.05 * 0.8
    cay = np.linalg.solve(np.eye(n) + th * D, np.eye(n) - th * D)
    ref = [cay @ p.f0[0]] + [u.copy() for u in p.f0[1:]]
    assert rel(cp_full(U), cp_full(ref)) <= 1e-12
    # extended-precision Gram expansion: cancellation floor ~ sqrt(1e-19) relative
    assert O.residual(p.A, p.B, U, p.f0) <= 1e-9


def fft_cn_evolution(f, a, dt, steps):
    """Full-grid CN for constant-velocity advection in Fourier space: each mode is
    multiplied by (1 - i th s)/(1 + i th s), s = sum_i a_i sin(2 pi m_i / n)/h."""
    n = f.shape[0]
    h = 2 * np.pi / n
    m = np.fft.fftfreq(n) * n
    sig = 0
    for i, ai in enumerate(a):
        shape = [1] * f.ndim
        shape[i] = n
        sig = sig + ai * (np.sin(2 * np.pi * m / n) / h).reshape(shape)
    th = 0.5 * dt
    G = (1 - 1j * th * sig) / (1 + 1j * th * sig)
    return np.real(np.fft.ifftn(np.fft.fftn(f) * G ** steps))


def test_cn_steps_track_fft_evolution_and_conserve_mass_and_norm():
    """Constant-velocity advection (the constant special case of eq. (PDE-advR)): CP-ALS
    with a fixed rank follows the full-grid CN evolution up to its rank-truncation
    error, conserves mass (1^T D = 0) and the L2 norm (D skew, so CN is unitary) up to
    the ALS residual."""
    p = W.advection_cn_constant(seed=6, d=3, n=16, dt=0.02, ic_rank=2, cap=3, n_steps=5)
    traj, reps = O.run(p, 5, max_sweeps=300, eps_reg=0.0)
    f0 = cp_full(p.f0)
    ref = fft_cn_evolution(f0, p.meta["velocity"], 0.02, 5)
    assert np.allclose(ref, full_step_n(p, f0, 5), atol=1e-12)
    err = rel(cp_full(traj[-1]), ref)
    assert err <= 1e-6, err
    mass0 = f0.sum()
    assert abs(cp_full(traj[-1]).sum() - mass0) <= 1e-7 * abs(mass0)
    assert abs(np.linalg.norm(cp_full(traj[-1])) - np.linalg.norm(f0)) <= 1e-6 * np.linalg.norm(f0)


def full_step_n(p, f, steps):
    for _ in range(steps):
        f = full_step(p.A, p.B, f)
    return f


def test_variable_coefficient_step_matches_full_grid():
    """The 13-term implicit-Euler operator with sin coefficients (d = 3 analogue).  Every
    ALS update minimises the residual (eq. (sequential_min)), so the full-grid residual
    never increases from one update to the next.  A = I + dt*(skew), hence
    ||A^{-1}|| <= 1 and the distance to the exact full-grid solve is bounded by the
    residual; mass is conserved (1^T D = 0, 1^T (S_j (x) D_i) = 0) up to the residual."""
    p = W.advection_ie_variable(seed=7, d=3, n=12, dt=0.05, ic_rank=2, cap=6, n_steps=1)
    Af, Bf = full_operator(p.A), full_operator(p.B)
    g = Bf @ cp_full(p.f0).reshape(-1)
    U = [u.copy() for u in p.guess]
    res = [np.linalg.norm(Af @ cp_full(U).reshape(-1) - g)]
    for sweep in range(30):
        for q in range(3):
            U[q], _ = O.update_dim(p.A, p.B, U, p.f0, q, eps_reg=0.0)
            res.append(np.linalg.norm(Af @ cp_full(U).reshape(-1) - g))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))
    assert res[-1] < 0.05 * res[0]
    exact = np.linalg.solve(Af, g)
    assert np.linalg.norm(cp_full(U).reshape(-1) - exact) <= res[-1] * (1 + 1e-9)
    assert abs(cp_full(U).sum() - exact.sum()) <= np.sqrt(exact.size) * res[-1]
    assert abs(exact.sum() - cp_full(p.f0).sum()) <= 1e-12 * abs(exact.sum())


# ------------------------------------------------------------------ rank truncation

def test_truncate_d2_is_truncated_svd():
    """Rank reduction by ALS (Section 2.1) in d = 2 converges to the Eckart-Young truncated
    SVD from a perturbed SVD start."""
    rng = np.random.default_rng(8)
    n, R, r = 20, 8, 3
    G = W.random_factors(rng, [n, n], R)
    Mfull = cp_full(G)
    Us, s, Vt = np.linalg.svd(Mfull)
    best = (Us[:, :r] * s[:r]) @ Vt[:r]
    start = [Us[:, :r] * s[:r] + 1e-3 * rng.standard_normal((n, r)),
             Vt[:r].T + 1e-3 * rng.standard_normal((n, r))]
    F, rep = O.truncate(G, start, tol=1e-14, max_sweeps=500, eps_reg=0.0)
    assert rel(cp_full(F), best) <= 1e-10


def test_truncate_orthogonal_terms_fixed_point():
    """A completely orthogonal CP tensor: its top-r terms are an ALS fixed point."""
    rng = np.random.default_rng(9)
    n, d, R, r = 10, 3, 5, 3
    Q = [np.linalg.qr(rng.standard_normal((n, R)))[0] for _ in range(d)]
    w = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    G = [Q[0] * w] + Q[1:]
    start = [u[:, :r].copy() for u in G]
    F, rep = O.truncate(G, start, tol=1e-14, max_sweeps=5, eps_reg=0.0)
    assert rel(cp_full(F), cp_full(start)) <= 1e-12
    assert rep["sweeps"] == 1


# ---------------------------------------------------------------- kinetic model

def small_kinetic(n=8, dt=0.05, nu=1.0):
    return W.kinetic_cn(seed=0, n=n, nu=nu, dt=dt, field_rank=1, cap=2, n_steps=1)


def test_kinetic_maxwellian_is_fixed_point():
    """f = M(v) (constant in x) is a steady state (v . grad_x M = 0 and the relaxation
    M rho[M] - M vanishes), the analogue of the paper's stable fixed point at f_eq
    (Section 4.2, steady state)."""
    p = small_kinetic()
    m = p.meta["maxwellian"]
    n = m.shape[0]
    f = [np.ones((n, 1)) for _ in range(3)] + [m[:, None].copy() for _ in range(3)]
    U, rep = O.als_step(p.A, p.B, f, f, tol=1e-13, max_sweeps=5, eps_reg=0.0)
    assert rel(cp_full(U), cp_full(f)) <= 1e-12
    assert rep["sweeps"] == 1


@pytest.mark.parametrize("n", [4, 16])
def test_kinetic_relaxation_rate(n):
    """Space-homogeneous perturbation with zero mass decays by (1 - nu dt/2)/(1 + nu dt/2)
    per CN step: the discrete analogue of exponential relaxation at rate nu (Section 4.2,
    relaxation experiment)."""
    dt, nu = 0.05, 1.0
    p = small_kinetic(n=n, dt=dt, nu=nu)
    m = p.meta["maxwellian"]
    v = W.grid(n, -5.0, 5.0)
    g1 = v - (m * v).sum() / m.sum()      # zero mean under the Maxwellian weight
    eps = 0.2
    f = [np.ones((n, 2)) for _ in range(3)] + [np.stack([m, m], 1) for _ in range(3)]
    f[3][:, 1] = m * g1 * eps
    # the two columns coincide in five dimensions, so the factor problem is singular (the
    # tensor is not): a tiny shift picks the minimum-norm factors
    U, rep = O.als_step(p.A, p.B, f, f, tol=1e-14, max_sweeps=50, eps_reg=1e-14)
    fac = (1 - 0.5 * nu * dt) / (1 + 0.5 * nu * dt)
    ref = [u.copy() for u in f]
    ref[3][:, 1] *= fac
    assert rel(cp_full(U), cp_full(ref)) <= 1e-10
    if n <= 4:
        full = full_step(p.A, p.B, cp_full(f))
        assert rel(full, cp_full(ref)) <= 1e-12


def test_kinetic_mass_conservation():
    """Transport and Maxwellian relaxation both conserve mass: the full-grid CN step
    conserves it exactly and CP-ALS up to its residual."""
    p = W.kinetic_cn(seed=1, n=4, dt=0.05, field_rank=2, cap=4, n_steps=1)
    U, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=1e-12, max_sweeps=300, eps_reg=0.0)
    hx = 2 * np.pi / 4
    w = p.meta["w"]
    def mass(f):
        return np.einsum("abcdef,d,e,f->", f, w, w, w) * hx ** 3
    f0 = cp_full(p.f0)
    assert abs(mass(full_step(p.A, p.B, f0)) - mass(f0)) <= 1e-13 * abs(mass(f0))
    assert abs(mass(cp_full(U)) - mass(f0)) <= 1e-7 * abs(mass(f0))


# --------------------------------------------------------------- residual helpers

def test_residual_and_distance_match_full_grid():
    rng = np.random.default_rng(11)
    dims = [5, 4, 6]
    A = mixed_operator(rng, dims, 4)
    B = mixed_operator(rng, dims, 2)
    U = W.random_factors(rng, dims, 3)
    V = W.random_factors(rng, dims, 2)
    R = (full_operator(A) @ cp_full(U).reshape(-1)) - (full_operator(B) @ cp_full(V).reshape(-1))
    g = full_operator(B) @ cp_full(V).reshape(-1)
    assert abs(O.residual(A, B, U, V) - np.linalg.norm(R) / np.linalg.norm(g)) <= 1e-12
    assert abs(O.rel_distance(U, V) - rel(cp_full(U), cp_full(V))) <= 1e-12


# ---------------------------------------------------------------- linearised BGK (fixed f_eq)

def bgk_gamma(p):
    nu, dt = p.meta["nu"], p.dt
    return (1.0 - 0.5 * nu * dt) / (1.0 + 0.5 * nu * dt)


def cp_mass(U):
    """Sum of the represented tensor over the grid (products of the factors' column sums)."""
    return float(np.sum(np.prod([u.sum(axis=0) for u in U], axis=0)))


def test_bgk_equilibrium_is_fixed_point():
    """f = f_eq = M(v) (x) 1_x: v.grad_x f_eq = 0 and the relaxation term vanishes, so the
    forced Crank-Nicolson step A f = B f_eq + dt nu f_eq has f_eq as its exact solution."""
    p = W.bgk_linear_cn(seed=0, n=8, cap=1)
    feq = p.meta["feq"]
    U, rep = O.als_step(p.A, p.B, feq, feq, tol=1e-14, max_sweeps=50, eps_reg=0.0, source=p.meta["source"])
    assert O.rel_distance(U, feq) <= 1e-12


def test_bgk_x_independent_relaxation_is_exact():
    """An x-independent perturbation h(v) of f_eq is not transported, and f - f_eq decays by
    exactly gamma = (1 - nu dt/2) / (1 + nu dt/2) per step (the relaxation experiment of
    Section 4.2): after N steps f_N = f_eq + gamma^N (f_0 - f_eq)."""
    p = W.bgk_linear_cn(seed=3, n=8, field_rank=1, cap=2, dt=0.05, x_dependent=False)
    g = bgk_gamma(p)
    U = [u.copy() for u in p.f0]
    for _ in range(4):
        U, _ = O.als_step(p.A, p.B, U, U, tol=1e-14, max_sweeps=100, eps_reg=0.0, source=p.meta["source"])
    pert = [u[:, 1:].copy() for u in p.f0]
    pert[0] *= g ** 4
    expect = [np.concatenate([f, q], axis=1) for f, q in zip(p.meta["feq"], pert)]
    assert O.rel_distance(U, expect) <= 1e-11


def test_bgk_mass_relaxes_at_the_exact_rate():
    """Transport conserves the grid sum (periodic differences), so the full-grid step gives
    M_{n+1} - M_eq = gamma (M_n - M_eq) for any f; the CP-ALS steps follow it to the ALS
    residual (an x-dependent rank-4 state, rank cap 8, three steps)."""
    p = W.bgk_linear_cn(seed=5, n=8, field_rank=3, cap=8, dt=0.05, eps=0.3)
    g = bgk_gamma(p)
    Meq = cp_mass(p.meta["feq"])
    M0 = cp_mass(p.f0)
    U, G = p.f0, p.guess
    for s in range(3):
        U, rep = O.als_step(p.A, p.B, U, G, tol=1e-12, max_sweeps=200, source=p.meta["source"])
        G = U
        pred = Meq + g ** (s + 1) * (M0 - Meq)
        assert abs(cp_mass(U) - pred) <= 1e-9 * abs(Meq)


# ---------------------------------------------------------------- linear-velocity advection

def test_spiral_operator_is_sixth_order_accurate():
    """The separable generator of eq. (PDE-advR) in the ordering of Table (tab:ordering0),
    applied to the separable f0 = exp(-|z|^2) (N = 2), against the exact
    -sum_{j,k} C_jk z_k df/dz_j on the grid: the error falls by 2^6 when h halves (sixth-order
    central differences), and the term table's signs and dimension placement are right."""
    errs = []
    for n in (48, 96):
        x = W.grid(n, -6.0, 6.0)
        C = W.spiral_matrix(3, 2)
        L = W.spiral_generator(C, x)
        f0 = [np.exp(-x * x)[:, None] for _ in range(2)]
        Lf = cp_full(O.cp_apply_operator(L, f0))
        X, Y = np.meshgrid(x, x, indexing="ij")
        f = np.exp(-X * X - Y * Y)
        fx, fy = -2 * X * f, -2 * Y * f
        exact = -((C[0, 0] * X + C[0, 1] * Y) * fx + (C[1, 0] * X + C[1, 1] * Y) * fy)
        errs.append(np.abs(Lf - exact).max() / np.abs(exact).max())
    assert errs[1] < 1e-4
    assert 45 < errs[0] / errs[1] < 90, errs


def test_spiral_exact_solution_satisfies_the_pde():
    """f(z, t) = f0(exp(-tC) z) (eq. solutionF): its time derivative, by central differences
    in t, equals -sum_{j,k} C_jk z_k df/dz_j at random points."""
    rng = np.random.default_rng(2)
    C = W.spiral_matrix(1, 3)
    for _ in range(5):
        z = rng.uniform(-1, 1, 3)
        t, e = 0.3, 1e-5
        ft = (W.spiral_exact(C, z, t + e) - W.spiral_exact(C, z, t - e)) / (2 * e)
        grad = np.array([(W.spiral_exact(C, z + e * np.eye(3)[j], t) - W.spiral_exact(C, z - e * np.eye(3)[j], t)) / (2 * e)
                         for j in range(3)])
        assert abs(ft + (C @ z) @ grad) <= 1e-7


# ---------------------------------------------------------------- damped Jacobi sweeps (App. B)

def test_jacobi_d1_is_damped_fixed_point_iteration():
    """d = 1: the one update is the exact minimiser U*, so damped Jacobi sweeps give
    U_s = U* + (1 - w)^s (U_0 - U*) exactly (checked after three sweeps, w = 1/4)."""
    p = W.advection_cn_constant(seed=0, d=1, n=24, ic_rank=1, cap=1)
    Ustar, _ = O.als_step(p.A, p.B, p.f0, p.guess, tol=0.0, max_sweeps=1, eps_reg=0.0)
    U0 = p.guess[0]
    U3, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=0.0, max_sweeps=3, eps_reg=0.0, sweep="jacobi", damping=0.25)
    expect = Ustar[0] + 0.75 ** 3 * (U0 - Ustar[0])
    assert np.abs(U3[0] - expect).max() <= 1e-13 * np.abs(expect).max()


def test_jacobi_single_direction_advection_is_exact():
    """Velocity along x_1 only, rank-2 state: the exact step keeps the rank (every column's
    first factor evolves by the 1-D Crank-Nicolson solve), and the damped Jacobi sweeps
    converge to that solution as the Gauss-Seidel ones do."""
    p = W.advection_cn_constant(seed=5, d=3, n=16, dt=0.05, ic_rank=2, cap=2,
                                velocity=np.array([0.8, 0.0, 0.0]))
    U, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=1e-13, max_sweeps=2000, eps_reg=0.0, sweep="jacobi")
    n = 16
    D = dense_op(W.op_central_diff(n))
    th = 0.5 * 0.05 * 0.8
    cay = np.linalg.solve(np.eye(n) + th * D, np.eye(n) - th * D)
    ref = [cay @ p.f0[0]] + [u.copy() for u in p.f0[1:]]
    assert rep["flags"] == 0
    assert rel(cp_full(U), cp_full(ref)) <= 1e-11
