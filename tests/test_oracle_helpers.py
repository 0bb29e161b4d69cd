"""Pins of the oracle's helper routines, each against a computation that does not share its
formula: the full tensor reconstructed by einsum, explicit Khatri-Rao products, dense
Kronecker operators and closed forms."""
import numpy as np

from bruteforce import cp_full, full_operator
from oracle import cpals_oracle as O
from paper_1803_10270_amd import workloads as W


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def khatri_rao(mats):
    """Columns l of the result are the Kronecker products of the columns l of `mats`."""
    out = mats[0]
    for m in mats[1:]:
        out = np.einsum("il,jl->ijl", out, m).reshape(-1, m.shape[1])
    return out


def test_balance_keeps_the_tensor_and_equalises_norms():
    """Balancing (the column scaling after every sweep) leaves the represented tensor
    unchanged, gives every factor of a column the geometric mean of its norms, keeps signs,
    and leaves a column with a zero factor alone."""
    rng = np.random.default_rng(3)
    U = W.random_factors(rng, [5, 6, 7], 4)
    U[1][:, 2] = 0.0
    before = cp_full(U)
    norms0 = np.array([[np.linalg.norm(u[:, l]) for l in range(4)] for u in U])
    signs0 = [np.sign(u) for u in U]
    V = [u.copy() for u in U]
    O.balance(V)
    assert rel(cp_full(V), before) <= 1e-14
    for l in (0, 1, 3):
        g = np.prod(norms0[:, l]) ** (1.0 / 3.0)
        for k in range(3):
            assert abs(np.linalg.norm(V[k][:, l]) - g) <= 1e-13 * g
    for k in range(3):
        assert np.array_equal(np.sign(V[k]), signs0[k])
        assert np.array_equal(V[k][:, 2], U[k][:, 2])


def test_cp_eval_matches_the_full_tensor():
    rng = np.random.default_rng(4)
    U = W.random_factors(rng, [4, 5, 6], 3)
    F = cp_full(U)
    idx = np.stack([rng.integers(0, n, 50) for n in (4, 5, 6)], axis=1)
    vals = O.cp_eval(U, idx)
    assert np.allclose(vals, F[idx[:, 0], idx[:, 1], idx[:, 2]], rtol=1e-14, atol=1e-14)


def test_sampled_distance_closed_forms():
    """x = 2 y differs from y by exactly y at every point: the sampled relative distance is 1;
    x = y gives 0."""
    rng = np.random.default_rng(5)
    Y = W.random_factors(rng, [8, 9, 10], 2)
    X = [Y[0] * 2.0] + [y.copy() for y in Y[1:]]
    assert abs(O.sampled_rel_distance(X, Y, 4096) - 1.0) <= 1e-14
    assert O.sampled_rel_distance(Y, Y, 4096) == 0.0


def test_identity_hadamard_is_the_khatri_rao_gram():
    """H_q = o_{k != q} U_k^T U_k equals K^T K for the Khatri-Rao product K of the other
    dimensions' factors (the Gram of the tensor's other-dimension columns)."""
    rng = np.random.default_rng(6)
    U = W.random_factors(rng, [4, 5, 6, 3], 3)
    for q in range(4):
        K = khatri_rao([U[k] for k in range(4) if k != q])
        assert rel(O.identity_hadamard(U, q), K.T @ K) <= 1e-13


def test_term_weights_are_rank_one_norms():
    rng = np.random.default_rng(7)
    U = W.random_factors(rng, [4, 5, 6], 3)
    w = O.term_weights(U)
    for l in range(3):
        assert abs(w[l] - np.linalg.norm(cp_full([u[:, l:l + 1] for u in U]))) <= 1e-13 * w[l]


def test_stacked_norm_is_the_full_norm():
    rng = np.random.default_rng(8)
    U = W.random_factors(rng, [5, 4, 6], 5)
    assert abs(O.stacked_norm2(U) - np.sum(cp_full(U) ** 2)) <= 1e-12 * np.sum(cp_full(U) ** 2)


def test_axpby_and_residual_tensor_on_the_full_grid():
    """alpha x + beta y as stacked columns, and the residual tensor g - A f, reconstructed on the
    full grid against the dense Kronecker operator."""
    rng = np.random.default_rng(9)
    dims = [5, 6, 4]
    X = W.random_factors(rng, dims, 2)
    Y = W.random_factors(rng, dims, 3)
    assert rel(cp_full(O.cp_axpby(1.5, X, -0.25, Y)), 1.5 * cp_full(X) - 0.25 * cp_full(Y)) <= 1e-14
    p = W.advection_ie_variable(seed=2, d=3, n=6, ic_rank=2, cap=3, dt=1e-1)
    U = W.random_factors(rng, [6, 6, 6], 3)
    A, Bm = full_operator(p.A), full_operator(p.B)
    ref = (Bm @ cp_full(p.f0).ravel() - A @ cp_full(U).ravel()).reshape(6, 6, 6)
    assert rel(cp_full(O.residual_tensor(p.A, p.B, U, p.f0)), ref) <= 1e-13


def test_reduce_rank_keeps_small_ranks_and_compresses_exact_duplicates():
    """A tensor within the cap is returned as it is; [x, x] (rank 2r, exactly 2 x) reduced to
    rank r is 2 x."""
    rng = np.random.default_rng(10)
    X = W.random_factors(rng, [6, 7, 5], 2)
    same, rep = O.reduce_rank(X, cap=3)
    assert rep["sweeps"] == 0 and all(np.array_equal(a, b) for a, b in zip(same, X))
    G = [np.concatenate([x, x], axis=1) for x in X]
    red, _ = O.reduce_rank(G, cap=2, tol=1e-13, max_sweeps=300, eps_reg=0.0)
    assert rel(cp_full(red), 2.0 * cp_full(X)) <= 1e-8


def test_run_adaptive_replay_and_exact_rank():
    """Single-direction advection keeps a rank-1 initial condition rank 1 (the exact solution
    of every step is rank 1): the adaptive run never grows, every step's residual is at the
    solver's level, and replaying the logged ranks gives the same states."""
    p = W.advection_cn_constant(seed=4, d=3, n=16, ic_rank=1, cap=1, velocity=np.array([1.0, 0.0, 0.0]))
    traj, reps = O.run_adaptive(p.A, p.B, p.f0, cap=4, tau=1e-9, n_steps=3, tol=1e-12, max_sweeps=100)
    assert [r["final_rank"] for r in reps] == [1, 1, 1]
    assert all(r["rel_residual"] <= 1e-9 for r in reps)
    traj2, reps2 = O.run_adaptive(p.A, p.B, p.f0, cap=4, tau=1e-9, n_steps=3, tol=1e-12, max_sweeps=100,
                                  replay_ranks=[r["grown_rank"] for r in reps])
    for a, b in zip(traj, traj2):
        assert rel(cp_full(a), cp_full(b)) <= 1e-14
