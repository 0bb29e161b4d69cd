"""GPU parity of the step residual (double-double), adaptive rank and the caller-owned
workspace, through the C ABI, against the FP64 oracle on the same seeded inputs.

Adaptive rank is checked by replay: the oracle is run with replay_rank = the rank the GPU
grew to (report.grown_rank), so both take the same growth decisions; the GPU's decisions are
then checked against the oracle's logged residuals (every growth had rho > tau, the last
rho <= tau unless the cap was reached)."""
import numpy as np
import pytest

from gpu_util import dev, host, log
from oracle import cpals_oracle as O
from paper_1803_10270_amd import binding as B
from paper_1803_10270_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def handle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = B.Handle()
    yield h
    h.close()


def padded(U, cap):
    """Panels holding cap columns, the first U's."""
    return [np.concatenate([u, np.zeros((u.shape[0], cap - u.shape[1]))], axis=1) for u in U]


def adaptive_opts(cap, tau, **kw):
    o = B.default_opts(rank_mode=B.RANK_ADAPTIVE, rank_cap=cap, tau_rank=tau, **kw)
    return o


# ------------------------------------------------------------------ residual in double-double

def test_residual_resolves_a_known_tiny_residual(handle):
    """A = B = I and f = g + delta with delta one term of relative size 1e-12: the residual is
    exactly ||delta|| / ||g||, far below the ~1e-8 floor of a float64 Gram expansion."""
    log("residual tiny")
    rng = np.random.default_rng(31)
    dims = [24, 40, 16, 32]
    G = W.random_factors(rng, dims, 5)
    D = W.random_factors(rng, dims, 1)
    gnorm, dnorm = O.cp_norm(G), O.cp_norm(D)
    D[0] *= 1e-12 * gnorm / dnorm
    F = [np.concatenate([g, dd], axis=1) for g, dd in zip(G, D)]
    I = W.identity_operator(dims)
    exact = float(np.prod([np.linalg.norm(x[:, 0]) for x in D])) / gnorm
    got = B.cp_residual(handle, I, I, dev(F), dev(G))
    ora = O.residual(I, I, F, G)
    log("rho: gpu %.12e oracle %.12e exact %.12e" % (got, ora, exact))
    assert abs(got - exact) <= 1e-6 * exact
    assert abs(got - ora) <= 1e-6 * exact


@pytest.mark.parametrize("case", ["guess", "converged"])
def test_residual_matches_oracle_variable_advection(handle, case):
    """The 13-term implicit-Euler operator (d = 4, n = 32, rank 6): an O(1e-3) residual of the
    padded guess and the small residual of a converged step agree with the oracle's
    double-double value to 1e-7 relative."""
    log("residual", case)
    p = W.advection_ie_variable(seed=2, d=4, n=32, ic_rank=3, cap=6)
    U = p.guess
    if case == "converged":
        U, _ = O.als_step(p.A, p.B, p.f0, p.guess, tol=1e-10, max_sweeps=60)
    got = B.cp_residual(handle, p.A, p.B, dev(U), dev(p.f0))
    ora = O.residual(p.A, p.B, U, p.f0)
    log("rho: gpu %.12e oracle %.12e" % (got, ora))
    assert abs(got - ora) <= 1e-7 * ora


def test_report_residual_in_fixed_rank(handle):
    """opts.report_residual = 1 puts the step residual of every step into the report; it equals
    cp_residual of the result."""
    log("report residual")
    p = W.advection_ie_variable(seed=4, d=4, n=32, ic_rank=2, cap=4, n_steps=2)
    V, U = dev(p.f0), dev(p.guess)
    reps = B.cp_als_run(handle, p.A, p.B, V, U, 2, B.default_opts(tol=1e-9, max_sweeps=80, report_residual=1))
    log(reps)
    U1 = [u.clone() for u in U]
    # the residual of step 2 is that of U against the result of step 1: recompute step 1
    V2, Ua = dev(p.f0), dev(p.guess)
    B.cp_als_run(handle, p.A, p.B, V2, Ua, 1, B.default_opts(tol=1e-9, max_sweeps=80, report_residual=1))
    rho2 = B.cp_residual(handle, p.A, p.B, U1, Ua)
    assert reps[1]["final_rank"] == 4 and reps[1]["grown_rank"] == 4
    assert abs(reps[1]["rel_residual"] - rho2) <= 1e-9 * rho2
    assert reps[0]["rel_residual"] > 0.0


# ------------------------------------------------------------------ adaptive rank

def check_decisions(rep_gpu, log_ora, tau, cap):
    """The GPU's growth decisions are those the oracle's residuals call for (ties within 1e-6
    relative of tau are not decided)."""
    ranks = [r for r, _ in log_ora]
    assert ranks[-1] == rep_gpu["grown_rank"]
    for r, rho in log_ora[:-1]:
        assert rho > tau * (1 - 1e-6), (r, rho, tau)
    r_last, rho_last = log_ora[-1]
    assert rho_last <= tau * (1 + 1e-6) or r_last == cap


@pytest.mark.parametrize("tau", [1.5e-4, 0.0])
def test_adaptive_step_matches_oracle_replay(handle, tau):
    """Variable-coefficient advection (d = 3, n = 16) from its rank-2 initial state, 20 sweeps
    per solve (the oracle's residuals: 2.1e-4, 9.8e-5, 4.1e-5 at ranks 2, 3, 4): tau = 1.5e-4
    grows to rank 3; tau = 0 grows to the cap 4.  The oracle replays the
    GPU's grown rank; final rank, growth terms and result agree."""
    log("adaptive replay tau", tau)
    p = W.advection_ie_variable(seed=3, d=3, n=16, ic_rank=2, cap=4)
    cap = 4
    g = dev(padded(p.f0, cap))
    o = adaptive_opts(cap, tau, tol=0.0, max_sweeps=20, seed=7)
    rep = B.cp_als_step(handle, p.A, p.B, dev(p.f0), g, o, rank=2)
    log(rep)
    Uo, ro = O.adaptive_step(p.A, p.B, p.f0, p.f0, cap=cap, tau=tau, tol=0.0, max_sweeps=20, seed=7,
                             replay_rank=rep["grown_rank"])
    log("oracle", ro["log"], ro["final_rank"])
    check_decisions(rep, ro["log"], tau, cap)
    assert rep["final_rank"] == ro["final_rank"]
    assert rep["sweeps"] == ro["sweeps"]
    got = [u[:, :rep["final_rank"]] for u in host(g)]
    dist = O.rel_distance(got, Uo)
    log("distance %.3e, rho gpu %.6e oracle %.6e" % (dist, rep["rel_residual"], ro["rel_residual"]))
    assert dist <= TOL
    # the applied panels are rounded in FP64 on both sides: rho agrees to ~1e-15 absolute
    assert abs(rep["rel_residual"] - ro["rel_residual"]) <= 1e-7 * ro["rel_residual"] + 1e-14
    if tau > 0.0:
        assert rep["grown_rank"] == 3


def test_adaptive_truncation_grows_to_exact_rank(handle):
    """A = B = I (rank reduction of a rank-3 tensor from a rank-1 start): the rank grows to
    exactly 3, the residual falls to the rounding level and the represented tensor equals g."""
    log("adaptive truncation")
    rng = np.random.default_rng(21)
    dims = [16, 32, 16]
    G = W.random_factors(rng, dims, 3)
    I = W.identity_operator(dims)
    start = [gk[:, :1] + 0.1 * rng.standard_normal((gk.shape[0], 1)) for gk in G]
    cap = 6
    f = dev(padded(start, cap))
    o = adaptive_opts(cap, 1e-10, tol=1e-13, max_sweeps=2000, eps_reg=1e-14, seed=11)
    rep = B.cp_als_step(handle, I, I, dev(G), f, o, rank=1)
    log(rep)
    assert rep["final_rank"] == 3 and rep["grown_rank"] == 3
    assert rep["rel_residual"] <= 1e-12
    got = [u[:, :3] for u in host(f)]
    assert O.rel_distance(got, G) <= 1e-12


def test_adaptive_run_two_steps_matches_oracle(handle):
    """Two adaptive steps in one launch (step 2 starts from f_1 at its own rank) against the
    oracle's adaptive time loop replaying the GPU's per-step ranks."""
    log("adaptive run")
    p = W.advection_ie_variable(seed=3, d=3, n=16, ic_rank=2, cap=4)
    cap = 4
    V, U = dev(padded(p.f0, cap)), dev(padded(p.f0, cap))
    o = adaptive_opts(cap, 1.5e-4, tol=0.0, max_sweeps=15, seed=2)
    reps = B.cp_als_run(handle, p.A, p.B, V, U, 2, o, rank=2, f_init_rank=2)
    log(reps)
    traj, ro = O.run_adaptive(p.A, p.B, p.f0, cap=cap, tau=1.5e-4, n_steps=2, tol=0.0, max_sweeps=15, seed=2,
                              replay_ranks=[r["grown_rank"] for r in reps])
    for s in range(2):
        check_decisions(reps[s], ro[s]["log"], 1.5e-4, cap)
        assert reps[s]["final_rank"] == ro[s]["final_rank"]
    got = [u[:, :reps[1]["final_rank"]] for u in host(U)]
    dist = O.rel_distance(got, traj[1])
    log("distance %.3e" % dist)
    assert dist <= TOL


def test_adaptive_batched_matches_single(handle):
    """Three problems with their own caps and tolerances in one batched launch: every result
    and report equals the single-problem call bit for bit (both run one workgroup)."""
    log("adaptive batched")
    probs = [W.advection_ie_constant(seed=50 + i, d=3 + (i % 2), n=16 * (i + 1), cap=4, ic_rank=2)
             for i in range(3)]
    caps = [3, 4, 5]
    taus = [6e-7, 1e-6, 0.0]   # grow to 3, to the cap 4, to the cap 5
    opts = [adaptive_opts(c, t, tol=0.0, max_sweeps=10, seed=5) for c, t in zip(caps, taus)]
    fo = [dev(padded(p.f0, c)) for p, c in zip(probs, caps)]
    reps = B.cp_als_run_batched(handle, [p.A for p in probs], [p.B for p in probs], [dev(p.f0) for p in probs],
                                fo, 1, opts, ranks=[2, 2, 2])
    assert [r[0]["grown_rank"] for r in reps] == [3, 4, 5]
    for i, p in enumerate(probs):
        g = dev(padded(p.f0, caps[i]))
        rep = B.cp_als_step(handle, p.A, p.B, dev(p.f0), g, opts[i], rank=2)
        log(i, rep, reps[i][0])
        assert rep == reps[i][0]
        fr = rep["final_rank"]
        for a, b in zip(host(g), host(fo[i])):
            assert np.array_equal(a[:, :fr], b[:, :fr])


# ------------------------------------------------------------------ caller-owned workspace

def test_caller_workspace_matches_library_workspace(handle):
    """With the exact workspace the size queries give, every call runs in the caller's buffer
    and gives bit-identical results to the library-owned workspace; one byte less is
    CP_ERR_WORKSPACE before anything is launched."""
    import torch
    log("workspace")
    p = W.advection_cn_constant(seed=5, d=4, n=32, cap=4)
    rng = np.random.default_rng(3)
    src = [0.01 * u for u in W.random_factors(rng, p.A.dims(), 2)]
    h2 = B.Handle()
    o = B.default_opts(tol=1e-10, max_sweeps=50)
    need = max(B.workspace_size_step(h2, p.A, p.B, dev(p.f0), dev(p.guess), 1, o),
               B.workspace_size_step(h2, p.A, p.B, dev(p.f0), dev(p.guess), 1, o, source=dev(src)),
               B.workspace_size_inner(h2, dev(p.guess), dev(p.f0)),
               B.workspace_size_apply(h2, p.A, dev(p.f0)))
    log("workspace bytes", need)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h2.set_workspace(ws)
    results = []
    for h in (handle, h2):
        g1, g2 = dev(p.guess), dev(p.guess)
        r1 = B.cp_als_step(h, p.A, p.B, dev(p.f0), g1, o)
        r2 = B.cp_als_step_source(h, p.A, p.B, dev(p.f0), dev(src), g2, o)
        rho = B.cp_residual(h, p.A, p.B, g1, dev(p.f0))
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.cp_inner(h, g1, dev(p.f0), out)
        y = [torch.empty((p.A.n_terms * 4, n), dtype=torch.float64, device="cuda") for n in p.A.dims()]
        B.cp_apply_operator(h, p.A, g1, y)
        results.append((r1, r2, rho, float(out.item()), host(g1), host(g2), host(y)))
    a, b = results
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
    for xs, ys in zip(a[4:], b[4:]):
        for x, y in zip(xs, ys):
            assert np.array_equal(x, y)
    need_src = B.workspace_size_step(h2, p.A, p.B, dev(p.f0), dev(p.guess), 1, o, source=dev(src))
    small = torch.empty(need_src - 256, dtype=torch.uint8, device="cuda")
    h3 = B.Handle()
    h3.set_workspace(small)
    g3 = dev(p.guess)
    before = host(g3)
    with pytest.raises(B.CpalsError) as ei:
        B.cp_als_step_source(h3, p.A, p.B, dev(p.f0), dev(src), g3, o)
    assert ei.value.status == B.CP_ERR_WORKSPACE
    for x, y in zip(before, host(g3)):
        assert np.array_equal(x, y)
    h3.close()
    h2.close()
