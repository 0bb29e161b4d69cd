"""GPU tests of the linearised BGK equation with a fixed equilibrium (Section 4.2: the forced
Crank-Nicolson step A f_{n+1} = B f_n + dt nu f_eq through cp_als_step_source), against the
closed forms the paper's experiments rest on -- the equilibrium is a fixed point (steady
state), an x-independent perturbation decays by exactly gamma = (1 - nu dt/2)/(1 + nu dt/2)
per step (relaxation), and the grid mass relaxes to the equilibrium mass at that rate
(moments) -- and against the FP64 oracle on the same steps."""
import numpy as np
import pytest

from gpu_util import dev, host, log
from oracle import cpals_oracle as O
from paper_1803_10270_amd import binding as B
from paper_1803_10270_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = B.Handle()
    yield h
    h.close()


def gamma(p):
    nu, dt = p.meta["nu"], p.dt
    return (1.0 - 0.5 * nu * dt) / (1.0 + 0.5 * nu * dt)


def cp_mass(U):
    return float(np.sum(np.prod([u.sum(axis=0) for u in U], axis=0)))


def test_bgk_equilibrium_is_a_fixed_point(handle):
    log("bgk equilibrium")
    p = W.bgk_linear_cn(seed=0, n=32, cap=1)
    feq = p.meta["feq"]
    g = dev(feq)
    rep = B.cp_als_step_source(handle, p.A, p.B, dev(feq), dev(p.meta["source"]), g,
                               B.default_opts(tol=1e-14, max_sweeps=50, eps_reg=0.0))
    dist = O.rel_distance(host(g), feq)
    log(rep, "distance to f_eq %.3e" % dist)
    assert dist <= 1e-12


def test_bgk_x_independent_relaxation(handle):
    log("bgk relaxation")
    p = W.bgk_linear_cn(seed=3, n=32, field_rank=1, cap=2, dt=0.05, x_dependent=False)
    g = gamma(p)
    U = dev(p.f0)
    src = dev(p.meta["source"])
    opts = B.default_opts(tol=1e-14, max_sweeps=100, eps_reg=0.0)
    for _ in range(6):
        nxt = [u.clone() for u in U]
        B.cp_als_step_source(handle, p.A, p.B, U, src, nxt, opts)
        U = nxt
    pert = [u[:, 1:].copy() for u in p.f0]
    pert[0] *= g ** 6
    expect = [np.concatenate([f, q], axis=1) for f, q in zip(p.meta["feq"], pert)]
    dist = O.rel_distance(host(U), expect)
    log("distance to f_eq + gamma^6 (f_0 - f_eq): %.3e" % dist)
    assert dist <= 1e-11


def test_bgk_mass_relaxation_and_oracle_parity(handle):
    """An x-dependent rank-4 state (n = 16, rank cap 8), three forced steps at tol 1e-11: the
    mass follows M_eq + gamma^n (M_0 - M_eq) to the ALS residual, and each step equals the
    oracle's forced step from the same state."""
    log("bgk mass")
    p = W.bgk_linear_cn(seed=5, n=16, field_rank=3, cap=8, dt=0.05, eps=0.3)
    g = gamma(p)
    Meq, M0 = cp_mass(p.meta["feq"]), cp_mass(p.f0)
    src = p.meta["source"]
    V, G = p.f0, p.guess
    opts = B.default_opts(tol=1e-11, max_sweeps=300)
    for s in range(3):
        U = dev(G)
        rep = B.cp_als_step_source(handle, p.A, p.B, dev(V), dev(src), U, opts)
        Ug = host(U)
        Uo, ro = O.als_step(p.A, p.B, V, G, tol=1e-11, max_sweeps=300, source=src)
        pred = Meq + g ** (s + 1) * (M0 - Meq)
        dist = O.rel_distance(Ug, Uo)
        log("step %d: sweeps gpu %d oracle %d, distance %.3e, mass error %.3e" % (
            s + 1, rep["sweeps"], ro["sweeps"], dist, abs(cp_mass(Ug) - pred) / abs(Meq)))
        assert rep["flags"] == 0 and rep["sweeps"] == ro["sweeps"]
        assert dist <= 1e-10
        assert abs(cp_mass(Ug) - pred) <= 1e-9 * abs(Meq)
        V, G = Ug, Ug
