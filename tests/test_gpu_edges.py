"""GPU parity at the edges of the supported shapes: one dimension, the maximum number of
dimensions, rank one, the maximum rank, the maximum grid size, grids that are not a multiple
of the 16-row strips, tiny grids; and the shapes the library refuses before any launch
(empty and oversized panels).  Every case runs the step through the C ABI and compares it
with the FP64 oracle on the same seeded inputs (1e-10 relative L2 on the represented tensor;
the full-grid distance where the grid is small, else the double-double CP distance)."""
import numpy as np
import pytest

from gpu_util import dev, host, log, tensor_distance
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


def step_both(handle, p, tol, sweeps):
    Vd, Gd = dev(p.f0), dev(p.guess)
    rep = B.cp_als_step(handle, p.A, p.B, Vd, Gd, B.default_opts(tol=tol, max_sweeps=sweeps))
    Ug = host(Gd)
    Uo, ro = O.als_step(p.A, p.B, p.f0, p.guess, tol=tol, max_sweeps=sweeps)
    return Ug, rep, Uo, ro


def distance(Ug, Uo):
    if np.prod([u.shape[0] for u in Uo]) <= 2_000_000:
        return tensor_distance(Ug, Uo)
    return O.rel_distance(Ug, Uo)


@pytest.mark.parametrize("case", ["d1", "d8", "rank1", "rank64", "n4096", "n20", "n4"])
def test_step_at_shape_limits(handle, case):
    """Steps at the limits (converged where the oracle converges quickly, else a fixed number
    of sweeps): the same sweep count, convergence flag and represented tensor as the oracle."""
    if case == "d1":       # one dimension: the step is one banded solve per sweep
        p = W.advection_ie_constant(seed=11, d=1, n=64, cap=3, ic_rank=2, dt=1e-2)
        tol, sweeps = 1e-10, 50
    elif case == "d8":     # CP_MAX_DIMS dimensions
        p = W.advection_ie_constant(seed=12, d=8, n=16, cap=3, ic_rank=2, dt=1e-2)
        tol, sweeps = 0.0, 3
    elif case == "rank1":
        p = W.advection_ie_constant(seed=13, d=4, n=32, cap=1, ic_rank=1, dt=1e-2)
        tol, sweeps = 1e-10, 50
    elif case == "rank64":  # CP_MAX_RANK columns (a genuinely rank-64 f_n) on an 8-workgroup cluster
        p = W.advection_ie_constant(seed=14, d=3, n=128, cap=2, ic_rank=2, dt=1e-2)
        rng = np.random.default_rng(14)
        p.f0 = W.random_factors(rng, [128] * 3, 64)
        p.guess = [np.array(v) for v in p.f0]
        tol, sweeps = 0.0, 2
    elif case == "n4096":   # CP_MAX_N grid points
        p = W.advection_ie_constant(seed=15, d=2, n=4096, cap=4, ic_rank=2, dt=1e-3)
        tol, sweeps = 0.0, 2
    elif case == "n20":     # not a multiple of the 16-row strips: one workgroup
        p = W.advection_ie_constant(seed=16, d=3, n=20, cap=2, ic_rank=2, dt=1e-2)
        tol, sweeps = 1e-10, 60
    else:                   # a four-point grid: the five-point composite stencils wrap onto it
        p = W.advection_ie_constant(seed=17, d=3, n=4, cap=1, ic_rank=1, dt=1e-2)
        tol, sweeps = 1e-10, 60
    log("edge", case, [u.shape for u in p.guess], "tol", tol, "sweeps", sweeps)
    Ug, rep, Uo, ro = step_both(handle, p, tol, sweeps)
    d = distance(Ug, Uo)
    log("  gpu sweeps", rep["sweeps"], "oracle", ro["sweeps"], "distance", d)
    assert rep["sweeps"] == ro["sweeps"]
    assert (rep["flags"] & B.FLAG_NOT_CONVERGED) == (ro["flags"] & B.FLAG_NOT_CONVERGED)
    # the represented tensor is what is unique: with d = 1 or padded columns the split of a
    # tensor into columns is not, so the panels themselves are not compared
    assert d <= TOL


def test_refused_shapes_launch_nothing(handle):
    """Empty grids, zero rank and grids beyond CP_MAX_N are refused with CP_ERR_SHAPE by the
    host checks, before anything is launched; the handle stays usable."""
    import torch
    log("refused shapes")
    p = W.advection_ie_constant(seed=18, d=2, n=16, cap=2, ic_rank=1)
    Vd = dev(p.f0)
    with pytest.raises(B.CpalsError) as e:   # empty grid in one dimension
        bad = [torch.zeros((2, 16), dtype=torch.float64, device="cuda"),
               torch.zeros((2, 0), dtype=torch.float64, device="cuda")]
        B.cp_als_step(handle, p.A, p.B, Vd, bad)
    assert e.value.status == B.CP_ERR_SHAPE
    with pytest.raises(B.CpalsError) as e:   # zero rank
        zero = [torch.zeros((0, 16), dtype=torch.float64, device="cuda")] * 2
        B.cp_als_step(handle, p.A, p.B, Vd, zero)
    assert e.value.status == B.CP_ERR_SHAPE
    big = W.advection_ie_constant(seed=18, d=2, n=4097, cap=2, ic_rank=1)
    with pytest.raises(B.CpalsError) as e:   # one point beyond CP_MAX_N
        B.cp_als_step(handle, big.A, big.B, dev(big.f0), dev(big.guess))
    assert e.value.status == B.CP_ERR_SHAPE
    with pytest.raises(B.CpalsError) as e:   # inner product of an empty panel
        x = [torch.zeros((1, 0), dtype=torch.float64, device="cuda")] * 2
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        B.cp_inner(handle, x, x, out)
    assert e.value.status == B.CP_ERR_SHAPE
    # the handle still works
    Gd = dev(p.guess)
    rep = B.cp_als_step(handle, p.A, p.B, Vd, Gd, B.default_opts(tol=0.0, max_sweeps=1))
    assert rep["sweeps"] == 1


def test_nonfinite_guess_is_flagged(handle):
    """A NaN in the guess reaches the increments and the norm: the step ends flagged
    NONFINITE and not converged (a non-finite increment must not read as a zero one)."""
    log("nonfinite guess")
    p = W.advection_ie_constant(seed=19, d=3, n=16, cap=2, ic_rank=2, dt=1e-2)
    guess = [np.array(g) for g in p.guess]
    guess[1][3, 0] = np.nan
    rep = B.cp_als_step(handle, p.A, p.B, dev(p.f0), dev(guess), B.default_opts(tol=1e-8, max_sweeps=20))
    log("  flags", rep["flags"], "sweeps", rep["sweeps"], "eps", rep["eps_conv"])
    assert rep["flags"] & B.FLAG_NONFINITE
    assert rep["flags"] & B.FLAG_NOT_CONVERGED
