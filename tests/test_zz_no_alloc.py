"""cp_inner_noalloc (the scalar product for callers that cannot allocate) against cp_inner on
the same inputs, through the C ABI: two calls in a row, the second on a smaller input, and a
shape that uses the chunk cap (rank 64 x 64 over 2^20 rows)."""
import numpy as np
import pytest

from gpu_util import dev, log
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


def both(h, X, Y):
    import torch
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    x, y = dev(X), dev(Y)
    B.cp_inner(h, x, y, out[0:1])
    B.cp_inner_noalloc(h, x, y, out[1:2])
    return out.cpu().numpy()


def test_noalloc_matches_cp_inner_twice_second_smaller(handle):
    rng = np.random.default_rng(77)
    for dims, rx, ry in (([300, 4097, 64, 129], 33, 17), ([70, 9], 5, 3)):
        log("noalloc", dims, rx, ry)
        X = W.random_factors(rng, dims, rx)
        Y = W.random_factors(rng, dims, ry)
        got, ref = both(handle, X, Y)
        scale = O.cp_norm(X) * O.cp_norm(Y)
        log("cp_inner %.17e noalloc %.17e" % (got, ref))
        assert abs(got - ref) <= 1e-12 * scale
        assert abs(ref - O.cp_inner(X, Y)) <= 1e-12 * scale


def test_noalloc_with_capped_chunks(handle):
    """Rank 64 x 64: the 4 MiB scratch holds partials for ~120 chunks, so the 2^20-row panel
    is reduced in far fewer, longer chunks than cp_inner uses."""
    import torch
    log("noalloc capped")
    n, r = 1 << 20, 64
    g = torch.Generator(device="cuda").manual_seed(5)
    x = [torch.randn((r, n), dtype=torch.float64, device="cuda", generator=g),
         torch.randn((r, 16), dtype=torch.float64, device="cuda", generator=g)]
    y = [torch.randn((r, n), dtype=torch.float64, device="cuda", generator=g),
         torch.randn((r, 16), dtype=torch.float64, device="cuda", generator=g)]
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    B.cp_inner(handle, x, y, out[0:1])
    B.cp_inner_noalloc(handle, x, y, out[1:2])
    a, b = out.cpu().numpy()
    X = [t.cpu().numpy().T for t in x]
    Y = [t.cpu().numpy().T for t in y]
    ref = O.cp_inner(X, Y)
    scale = O.cp_norm(X) * O.cp_norm(Y)
    log("cp_inner %.17e noalloc %.17e oracle %.17e" % (a, b, ref))
    assert abs(a - b) <= 1e-12 * scale and abs(b - ref) <= 1e-12 * scale
