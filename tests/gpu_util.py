"""Helpers for the GPU parity tests: move problems to the device, run the library through the
C ABI, compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

from paper_1803_10270_amd import binding as B


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(U):
    return B.to_device(U)


def host(T):
    return B.to_host(T)


def rel_panels(X, Y):
    num = sum(np.linalg.norm(x - y) ** 2 for x, y in zip(X, Y))
    den = sum(np.linalg.norm(y) ** 2 for y in Y)
    return float(np.sqrt(num / den))


def tensor_distance(X, Y, n_samples=1 << 16):
    """Relative l2 distance of two represented CP tensors: exact on small grids, else over
    seeded sample points."""
    from oracle import cpals_oracle as O
    size = np.prod([x.shape[0] for x in X])
    if size <= 2_000_000:
        fx, fy = O.full_tensor(X), O.full_tensor(Y)
        return float(np.linalg.norm(fx - fy) / np.linalg.norm(fy))
    return O.sampled_rel_distance(X, Y, n_samples)
