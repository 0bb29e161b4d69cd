"""Double-double arithmetic for the oracle's residuals and distances.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A double-double (dd) number is an unevaluated sum hi + lo of two float64 values with
|lo| <= ulp(hi) / 2, carried here as a pair of NumPy arrays.  The building blocks are the
error-free transformations of the literature:

* TwoSum (Knuth, TAOCP vol. 2):  a + b = s + e exactly, s = fl(a + b);
* Split (Veltkamp) and TwoProduct (Dekker 1971):  a * b = p + e exactly, p = fl(a b),
  written without a fused multiply-add because NumPy has none;
* the compensated dot product Dot2 of Ogita, Rump & Oishi (SIAM J. Sci. Comput. 26,
  2005), whose result is as accurate as if it had been computed in twice the working
  precision; here its two accumulators are returned as a dd pair instead of being added.

Why it is needed: the residual of an implicit step is evaluated from scalar products of
CP tensors, ||A f - g||^2 = <Af, Af> - 2 <Af, g> + <g, g>.  In float64 the three terms
cancel and leave an absolute error of ~1e-16 ||g||^2, so a relative residual below ~1e-8
cannot be resolved.  Every Gram entry, Hadamard product and final sum in dd pushes that
floor down to ~1e-16 (limited then by the rounding of the applied operator's entries).
"""
from __future__ import annotations

import numpy as np

_SPLITTER = 134217729.0   # 2^27 + 1 (Veltkamp split of a 53-bit significand)


def two_sum(a, b):
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def fast_two_sum(a, b):
    """Exact for |a| >= |b| (or a == 0)."""
    s = a + b
    e = b - (s - a)
    return s, e


def split(a):
    c = _SPLITTER * a
    hi = c - (c - a)
    return hi, a - hi


def two_prod(a, b):
    p = a * b
    ah, al = split(a)
    bh, bl = split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def dd_add(xh, xl, yh, yl):
    s, e = two_sum(xh, yh)
    t, f = two_sum(xl, yl)
    e = e + t
    s, e = fast_two_sum(s, e)
    e = e + f
    return fast_two_sum(s, e)


def dd_mul(xh, xl, yh, yl):
    p, e = two_prod(xh, yh)
    e = e + (xh * yl + xl * yh)
    return fast_two_sum(p, e)


def dd_sum(h, l):
    """Sum of an array of dd numbers by pairwise dd additions (fixed order)."""
    h = np.ravel(np.asarray(h, dtype=np.float64))
    l = np.ravel(np.asarray(l, dtype=np.float64))
    if h.size == 0:
        return 0.0, 0.0
    while h.size > 1:
        if h.size % 2:
            h = np.append(h, 0.0)
            l = np.append(l, 0.0)
        h, l = dd_add(h[0::2], l[0::2], h[1::2], l[1::2])
    return float(h[0]), float(l[0])


def gram_dd(W: np.ndarray):
    """W^T W with every entry a Dot2 compensated sum over the rows: returns (hi, lo)."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    p = np.zeros((m, m))
    s = np.zeros((m, m))
    for t in range(n):
        h, r = two_prod(W[t][:, None], W[t][None, :])
        p, q = two_sum(p, h)
        s = s + (q + r)
    return fast_two_sum(p, s)


def stacked_norm2_dd(factors):
    """||sum_l prod_k W_k[:, l]||^2 of a CP tensor as a dd pair: the d Grams by Dot2, their
    Hadamard product and the sum of its entries in dd (Section 2.2's reduction of scalar
    products of canonical tensors to one-dimensional ones)."""
    Hh = Hl = None
    for Wk in factors:
        gh, gl = gram_dd(Wk)
        if Hh is None:
            Hh, Hl = gh, gl
        else:
            Hh, Hl = dd_mul(Hh, Hl, gh, gl)
    return dd_sum(Hh, Hl)
