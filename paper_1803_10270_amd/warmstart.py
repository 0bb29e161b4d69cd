"""Learned warm start around the implicit CP-ALS step (Section 3.1 solves each step by ALS
started from a guess of f_{n+1}; the plain method uses f_n).

Every numerical step runs in libcpals (include/cpals_ws.h, include/cpals.h): the guess is
the linear extrapolation 2 f_n - f_{n-1} of the factor columns plus the network's
correction, ALS refines it to the tolerance (and falls back to the plain warm start f_n
when it does not converge from the prediction), and the prediction's relative distance to
the converged result is reported.
"""
from __future__ import annotations

import numpy as np

from . import binding as B


def _clone(T):
    return [u.clone() for u in T]


def cp_dist2_parts(h, x, y, scratch):
    """(<x,x>, <x,y>, <y,y>) on the device (three cp_inner calls); scratch: float64 CUDA [3]."""
    B.cp_inner(h, x, x, scratch[0:1])
    B.cp_inner(h, x, y, scratch[1:2])
    B.cp_inner(h, y, y, scratch[2:3])
    return scratch


BAD = B.FLAG_NOT_CONVERGED | B.FLAG_NONFINITE


def learned_step(h, net, A, Bop, f_prev, f_cur, coef, opts, f_out=None):
    """One implicit step from the network's guess; ALS is the arbiter: when it does not
    converge from the prediction (or the prediction is not finite) the step is solved again
    from f_n, the plain warm start.  The report gains 'used_prediction', 'fallback_sweeps'
    and 'pred_rel_dist' (relative distance of the prediction to the converged result)."""
    import torch
    guess = [torch.empty_like(u) for u in f_cur]
    net.predict(f_prev, f_cur, coef, guess)
    scratch = torch.empty(3, dtype=torch.float64, device=f_cur[0].device)
    B.cp_norm(h, guess, scratch[0:1])
    finite = bool(np.isfinite(scratch[0].item()))
    start = _clone(guess) if finite else _clone(f_cur)
    rep = dict(B.cp_als_step(h, A, Bop, f_cur, start, opts))
    used, extra = finite, 0
    if finite and (rep['flags'] & BAD):
        start = _clone(f_cur)
        extra = rep['sweeps']
        rep = dict(B.cp_als_step(h, A, Bop, f_cur, start, opts))
        used = False
    if finite:
        cp_dist2_parts(h, guess, start, scratch)
        v = scratch.cpu().numpy()
        pred = float(np.sqrt(max(v[0] - 2.0 * v[1] + v[2], 0.0) / max(v[2], 1e-300)))
    else:
        pred = float('nan')
    rep.update(used_prediction=bool(used), fallback_sweeps=int(extra), pred_rel_dist=pred)
    rep['sweeps'] = rep['sweeps'] + extra
    if f_out is not None:
        for dst, src in zip(f_out, start):
            dst.copy_(src)
        return f_out, rep
    return start, rep


def init_params(seed=0):
    """Seeded initial parameters in the natural order of include/cpals_ws.h: He-uniform
    weights, zero biases, and a zero output layer (the untrained network predicts the linear
    extrapolation 2 f_n - f_{n-1} exactly)."""
    widths = (3, 32, 32, 32, 1)
    rng = np.random.default_rng(seed)
    out = []
    for li in range(4):
        cin, cout = widths[li], widths[li + 1]
        bound = np.sqrt(6.0 / (cin * 5))
        w = rng.uniform(-bound, bound, size=cout * cin * 5)
        if li == 3:
            w[:] = 0.0
        out += [w, np.zeros(cout)]
    return np.concatenate(out).astype(np.float32)


def trajectory_columns(traj, d, r, n):
    """View a cp_als_run trajectory buffer ([T, sum_k n r] of column-major panels) as
    columns [T, d r, n] (all n_k equal)."""
    T = traj.shape[0]
    return traj.view(T, d * r, n)


def column_coef(coef_dims, r):
    """Per-column scalar channel from the per-dimension one."""
    return np.repeat(np.asarray(coef_dims, dtype=np.float64), r)


def train(net, trajs, coefs, steps, batch, lr, seed=0, log=None):
    """Adam on random (time, column) samples drawn from a list of trajectories [T, C, n]."""
    rng = np.random.default_rng(seed)
    losses = []
    for it in range(steps):
        j = int(rng.integers(len(trajs)))
        tr, cf = trajs[j], coefs[j]
        T, C, _ = tr.shape
        t = rng.integers(1, T - 1, size=batch)
        c = rng.integers(0, C, size=batch)
        loss = net.train_step(tr, np.stack([t, c], axis=1).astype(np.int32), cf, lr)
        losses.append(loss)
        if log is not None and (it % max(1, steps // 10) == 0 or it == steps - 1):
            log("train step %d loss %.4e" % (it, loss))
    return losses
