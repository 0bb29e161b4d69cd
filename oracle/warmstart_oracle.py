"""Plain FP64 CPU oracle of the learned warm start (per-factor-column 1-D CNN).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and by the CPU-baseline leg of
``bench.py``; the HIP library never calls it and shares no code with it.

The paper advances the CP solution of an implicit step by ALS started from the previous
step's factors (Section 3.1, warm start of the sequential minimisation).  The learned form
replaces that starting point by a prediction of the next factors, column by column, and
ALS refines it to the same tolerance.  The network is not in the paper; it is specified
as follows and this module is its definition written out.  The network corrects the
linear extrapolation of the factor columns in time (an untrained, zero output layer
predicts exactly that extrapolation):

* one sample is one factor column l of one dimension k at step n:
    input  x[3, n_k] = (U_k(t_{n-1})[:, l] / s, U_k(t_n)[:, l] / s, c_k),
    s = rms(U_k(t_n)[:, l]) (1 if that is 0), c_k a per-dimension scalar channel;
    output y[n_k], prediction
      U_k(t_{n+1})[:, l] = 2 U_k(t_n)[:, l] - U_k(t_{n-1})[:, l] + OUT s y,
    training target (U_k(t_{n+1})[:, l] - 2 U_k(t_n)[:, l] + U_k(t_{n-1})[:, l]) / (OUT s),
    with the fixed output scale OUT = 2^-12: the correction is far smaller than the column,
    and the scale lets the network work with outputs of order one (a power of two, so
    exact in every precision);
* four circular convolutions of width 5 over the periodic grid,
    z[co, i] = b[co] + sum_{ci, t} W[co, ci, t] x[ci, (i + t - 2) mod n],
  with channel widths 3 -> 32 -> 32 -> 32 -> 1 and ReLU after the first three;
* loss = mean over samples and grid points of (y - target)^2;
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.
Storage precision: weights and stored activations/gradients are BF16 (round to nearest
even), sums are accumulated in FP32 on the device; with ``bf16=True`` this oracle rounds
the same stored quantities to BF16 and accumulates in FP64.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (3, 32, 32, 32, 1)
OUT = 2.0 ** -12   # output scale of the correction
KW = 5          # stencil width
HALF = KW // 2


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.

    BF16 keeps the upper 16 bits of the IEEE single; the value is first rounded to
    FP32 (the device stores FP32 sums), then the low 16 bits are rounded off."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def n_params():
    return sum(WIDTHS[i + 1] * WIDTHS[i] * KW + WIDTHS[i + 1] for i in range(len(WIDTHS) - 1))


def init_params(seed=0):
    """He-uniform weights, zero biases, last layer zero (prediction = linear extrapolation)."""
    rng = np.random.default_rng(seed)
    params = []
    for li in range(len(WIDTHS) - 1):
        cin, cout = WIDTHS[li], WIDTHS[li + 1]
        bound = np.sqrt(6.0 / (cin * KW))
        W = rng.uniform(-bound, bound, size=(cout, cin, KW))
        if li == len(WIDTHS) - 2:
            W[:] = 0.0
        params.append((W, np.zeros(cout)))
    return params


def conv1d_circ(x, W, b):
    """z[B, co, i] = b[co] + sum_{ci,t} W[co, ci, t] x[B, ci, (i + t - 2) mod n]  (plain loops
    over the taps; each tap is a cyclic shift and a channel contraction)."""
    B, cin, n = x.shape
    cout = W.shape[0]
    z = np.broadcast_to(b[None, :, None], (B, cout, n)).astype(np.float64).copy()
    for t in range(KW):
        xs = np.roll(x, -(t - HALF), axis=2)          # xs[..., i] = x[..., (i + t - 2) mod n]
        z += np.einsum('oc,bci->boi', W[:, :, t], xs)
    return z


def forward(params, x, bf16=False):
    """Activations of every layer: acts[0] = x, acts[l+1] = layer l output (after ReLU for
    the first three).  With bf16 the weights, input and stored activations are rounded."""
    rnd = bf16_round if bf16 else (lambda v: v)
    acts = [rnd(x)]
    L = len(params)
    for li, (W, b) in enumerate(params):
        z = conv1d_circ(acts[-1], rnd(W), rnd(b))
        if li < L - 1:
            z = np.maximum(z, 0.0)
            z = rnd(z)
        acts.append(z)
    return acts


def loss_and_grad_out(y, target):
    """MSE over all entries and its gradient with respect to y."""
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, acts, gy, bf16=False):
    """Gradients (dW, db) of every layer for the output gradient gy (manual chain rule:
    a circular convolution's adjoint in x is the convolution with the flipped stencil)."""
    rnd = bf16_round if bf16 else (lambda v: v)
    L = len(params)
    grads = [None] * L
    g = rnd(gy) if bf16 else gy
    for li in range(L - 1, -1, -1):
        W, b = params[li]
        Wr = rnd(W)
        x = acts[li]
        B, cin, n = x.shape
        dW = np.zeros_like(W)
        for t in range(KW):
            xs = np.roll(x, -(t - HALF), axis=2)
            dW[:, :, t] = np.einsum('boi,bci->oc', g, xs)
        db = g.sum(axis=(0, 2))
        grads[li] = (dW, db)
        if li > 0:
            gx = np.zeros_like(x)
            for t in range(KW):
                # z[i] uses x[i + t - 2]  =>  dx[j] += W[., ., t]^T g[j - t + 2]
                gx += np.roll(np.einsum('oc,boi->bci', Wr[:, :, t], g), (t - HALF), axis=2)
            gx = gx * (acts[li] > 0)                   # ReLU of the layer below
            g = rnd(gx) if bf16 else gx
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of the master weights (state: step count and moment arrays)."""
    t = state.get('t', 0) + 1
    state['t'] = t
    new = []
    for li, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
        out = []
        for j, (p, g) in enumerate(((W, dW), (b, db))):
            key = (li, j)
            m = state.get(('m',) + key, np.zeros_like(p))
            v = state.get(('v',) + key, np.zeros_like(p))
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            state[('m',) + key], state[('v',) + key] = m, v
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new


def make_inputs(u_prev, u_cur, coef):
    """Network inputs for a batch of columns (rows of u_prev/u_cur: [B, n]) and their scales."""
    u_prev = np.asarray(u_prev, dtype=np.float64)
    u_cur = np.asarray(u_cur, dtype=np.float64)
    B, n = u_cur.shape
    s = np.sqrt(np.mean(u_cur * u_cur, axis=1))
    s = np.where(s > 0, s, 1.0)
    x = np.empty((B, 3, n))
    x[:, 0] = u_prev / s[:, None]
    x[:, 1] = u_cur / s[:, None]
    x[:, 2] = np.asarray(coef, dtype=np.float64)[:, None] * np.ones((1, n))
    return x, s


def extrapolate(u_prev, u_cur):
    """Linear extrapolation of columns in time: 2 U(t_n) - U(t_{n-1})."""
    return 2.0 * np.asarray(u_cur, dtype=np.float64) - np.asarray(u_prev, dtype=np.float64)


def training_target(u_prev, u_cur, u_next):
    """Target of a batch of columns: the second difference in time over the column's scale
    and the output scale, (U(t_{n+1}) - 2 U(t_n) + U(t_{n-1})) / (OUT s)."""
    _, s = make_inputs(u_prev, u_cur, np.zeros(np.asarray(u_cur).shape[0]))
    return (np.asarray(u_next, dtype=np.float64) - extrapolate(u_prev, u_cur)) / (OUT * s[:, None])


def predict_columns_from_output(u_prev, u_cur, y):
    """The prediction 2 U(t_n) - U(t_{n-1}) + OUT s y for given network outputs y."""
    _, s = make_inputs(u_prev, u_cur, np.zeros(np.asarray(u_cur).shape[0]))
    return extrapolate(u_prev, u_cur) + (OUT * s[:, None]) * np.asarray(y, dtype=np.float64)


def predict_columns(params, u_prev, u_cur, coef, bf16=False):
    """Predicted next columns U(t_{n+1}) = 2 U(t_n) - U(t_{n-1}) + OUT s y for a batch of columns."""
    x, _ = make_inputs(u_prev, u_cur, coef)
    return predict_columns_from_output(u_prev, u_cur, forward(params, x, bf16=bf16)[-1][:, 0, :])
