"""GPU tests of the learned warm start, through the C ABI of include/cpals_ws.h:
forward outputs and parameter gradients against the FP64 oracle (which rounds the same
stored quantities to BF16), training, prediction, and the gain over the plain warm start."""
import numpy as np
import pytest

from gpu_util import dev, host, log
from oracle import warmstart_oracle as WO
from paper_1803_10270_amd import binding as B
from paper_1803_10270_amd import warmstart as WS
from paper_1803_10270_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def handle():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = B.Handle()
    yield h
    h.close()


def flat(params):
    out = []
    for Wt, b in params:
        out.append(np.asarray(Wt).reshape(-1))
        out.append(np.asarray(b).reshape(-1))
    return np.concatenate(out).astype(np.float32)


def unflat(v):
    params, o = [], 0
    for li in range(len(WO.WIDTHS) - 1):
        cin, cout = WO.WIDTHS[li], WO.WIDTHS[li + 1]
        nw = cout * cin * WO.KW
        Wt = v[o:o + nw].reshape(cout, cin, WO.KW).astype(np.float64)
        o += nw
        b = v[o:o + cout].astype(np.float64)
        o += cout
        params.append((Wt, b))
    return params


def random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    params = []
    for li in range(len(WO.WIDTHS) - 1):
        cin, cout = WO.WIDTHS[li], WO.WIDTHS[li + 1]
        bound = scale * np.sqrt(6.0 / (cin * WO.KW))
        params.append((rng.uniform(-bound, bound, size=(cout, cin, WO.KW)), rng.uniform(-0.1, 0.1, size=cout)))
    return flat(params)


@pytest.mark.parametrize("B_,n", [(5, 32), (64, 256), (1, 16)])
def test_forward_matches_oracle(handle, B_, n):
    import torch
    p = random_params(11)
    net = B.WarmStartNet(handle, p, n, max_batch=max(B_, 8))
    rng = np.random.default_rng(3)
    x = rng.normal(size=(B_, 3, n)).astype(np.float32)
    y = torch.empty((B_, n), dtype=torch.float32, device="cuda")
    net.forward(torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    yo = WO.forward(unflat(p), x.astype(np.float64), bf16=True)[-1][:, 0, :]
    yg = y.cpu().numpy().astype(np.float64)
    err = np.abs(yg - yo).max() / np.abs(yo).max()
    rel = np.linalg.norm(yg - yo) / np.linalg.norm(yo)
    log("forward B=%d n=%d: max err %.3e (of max |y|), rel L2 %.3e" % (B_, n, err, rel))
    # Both sides store BF16 activations; the sums are FP32 (device) vs FP64 (oracle), so a
    # stored activation can land one BF16 step (2^-8 relative) apart where the exact sum sits
    # near a rounding boundary.  Bound: a few such steps through three layers.
    assert rel <= 4e-3 and err <= 2e-2
    net.close()


def test_gradients_match_oracle(handle):
    import torch
    n, B_ = 64, 12
    p = random_params(21)
    net = B.WarmStartNet(handle, p, n, max_batch=B_)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(B_, 3, n)).astype(np.float32)
    tgt = rng.normal(size=(B_, n)).astype(np.float32)
    g = torch.empty(B.ws_num_params(), dtype=torch.float32, device="cuda")
    loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda(), g)
    params = unflat(p)
    acts = WO.forward(params, x.astype(np.float64), bf16=True)
    lo, gy = WO.loss_and_grad_out(acts[-1][:, 0:1, :], tgt.astype(np.float64)[:, None, :])
    go = WO.backward(params, acts, gy, bf16=True)
    gg = unflat(g.cpu().numpy())
    log("loss gpu %.6e oracle %.6e" % (loss, lo))
    assert abs(loss - lo) <= 1e-3 * lo
    for li, ((dWg, dbg), (dWo, dbo)) in enumerate(zip(gg, go)):
        rw = np.linalg.norm(dWg - dWo) / np.linalg.norm(dWo)
        rb = np.linalg.norm(dbg - dbo) / max(np.linalg.norm(dbo), 1e-30)
        log("layer %d: dW rel %.3e  db rel %.3e" % (li, rw, rb))
        # the output gradient and the gradients between layers are stored in BF16 on both
        # sides; the remaining difference is FP32 accumulation and boundary roundings
        assert rw <= 2e-2 and rb <= 2e-2
    net.close()


def test_zero_output_layer_predicts_linear_extrapolation(handle):
    import torch
    n, d, r = 32, 3, 4
    p = flat(WO.init_params(seed=2))          # last layer zero: guess = 2 f_cur - f_prev
    net = B.WarmStartNet(handle, p, n, max_batch=d * r)
    rng = np.random.default_rng(0)
    up = [rng.normal(size=(n, r)) for _ in range(d)]
    uc = [rng.normal(size=(n, r)) for _ in range(d)]
    fg = [torch.empty((r, n), dtype=torch.float64, device="cuda") for _ in range(d)]
    net.predict(dev(up), dev(uc), np.ones(d), fg)
    for a, b, c in zip(host(fg), uc, up):
        assert np.array_equal(a, 2.0 * b - c)
    # in place: the guess may overwrite f_cur
    fc = dev(uc)
    net.predict(dev(up), fc, np.ones(d), fc)
    for a, b, c in zip(host(fc), uc, up):
        assert np.array_equal(a, 2.0 * b - c)
    net.close()


def test_predict_matches_oracle(handle):
    import torch
    n, d, r = 64, 2, 3
    p = random_params(31, scale=0.5)
    net = B.WarmStartNet(handle, p, n, max_batch=d * r)
    rng = np.random.default_rng(5)
    up = [rng.normal(size=(n, r)) for _ in range(d)]
    uc = [u + 0.01 * rng.normal(size=(n, r)) for u in up]
    coef = np.array([0.3, -0.2])
    fg = [torch.empty((r, n), dtype=torch.float64, device="cuda") for _ in range(d)]
    net.predict(dev(up), dev(uc), coef, fg)
    params = unflat(p)
    for k in range(d):
        ref = WO.predict_columns(params, up[k].T, uc[k].T, np.full(r, coef[k]), bf16=True).T
        got = host(fg)[k]
        step = np.linalg.norm(ref - WO.extrapolate(up[k].T, uc[k].T).T)   # the network's part
        err = np.linalg.norm(got - ref) / max(step, 1e-30)
        log("predict dim %d: error %.3e of the network's correction" % (k, err))
        assert err <= 1e-2


def translating_trajectory(rng, T, C, n, speed):
    """Columns that translate on the periodic grid: sums of periodic Gaussians moving at
    their own speed (what CP factors of an advected state do)."""
    x = 2 * np.pi * np.arange(n) / n
    cols = np.zeros((T, C, n))
    for c in range(C):
        c0, w, amp = rng.uniform(0, 2 * np.pi), rng.uniform(0.3, 0.8), rng.uniform(0.5, 2.0)
        v = speed * rng.uniform(0.5, 1.5)
        for t in range(T):
            dxs = (x - c0 - v * t + np.pi) % (2 * np.pi) - np.pi
            cols[t, c] = amp * np.exp(-0.5 * (dxs / w) ** 2)
    return cols


def test_training_reduces_loss(handle):
    import torch
    n, C, T = 64, 48, 24
    rng = np.random.default_rng(7)
    tr = torch.from_numpy(translating_trajectory(rng, T, C, n, 0.05)).cuda()
    net = B.WarmStartNet(handle, flat(WO.init_params(seed=5)), n, max_batch=256)
    # the target is the second difference in time (the correction of the linear
    # extrapolation); the loss of the untrained network is that of the extrapolation alone
    losses = WS.train(net, [tr], [np.full(C, 0.5)], steps=400, batch=256, lr=3e-3, seed=1, log=log)
    last = float(np.mean(losses[-10:]))
    log("loss first %.4e last (mean of 10) %.4e" % (losses[0], last))
    assert np.isfinite(last) and last < 0.2 * losses[0]
    net.close()


def _solver_trajectory(h, p, n_steps):
    """Run the plain solver; return the trajectory as columns [T+1, d r, n] (level 0 = f_0
    padded to the rank cap, level t+1 = result of step t) and the per-step reports."""
    import torch
    d, r, n = p.A.d, p.rank_cap, p.A.dims()[0]
    V, U = dev(p.f0), dev(p.guess)
    traj = torch.zeros(n_steps * d * r * n, dtype=torch.float64, device="cuda")
    reps = B.cp_als_run(h, p.A, p.B, V, U, n_steps, B.default_opts(tol=p.tol, max_sweeps=200), traj=traj)
    cols = traj.view(n_steps, d * r, n)
    first = torch.stack([u for u in dev(p.guess)]).reshape(1, d * r, n)
    return torch.cat([first, cols], dim=0).contiguous(), reps


def test_learned_warm_start_saves_sweeps(handle):
    """The variable-coefficient advection step at full size (d=6, n=256, rank 32): trained on
    the converged solver trajectories of three seeds, evaluated on another.  Steps started
    from the prediction (linear extrapolation plus the network's correction) need fewer
    sweeps to the same 1e-8 tolerance than steps started from f_n and reach the same
    solution; the untrained network (the extrapolation alone) is run beside it."""
    import torch
    mk = lambda s: W.advection_ie_variable(seed=s, n_steps=20)
    p0 = mk(200)
    d, r, n = p0.A.d, p0.rank_cap, p0.A.dims()[0]
    dt = 1e-3
    coef = np.full(d, dt * n / (2 * np.pi))               # CFL number dt |a| / h with mean |a| = 1
    trajs = []
    for s in range(201, 211):
        tr, reps = _solver_trajectory(handle, mk(s), 16)
        ok = all(not (q["flags"] & B.FLAG_NOT_CONVERGED) for q in reps)
        log("seed %d: mean sweeps %.1f, converged %s" % (s, np.mean([q['sweeps'] for q in reps]), ok))
        if ok:                                            # only solutions are learned from
            trajs.append(tr[1:].contiguous())             # levels from the first solved step on
        if len(trajs) == 3:
            break
    assert len(trajs) == 3
    net = B.WarmStartNet(handle, flat(WO.init_params(seed=9)), n, max_batch=512)
    for lr, steps in ((2e-3, 200), (5e-4, 200), (1e-4, 100)):
        WS.train(net, trajs, [WS.column_coef(coef, r)] * len(trajs), steps=steps, batch=512, lr=lr, seed=3, log=log)
    # held-out seed: plain trajectory, then each step again from the prediction
    nt = 8
    tr, reps = _solver_trajectory(handle, p0, nt)
    opts = B.default_opts(tol=p0.tol, max_sweeps=200)
    plain, learned, extrap, used = [], [], [], 0
    net0 = B.WarmStartNet(handle, flat(WO.init_params(seed=9)), n, max_batch=512)   # extrapolation only
    from gpu_util import tensor_distance
    for t in range(2, nt):
        prev = [tr[t - 1, k * r:(k + 1) * r].clone() for k in range(d)]
        cur = [tr[t, k * r:(k + 1) * r].clone() for k in range(d)]
        ref = [tr[t + 1, k * r:(k + 1) * r].clone() for k in range(d)]
        out, rep = WS.learned_step(handle, net, p0.A, p0.B, prev, cur, coef, opts)
        learned.append(rep['sweeps'])
        extrap.append(WS.learned_step(handle, net0, p0.A, p0.B, prev, cur, coef, opts)[1]['sweeps'])
        plain.append(reps[t]['sweeps'])
        used += rep['used_prediction']
        dist = tensor_distance(host(out), host(ref))
        log("step %d: plain %d sweeps, learned %d (prediction used %s, its error %.2e, plain guess error %.2e); "
            "distance of the two solutions %.2e" % (t, reps[t]['sweeps'], rep['sweeps'], rep['used_prediction'],
                                                    rep['pred_rel_dist'], tensor_distance(host(cur), host(ref)), dist))
        assert dist <= 1e-5, dist
    log("mean sweeps plain %.2f learned %.2f (untrained: extrapolation alone %.2f)" % (
        np.mean(plain), np.mean(learned), np.mean(extrap)))
    net0.close()
    assert used >= len(learned) // 2
    assert np.mean(learned) <= 0.5 * np.mean(plain)
    assert np.mean(learned) <= np.mean(extrap)           # the training adds to the extrapolation
    net.close()
