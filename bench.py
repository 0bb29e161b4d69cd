"""Benchmark: implicit CP-ALS time steps per second on one MI355X.

Workload: 6-D advection with variable separable coefficients a_i(x) = 1 + 0.5 sin(x_{i+1}),
implicit Euler (13 Kronecker terms), n = 256 points per dimension, fixed separation rank 32
(from a rank-8 Gaussian-mixture initial condition), ALS tolerance 1e-8 on the relative
increment, at most 200 sweeps per step, FP64.  Synthetic seeded inputs.

A step is one implicit time step: the full ALS solve of A f_{n+1} = f_n (all sweeps), run
device-resident in one persistent kernel launch per batch of steps.

Beside the plain method (the headline value) the same run measures the two other forms at
the same 1e-8 tolerance:
  learned  the linear extrapolation 2 f_n - f_{n-1} corrected by the per-column CNN, trained
           on solver trajectories of new seeds, against the plain warm start f_n on a
           held-out instance of the same workload (the untrained network, i.e. the
           extrapolation alone, is reported beside it);
  batched  256 uneven advection instances in one persistent launch against the same
           instances advanced one launch at a time (a seeded sample, scaled by cost);
  mixed    FP32 matrix-core sweeps finished by an FP64 sweep, against FP64 throughout, on
           the kinetic Crank-Nicolson workload (d = 6, n = 128, rank 64).
It also reports the HBM rates of the streaming kernels (cp_inner, cp_apply_operator) on
gigabyte panels.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
    python bench.py --form batched|streaming     (that leg alone)

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CP-ALS time-steps/s (d=6,n=256,r=32) at equal residual, learned/batched vs plain"
FP64_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (= FP64 matrix) peak
HBM_PEAK_GBS = 8000.0


def flop_model(p, reports):
    """Algorithmic FP64 flops of the reported sweeps / PCG iterations (per launch).

    Per dimension update q (n = n_q, m = distinct ops of A in dim q, mb of B, r, r0):
      Gram refresh      2 n (m r)^2 + 2 n (m r)(mb r0)
      Hadamard assembly (T_A^2 (d-1) r^2 + T_A T_B (d-1) r r0) * 2
      right-hand side   2 n (mb r0)(m r)
      matvec (M+lam)x   2 n (m r)^2                    (the stencil parts are O(n r m) and omitted)
      preconditioner    2 n r^2
      increment         2 n r^2
    and one matvec for the initial residual, per update; per PCG iteration a matvec and a
    preconditioner application."""
    A, B = p.A, p.B
    d = A.d
    r = p.rank_cap
    dims = A.dims()
    T_A, T_B = A.n_terms, B.n_terms
    per_sweep = 0.0
    for q in range(d):
        n = dims[q]
        m = len(A.ops[q])
        mb = len(B.ops[q])
        r0 = r
        per_sweep += 2 * n * (m * r) ** 2 + 2 * n * (m * r) * (mb * r0)
        per_sweep += 2 * (T_A * T_A * (d - 1) * r * r + T_A * T_B * (d - 1) * r * r0)
        per_sweep += 2 * n * (mb * r0) * (m * r)
        per_sweep += 2 * n * (m * r) ** 2 + 2 * n * r * r      # initial residual + increment
    n_avg = float(np.mean(dims))
    m_avg = float(np.mean([len(o) for o in A.ops]))
    per_pcg = 2 * n_avg * (m_avg * r) ** 2 + 2 * n_avg * r * r
    sweeps = sum(rp["sweeps"] for rp in reports)
    iters = sum(rp["pcg_iters"] for rp in reports)
    return sweeps * per_sweep + iters * per_pcg


def cpu_baseline(p, sweeps_per_step, n_sweeps=4):
    """The FP64 oracle on the host: the first n_sweeps sweeps of the first step, scaled to
    time-steps/s with the GPU run's mean sweeps per step."""
    from oracle import cpals_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    O.als_step(p.A, p.B, p.f0, p.guess, tol=0.0, max_sweeps=n_sweeps)
    dt = time.perf_counter() - t0
    per_sweep = dt / n_sweeps
    return {"value": 1.0 / (per_sweep * sweeps_per_step), "unit": "time-steps/s", "cores": int(cores),
            "kind": "oracle",
            "sample": "first %d ALS sweeps of step 1 (%.1f s, %.2f s/sweep) scaled by %.1f sweeps/step; "
                      "dense BLAS threads=%d, sparse direct solve single-threaded" % (
                          n_sweeps, dt, per_sweep, sweeps_per_step, cores)}


def kernel_source_hash():
    """Hash of the kernel sources: a committed counter summary applies only to this code."""
    import hashlib
    hsh = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1803_10270_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def committed_traffic():
    """HBM bytes per launch of the timed configuration from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or None when
    the summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "als_persistent_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def bench_learned(args, log):
    """Learned warm start vs plain warm start on held-out steps (same tolerance); the untrained
    network (the linear extrapolation alone) is timed beside them."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import warmstart as WS
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    mk = lambda s: W.advection_ie_variable(seed=s, n_steps=args.learned_train_steps + 1)
    p0 = mk(args.seed + 300)
    d, r, n = p0.A.d, p0.rank_cap, p0.A.dims()[0]
    coef = np.full(d, 1e-3 * n / (2 * np.pi))
    opts = B.default_opts(tol=p0.tol, max_sweeps=args.max_sweeps)

    def trajectory(p, steps):
        V, U = B.to_device(p.f0), B.to_device(p.guess)
        traj = torch.zeros(steps * d * r * n, dtype=torch.float64, device="cuda")
        reps = B.cp_als_run(h, p.A, p.B, V, U, steps, opts, traj=traj)
        return traj.view(steps, d * r, n), reps

    t0 = time.perf_counter()
    trajs = []
    # training data: the trajectories of new seeds whose every step converged (an unconverged
    # step is an ALS iterate, not a solution of the step)
    for sd in range(args.seed + 301, args.seed + 301 + 4 * args.learned_train_seeds):
        tr, reps = trajectory(mk(sd), args.learned_train_steps)
        if all(not (q["flags"] & B.FLAG_NOT_CONVERGED) for q in reps):
            trajs.append(tr.contiguous())
        if len(trajs) == args.learned_train_seeds:
            break
    t_data = time.perf_counter() - t0
    net = B.WarmStartNet(h, WS.init_params(seed=9), n, max_batch=512)
    t0 = time.perf_counter()
    losses = []
    for lr, steps in ((2e-3, 200), (5e-4, 200), (1e-4, 100)):
        losses += WS.train(net, trajs, [WS.column_coef(coef, r)] * len(trajs), steps=steps, batch=512, lr=lr, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    log("learned: %d training trajectories in %.1f s, %d Adam steps in %.1f s (loss %.2e -> %.2e)" % (
        len(trajs), t_data, len(losses), t_train, losses[0], losses[-1]))
    # held-out instance: warm up 2 steps (the predictor needs two levels), then K steps each way
    K = args.learned_eval_steps
    V, U = B.to_device(p0.f0), B.to_device(p0.guess)
    B.cp_als_run(h, p0.A, p0.B, V, U, 1, opts)
    lvl1 = [u.clone() for u in U]
    B.cp_als_run(h, p0.A, p0.B, [u.clone() for u in U], U, 1, opts)
    lvl2 = [u.clone() for u in U]
    # plain: K steps from level 2, one step per call (the same granularity as the learned form)
    cur = [u.clone() for u in lvl2]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_sweeps = []
    for _ in range(K):
        nxt = [u.clone() for u in cur]
        rep = B.cp_als_step(h, p0.A, p0.B, cur, nxt, opts)
        plain_sweeps.append(rep["sweeps"])
        cur = nxt
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    # learned: the same K steps from the same levels; then the untrained network (zero output
    # layer: the linear extrapolation alone) to show what the training adds
    def predicted_run(model):
        prev, cur = [u.clone() for u in lvl1], [u.clone() for u in lvl2]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sw, used, errs = [], 0, []
        for _ in range(K):
            out, rep = WS.learned_step(h, model, p0.A, p0.B, prev, cur, coef, opts)
            sw.append(rep["sweeps"])
            used += rep["used_prediction"]
            errs.append(rep["pred_rel_dist"])
            prev, cur = cur, out
        torch.cuda.synchronize()
        return time.perf_counter() - t0, sw, used, errs

    t_learned, learned_sweeps, used, errs = predicted_run(net)
    net0 = B.WarmStartNet(h, WS.init_params(seed=9), n, max_batch=512)
    t_extrap, extrap_sweeps, _, extrap_errs = predicted_run(net0)
    net0.close()
    net.close()
    h.close()
    return {"form": "learned", "workload": "advection_ie_variable d=6 n=256 r=32, held-out seed %d, %d steps" % (
                args.seed + 300, K),
            "train": {"trajectories": len(trajs), "levels_each": args.learned_train_steps, "adam_steps": len(losses),
                      "batch": 512, "loss_first": losses[0], "loss_last": losses[-1], "seconds": t_train},
            "plain_steps_per_s": K / t_plain, "learned_steps_per_s": K / t_learned,
            "speedup": t_plain / t_learned, "plain_mean_sweeps": float(np.mean(plain_sweeps)),
            "learned_mean_sweeps": float(np.mean(learned_sweeps)), "prediction_used": used,
            "prediction_rel_error_mean": float(np.nanmean(errs)),
            "untrained_extrapolation": {"steps_per_s": K / t_extrap, "mean_sweeps": float(np.mean(extrap_sweeps)),
                                        "prediction_rel_error_mean": float(np.nanmean(extrap_errs))}}


def bench_batched(args):
    """Batched form: uneven advection instances (d in {4,6}, n in {64..512}, rank caps 4..48) in one
    persistent launch, against the same instances advanced one at a time (a seeded sample of
    them, scaled by the instances' cost model)."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    probs = W.batched_instances(args.batch_count, n_steps=args.batch_steps)
    h = B.Handle()
    opts = B.default_opts(tol=1e-8, max_sweeps=args.max_sweeps)

    def cost(p):
        return sum(n * len(ops) ** 2 * p.rank_cap ** 2 for n, ops in zip(p.A.dims(), p.A.ops))

    fi = [B.to_device(p.f0) for p in probs]
    fo = [B.to_device(p.guess) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = B.cp_als_run_batched(h, [p.A for p in probs], [p.B for p in probs], fi, fo, args.batch_steps, opts)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    steps_total = args.batch_count * args.batch_steps
    sample = list(range(0, args.batch_count, max(1, args.batch_count // args.plain_sample)))[:args.plain_sample]
    t_plain_sample = 0.0
    for i in sample:
        p = probs[i]
        v, u = B.to_device(p.f0), B.to_device(p.guess)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        B.cp_als_run(h, p.A, p.B, v, u, args.batch_steps, opts)
        torch.cuda.synchronize()
        t_plain_sample += time.perf_counter() - t1
    scale = sum(cost(p) for p in probs) / sum(cost(probs[i]) for i in sample)
    t_plain = t_plain_sample * scale
    sweeps = [r["sweeps"] for rr in reps for r in rr]
    # whole-chip matrix-core use of the batched launch: the instances' algorithmic flops
    # (same model as the headline roofline) over the launch's wall time
    flops = sum(flop_model(p, rr) for p, rr in zip(probs, reps))
    out = {"form": "batched", "instances": args.batch_count, "steps_each": args.batch_steps,
           "roofline": {"bound": "mfma", "achieved": flops / t_batched / 1e12, "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": flops / t_batched / 1e12 / FP64_PEAK_TFLOPS,
                        "flops": flops, "seconds": t_batched},
           "batched_s": t_batched, "batched_steps_per_s": steps_total / t_batched,
           "plain_sample": len(sample), "plain_s_sample": t_plain_sample, "plain_s_estimated": t_plain,
           "plain_steps_per_s": steps_total / t_plain, "speedup": t_plain / t_batched,
           "mean_sweeps_per_step": float(np.mean(sweeps)),
           "converged_steps": int(sum(1 for rr in reps for r in rr if not (r["flags"] & B.FLAG_NOT_CONVERGED)))}
    h.close()
    return out


def bench_mixed(args, log):
    """Mixed-precision form on the linearised kinetic workload (d = 6, n = 128, rank 64,
    Crank-Nicolson, tol 1e-8): the same steps in FP64 and mixed precision from the same
    state, their rates and the distance of the two results."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    p = W.kinetic_cn(seed=0, n=128, cap=64)
    K = 2
    res = {}
    for name, prec in (("fp64", B.PREC_FP64), ("mixed", B.PREC_MIXED)):
        V, U = B.to_device(p.f0), B.to_device(p.guess)
        opts = B.default_opts(tol=p.tol, max_sweeps=args.max_sweeps, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = B.cp_als_run(h, p.A, p.B, V, U, K, opts)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0, reps, U)
    # ||x - y|| / ||y|| from device scalar products (resolves distances above ~1e-7)
    dots = torch.zeros(3, dtype=torch.float64, device="cuda")
    x, y = res["mixed"][2], res["fp64"][2]
    B.cp_inner(h, x, x, dots[0:1])
    B.cp_inner(h, x, y, dots[1:2])
    B.cp_inner(h, y, y, dots[2:3])
    xx, xy, yy = dots.cpu().tolist()
    dist = float(np.sqrt(max(xx - 2 * xy + yy, 0.0) / yy))
    h.close()
    log("mixed: kinetic d=6 n=128 r=64, %d steps: fp64 %.2f s, mixed %.2f s, distance %.2e" % (
        K, res["fp64"][0], res["mixed"][0], dist))
    return {"form": "mixed", "workload": "kinetic_cn d=6 n=128 r=64 (5 Kronecker terms, CN, dt=0.01, tol=1e-8), "
                                         "%d steps" % K,
            "fp64_steps_per_s": K / res["fp64"][0], "mixed_steps_per_s": K / res["mixed"][0],
            "speedup": res["fp64"][0] / res["mixed"][0],
            "fp64_sweeps": [r["sweeps"] for r in res["fp64"][1]], "mixed_sweeps": [r["sweeps"] for r in res["mixed"][1]],
            "rel_distance_to_fp64": dist}


def bench_streaming(log):
    """The HBM-bound kernels on gigabyte inputs: cp_inner (d = 2, n = 2^22, ranks 16 and 16)
    and cp_apply_operator (d = 2, n = 2^21, rank 16, 3 terms), achieved GB/s of their
    algorithmic bytes against the 8 TB/s HBM peak (HIP events, median of 5 calls).  The
    applied operator's terms are scaled identities: banded and diagonal 1-D operators carry
    per-row coefficients that every call copies from host memory (the API's contract), and
    that upload, not the kernel, would be timed."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    out = {}
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=5):
        fn()
        ts = []
        for _ in range(reps):
            a, b = ev(), ev()
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) * 1e-3)
        return float(np.median(ts))

    n, r = 1 << 22, 16
    g = torch.Generator(device="cuda").manual_seed(0)
    x = [torch.randn((r, n), dtype=torch.float64, device="cuda", generator=g) for _ in range(2)]
    y = [torch.randn((r, n), dtype=torch.float64, device="cuda", generator=g) for _ in range(2)]
    o = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = timed(lambda: B.cp_inner(h, x, y, o))
    nbytes = 2 * 8 * n * (r + r)
    out["cp_inner"] = {"shape": "d=2 n=2^22 r=16 x 16", "bytes": nbytes, "seconds": t, "GB_per_s": nbytes / t / 1e9,
                       "frac_of_hbm_peak": nbytes / t / 1e9 / HBM_PEAK_GBS}
    del x, y
    n2 = 1 << 21
    L = W.SepOperator(np.array([1.0, 0.5, 0.25]), np.zeros((3, 2), dtype=np.int32), [[W.op_identity(n2)]] * 2)
    xa = [torch.randn((r, n2), dtype=torch.float64, device="cuda", generator=g) for _ in range(2)]
    ya = [torch.empty((3 * r, n2), dtype=torch.float64, device="cuda") for _ in range(2)]
    t = timed(lambda: B.cp_apply_operator(h, L, xa, ya))
    nbytes = 2 * 8 * n2 * r * (1 + 3)
    out["cp_apply_operator"] = {"shape": "d=2 n=2^21 r=16, 3 scaled-identity terms", "bytes": nbytes, "seconds": t,
                                "GB_per_s": nbytes / t / 1e9, "frac_of_hbm_peak": nbytes / t / 1e9 / HBM_PEAK_GBS}
    del xa, ya
    h.close()
    log("streaming: cp_inner %.0f GB/s, cp_apply_operator %.0f GB/s" % (out["cp_inner"]["GB_per_s"],
                                                                     out["cp_apply_operator"]["GB_per_s"]))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-sweeps", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "streaming"],
                    help="plain: the headline line; batched / streaming: that leg alone")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--no-forms", action="store_true", help="skip the learned and batched forms")
    ap.add_argument("--learned-train-seeds", type=int, default=3)
    ap.add_argument("--learned-train-steps", type=int, default=16)
    ap.add_argument("--learned-eval-steps", type=int, default=6)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only (sharding the step across GPUs is not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.form == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.form == "streaming":
        print(json.dumps(bench_streaming(log)), flush=True)
        return
    p = W.advection_ie_variable(seed=args.seed)
    h = B.Handle()
    opts = B.default_opts(tol=p.tol, max_sweeps=args.max_sweeps)
    V = B.to_device(p.f0)
    U = B.to_device(p.guess)
    # warmup: the first W steps (untimed); they also leave f_W as the state to continue from
    t_w = time.perf_counter()
    if args.warmup > 0:
        B.cp_als_run(h, p.A, p.B, V, U, args.warmup, opts)
    torch.cuda.synchronize()
    t_w = time.perf_counter() - t_w
    print("warmup %d steps: %.2f s" % (args.warmup, t_w), file=sys.stderr, flush=True)
    V2 = [u.clone() for u in U]
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    reports = B.cp_als_run(h, p.A, p.B, V2, U, args.steps, opts)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    print("timed %d steps: %.3f s wall, %.3f ms events" % (args.steps, wall, gpu_ms), file=sys.stderr, flush=True)
    sweeps = [r["sweeps"] for r in reports]
    flops = flop_model(p, reports)
    achieved = flops / (gpu_ms * 1e-3) / 1e12
    value = args.steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "advection_ie_variable d=6 n=256 r=32 (13 Kronecker terms, implicit Euler, "
                               "dt=1e-3, tol=1e-8, max_sweeps=%d, seed %d)" % (args.max_sweeps, args.seed),
                   "d": 6, "n": 256, "r": 32, "form": "plain", "precision": "fp64"},
        "sweeps_per_step": float(np.mean(sweeps)),
        "pcg_iters_per_update": float(sum(r["pcg_iters"] for r in reports) / max(1, 6 * sum(sweeps))),
        "converged_steps": int(sum(1 for r in reports if not (r["flags"] & B.FLAG_NOT_CONVERGED))),
        "eps_conv_last": reports[-1]["eps_conv"],
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "als_persistent", "flops_per_launch": flops, "launch_ms": gpu_ms,
                     "source_hash": kernel_source_hash()},
    }
    tr = committed_traffic()
    if tr is not None and tr.get("steps") == args.steps and tr.get("max_sweeps") == args.max_sweeps:
        out["roofline"]["traffic"] = tr["bytes_per_launch"]
    if not args.no_forms:
        forms = {}
        try:
            forms["learned"] = bench_learned(args, log)
        except Exception as e:   # a form that cannot run is reported, the headline stands
            forms["learned"] = {"error": repr(e)}
        try:
            args_b = argparse.Namespace(**vars(args))
            args_b.batch_steps = 2
            forms["batched"] = bench_batched(args_b)
        except Exception as e:
            forms["batched"] = {"error": repr(e)}
        try:
            forms["mixed"] = bench_mixed(args, log)
        except Exception as e:
            forms["mixed"] = {"error": repr(e)}
        out["forms"] = forms
        try:
            out["streaming"] = bench_streaming(log)
        except Exception as e:
            out["streaming"] = {"error": repr(e)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, float(np.mean(sweeps)))
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
