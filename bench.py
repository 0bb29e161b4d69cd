"""Benchmark: implicit CP-ALS time steps per second on one MI355X.

Workload (the headline): 6-D advection with variable separable coefficients
a_i(x) = 1 + 0.5 sin(x_{i+1}), implicit Euler (13 Kronecker terms), n = 256 points per
dimension, fixed separation rank 32 (from a rank-8 Gaussian-mixture initial condition), ALS
tolerance 1e-8 on the relative increment, at most 200 sweeps per step, FP64.  Synthetic
seeded inputs.  A step is one implicit time step: the full ALS solve of A f_{n+1} = f_n (all
sweeps), run device-resident in one persistent kernel launch per batch of steps on a
16-workgroup cluster; the K timed steps are one launch.  After the timed region every timed
step's residual rho = ||A f_{n+1} - f_n|| / ||f_n|| is formed in double-double from the
trajectory buffer the launch filled.

Beside it, every form is run to the same stopping rule (eps_conv <= 1e-8 every step) and
reports converged / total steps and its residuals rho:
  learned  the linear extrapolation 2 f_n - f_{n-1} corrected by the per-column CNN, trained
           on 10^4 solver steps of new seeds (100 trajectories x 100 steps, generated in one
           batched launch), against the plain warm start f_n on held-out instances of the
           same workload; the untrained network (the extrapolation alone) beside it;
  batched  the 256 uneven advection instances (d in {4,6}, n in {64..512}, rank caps 4-48),
           20 steps each, adaptive rank up to each instance's cap, in one persistent launch,
           against a seeded sample of the same instances advanced one launch at a time
           (scaled by a cost model from the batched reports);
  mixed    FP32 matrix-core sweeps followed by FP64 sweeps to the tolerance, against FP64
           throughout, on the kinetic Crank-Nicolson workload (d = 6, n = 128, rank 64,
           50 steps).
Under "next" it times the paper's other steps and experiments (damped Jacobi sweeps, the
linearised BGK equation, the linear-velocity advection with the implicit and the explicit AB2
step).  It also reports the HBM rates of the streaming kernels (cp_inner, cp_apply_operator) and, as
cpu_baseline, one converged step of the FP64 oracle on the host (all cores; a single thread
beside it).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]
    python bench.py --form learned|batched|mixed|next|streaming   (that leg alone)
    python bench.py --form calibrate   (a 1 GiB device copy: the load that calibrates the
                                        rocprofv3 FETCH_SIZE / WRITE_SIZE counters)

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
TOL = 1e-8
TAU_BATCHED = 1e-5        # relative step residual that adaptive rank grows above (batched form)


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


def flop_model_ranks(p, reports):
    """flop_model with every step's own final rank (adaptive rank)."""
    A, Bop = p.A, p.B
    d = A.d
    dims = A.dims()
    T_A, T_B = A.n_terms, Bop.n_terms
    total = 0.0
    for rp in reports:
        r = max(1, rp["final_rank"])
        per_sweep = 0.0
        for q in range(d):
            n, m, mb = dims[q], len(A.ops[q]), len(Bop.ops[q])
            per_sweep += 2 * n * (m * r) ** 2 + 2 * n * (m * r) * (mb * r)
            per_sweep += 2 * (T_A * T_A * (d - 1) * r * r + T_A * T_B * (d - 1) * r * r)
            per_sweep += 2 * n * (mb * r) * (m * r)
            per_sweep += 2 * n * (m * r) ** 2 + 2 * n * r * r
        n_avg = float(np.mean(dims))
        m_avg = float(np.mean([len(o) for o in A.ops]))
        total += rp["sweeps"] * per_sweep + rp["pcg_iters"] * (2 * n_avg * (m_avg * r) ** 2 + 2 * n_avg * r * r)
    return total


def cost_proxy(p, reports):
    """Relative cost of an instance's run (sweeps x sum_k n_k (m_k r)^2), for scaling the
    one-at-a-time sample to all instances."""
    return sum(rp["sweeps"] * sum(n * (len(ops) * max(1, rp["final_rank"])) ** 2 for n, ops in zip(p.A.dims(), p.A.ops))
               for rp in reports)


def cpu_baseline(p, log):
    """The FP64 oracle on the host: one full converged step (tol 1e-8) of the headline
    workload from its first state, timed with all BLAS threads, and the same step on a
    single thread (the oracle's sparse direct solves are single-threaded either way)."""
    from oracle import cpals_oracle as O
    from threadpoolctl import threadpool_info, threadpool_limits
    cores = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    t0 = time.perf_counter()
    _, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=p.tol, max_sweeps=200)
    t_all = time.perf_counter() - t0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        _, rep1 = O.als_step(p.A, p.B, p.f0, p.guess, tol=p.tol, max_sweeps=200)
        t_one = time.perf_counter() - t0
    log("cpu baseline: one step %.1f s on %d threads, %.1f s on one (%d sweeps)" % (t_all, cores, t_one, rep["sweeps"]))
    return {"value": 1.0 / t_all, "unit": "time-steps/s", "cores": int(cores), "kind": "oracle",
            "nproc": os.cpu_count(), "single_thread_value": 1.0 / t_one,
            "sample": "one converged step (step 1, %d sweeps, tol 1e-8) of the headline workload: %.1f s with %d BLAS "
                      "threads, %.1f s with one" % (rep["sweeps"], t_all, cores, t_one)}


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
    """HBM bytes per time step of the headline launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel calibration), or None when
    the summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "als_persistent_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or "bytes_per_step" not in rec:
        return None
    return rec


def identity(dims):
    from paper_1803_10270_amd import workloads as W
    return W.identity_operator(list(dims))


def rel_distance_dev(h, x, y):
    """||x - y|| / ||y|| of two device CP tensors in double-double (the step residual of
    A = B = I)."""
    from paper_1803_10270_amd import binding as B
    dims = [int(t.shape[1]) for t in x]
    I = identity(dims)
    return B.cp_residual(h, I, I, x, y)


def traj_states(traj, n_steps, dims, rc):
    """Factor panels (lists of (rc, n_k) views) of every step of a trajectory buffer."""
    out = []
    per = sum(dims) * rc
    for s in range(n_steps):
        base = traj[s * per:(s + 1) * per]
        o, st = 0, []
        for n in dims:
            st.append(base[o:o + n * rc].view(rc, n))
            o += n * rc
        out.append(st)
    return out


def step_residuals(h, A, Bop, f0, states, ranks=None):
    """rho of every step of a trajectory (f0 the state before the first)."""
    from paper_1803_10270_amd import binding as B
    rhos = []
    prev, prev_r = f0, None
    for s, st in enumerate(states):
        r = None if ranks is None else ranks[s]
        rhos.append(B.cp_residual(h, A, Bop, st, prev, f_rank=r, f_n_rank=prev_r))
        prev, prev_r = st, r
    return rhos


def summarize_rho(rhos):
    a = np.asarray(rhos, dtype=np.float64)
    return {"max": float(a.max()), "median": float(np.median(a)), "last": float(a[-1])}


def bench_learned(args, log):
    """Learned warm start on the d = 6, n = 256, rank-32 workload: training data are solver
    trajectories of new seeds, generated in one batched launch (every step converged); the
    network is trained on them; held-out instances are stepped K times from the same two
    levels three ways: plain (f_n), the trained network's prediction, and the untrained
    network's (the linear extrapolation alone).  Every step of every leg stops at
    eps_conv <= 1e-8; rho of every step is reported."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import warmstart as WS
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    steps_per = args.learned_train_steps
    mk = lambda s, k: W.advection_ie_variable(seed=s, n_steps=k)
    p0 = mk(args.seed + 2000, 1)
    d, r, n = p0.A.d, p0.rank_cap, p0.A.dims()[0]
    coef = np.full(d, 1e-3 * n / (2 * np.pi))
    opts = B.default_opts(tol=TOL, max_sweeps=args.max_sweeps)
    # training trajectories: one batched launch, one workgroup per trajectory
    t0 = time.perf_counter()
    seeds = [args.seed + 1000 + i for i in range(args.learned_train_trajs)]
    probs = [mk(s, steps_per) for s in seeds]
    trajs = [torch.zeros(steps_per * d * r * n, dtype=torch.float64, device="cuda") for _ in probs]
    reps = B.cp_als_run_batched(h, [p.A for p in probs], [p.B for p in probs], [B.to_device(p.f0) for p in probs],
                                [B.to_device(p.guess) for p in probs], steps_per, opts, trajs=trajs)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    keep = [i for i, rr in enumerate(reps) if all(not (q["flags"] & B.FLAG_NOT_CONVERGED) for q in rr)]
    train = [trajs[i].view(steps_per, d * r, n) for i in keep]
    log("learned: %d training trajectories x %d steps in %.1f s (%d fully converged)" % (
        len(probs), steps_per, t_data, len(keep)))
    net = B.WarmStartNet(h, WS.init_params(seed=9), n, max_batch=512)
    t0 = time.perf_counter()
    losses = []
    for lr, nsteps in ((2e-3, args.learned_adam // 2), (5e-4, args.learned_adam // 3), (1e-4, args.learned_adam // 6)):
        losses += WS.train(net, train, [WS.column_coef(coef, r)] * len(train), steps=nsteps, batch=512, lr=lr, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del trajs, train
    log("learned: %d Adam steps in %.1f s (loss %.2e -> %.2e)" % (len(losses), t_train, losses[0], losses[-1]))
    net0 = B.WarmStartNet(h, WS.init_params(seed=9), n, max_batch=512)
    K = args.learned_eval_steps
    per_seed = []
    tot = {"plain": 0.0, "learned": 0.0, "extrap": 0.0}
    for j in range(args.learned_eval_seeds):
        p = mk(args.seed + 2000 + j, 1)
        V, U = B.to_device(p.f0), B.to_device(p.guess)
        B.cp_als_run(h, p.A, p.B, V, U, 1, opts)
        lvl1 = [u.clone() for u in U]
        B.cp_als_run(h, p.A, p.B, [u.clone() for u in U], U, 1, opts)
        lvl2 = [u.clone() for u in U]

        def run(kind):
            prev, cur = [u.clone() for u in lvl1], [u.clone() for u in lvl2]
            states, reps_k = [], []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(K):
                if kind == "plain":
                    nxt = [u.clone() for u in cur]
                    rep = B.cp_als_step(h, p.A, p.B, cur, nxt, opts)
                else:
                    nxt, rep = WS.learned_step(h, net if kind == "learned" else net0, p.A, p.B, prev, cur, coef, opts)
                reps_k.append(rep)
                states.append(nxt)
                prev, cur = cur, nxt
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rhos = step_residuals(h, p.A, p.B, lvl2, states)
            return dt, reps_k, rhos

        row = {"seed": args.seed + 2000 + j}
        for kind in ("plain", "learned", "extrap"):
            dt, reps_k, rhos = run(kind)
            tot[kind] += dt
            row[kind] = {"steps_per_s": K / dt, "mean_sweeps": float(np.mean([q["sweeps"] for q in reps_k])),
                         "converged": int(sum(1 for q in reps_k if not (q["flags"] & B.FLAG_NOT_CONVERGED))),
                         "rho": summarize_rho(rhos)}
            if kind != "plain":
                row[kind]["prediction_used"] = int(sum(q["used_prediction"] for q in reps_k))
                row[kind]["prediction_rel_error_mean"] = float(np.nanmean([q["pred_rel_dist"] for q in reps_k]))
        log("learned eval seed %d: sweeps plain %.1f learned %.1f extrapolation %.1f" % (
            row["seed"], row["plain"]["mean_sweeps"], row["learned"]["mean_sweeps"], row["extrap"]["mean_sweeps"]))
        per_seed.append(row)
    net.close()
    net0.close()
    h.close()
    nK = K * args.learned_eval_seeds
    conv = {k: sum(r[k]["converged"] for r in per_seed) for k in ("plain", "learned", "extrap")}
    return {"form": "learned",
            "workload": "advection_ie_variable d=6 n=256 r=32, held-out seeds %d..%d, %d steps each" % (
                args.seed + 2000, args.seed + 2000 + args.learned_eval_seeds - 1, K),
            "train": {"trajectories": len(probs), "fully_converged": len(keep), "steps_each": steps_per,
                      "solver_steps": len(keep) * steps_per, "generation_s": t_data, "adam_steps": len(losses),
                      "batch": 512, "loss_first": losses[0], "loss_last": losses[-1], "seconds": t_train},
            "plain_steps_per_s": nK / tot["plain"], "learned_steps_per_s": nK / tot["learned"],
            "extrapolation_steps_per_s": nK / tot["extrap"],
            "speedup": tot["plain"] / tot["learned"] if conv["learned"] == conv["plain"] == nK else None,
            "network_gain_over_extrapolation": tot["extrap"] / tot["learned"],
            "converged": {k: "%d/%d" % (v, nK) for k, v in conv.items()},
            "rho_max": {k: max(r[k]["rho"]["max"] for r in per_seed) for k in ("plain", "learned", "extrap")},
            "per_seed": per_seed}


def bench_batched(args, log):
    """Batched form: 256 uneven advection instances, n_steps each, adaptive rank up to each
    instance's cap (tau_rank TAU_BATCHED), tol 1e-8, in one persistent launch; a seeded
    sample advanced one launch at a time with the same options (their results equal the
    batched ones bit for bit: both run one workgroup per instance), scaled to all instances
    by a cost model from the batched reports."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    probs = W.batched_instances(args.batch_count, n_steps=args.batch_steps)
    h = B.Handle()
    K = args.batch_steps
    opts = [B.default_opts(tol=TOL, max_sweeps=args.batch_max_sweeps, rank_mode=B.RANK_ADAPTIVE,
                           rank_cap=p.rank_cap, tau_rank=TAU_BATCHED, seed=i) for i, p in enumerate(probs)]
    r0 = [p.f0[0].shape[1] for p in probs]
    fi = [B.to_device(p.f0) for p in probs]
    fo = [B.to_device(p.guess) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = B.cp_als_run_batched(h, [p.A for p in probs], [p.B for p in probs], fi, fo, K, opts, ranks=r0)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    n_inst = len(probs)
    sample = list(range(0, n_inst, max(1, n_inst // args.plain_sample)))[:args.plain_sample]
    t_sample, same = 0.0, True
    for i in sample:
        p = probs[i]
        v, u = B.to_device(p.f0), B.to_device(p.guess)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rr = B.cp_als_run(h, p.A, p.B, v, u, K, opts[i], rank=r0[i], f_init_rank=r0[i])
        torch.cuda.synchronize()
        t_sample += time.perf_counter() - t1
        fr = rr[-1]["final_rank"]
        same = same and rr == reps[i] and all(torch.equal(a[:fr], b[:fr]) for a, b in zip(u, fo[i]))
    cost = [cost_proxy(p, rr) for p, rr in zip(probs, reps)]
    t_plain = t_sample * sum(cost) / sum(cost[i] for i in sample)
    flat = [q for rr in reps for q in rr]
    conv = sum(1 for q in flat if not (q["flags"] & B.FLAG_NOT_CONVERGED))
    rhos = [q["rel_residual"] for q in flat]
    flops = sum(flop_model_ranks(p, rr) for p, rr in zip(probs, reps))
    steps_total = n_inst * K
    log("batched: %d instances x %d steps in %.2f s (%d/%d converged), sample of %d one at a time %.2f s" % (
        n_inst, K, t_batched, conv, steps_total, len(sample), t_sample))
    h.close()
    return {"form": "batched", "instances": n_inst, "steps_each": K,
            "options": "adaptive rank up to each instance's cap, tau_rank %g, tol %g, max_sweeps %d" % (
                TAU_BATCHED, TOL, args.batch_max_sweeps),
            "batched_s": t_batched, "batched_steps_per_s": steps_total / t_batched,
            "plain_sample": len(sample), "plain_s_sample": t_sample, "plain_s_estimated": t_plain,
            "plain_steps_per_s": steps_total / t_plain,
            "speedup": t_plain / t_batched if conv == steps_total else None,
            "sample_results_equal_batched": bool(same),
            "converged": "%d/%d" % (conv, steps_total),
            "rho": summarize_rho(rhos), "rank_final_mean": float(np.mean([q["final_rank"] for q in flat])),
            "rank_growths": int(sum(max(0, q["grown_rank"] - (r0[i] if s == 0 else reps[i][s - 1]["final_rank"]))
                                    for i, rr in enumerate(reps) for s, q in enumerate(rr))),
            "mean_sweeps_per_step": float(np.mean([q["sweeps"] for q in flat])),
            "roofline": {"bound": "mfma", "achieved": flops / t_batched / 1e12, "peak": FP64_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": flops / t_batched / 1e12 / FP64_PEAK_TFLOPS, "flops": flops,
                         "seconds": t_batched}}


def bench_mixed(args, log):
    """Mixed precision on the kinetic Crank-Nicolson workload (d = 6, n = 128, rank 64, 5 Kronecker
    terms), K steps in FP64 and in mixed precision (FP32 matrix-core sweeps, then FP64 sweeps
    to the tolerance) from the same state: rates, FP32/FP64 sweeps, converged steps, rho of
    sampled steps, and the double-double distance of the two final states."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    K = args.mixed_steps
    p = W.kinetic_cn(seed=0, n=128, cap=64, n_steps=K)
    dims, rc = p.A.dims(), p.rank_cap
    res = {}
    for name, prec in (("fp64", B.PREC_FP64), ("mixed", B.PREC_MIXED)):
        V, U = B.to_device(p.f0), B.to_device(p.guess)
        traj = torch.zeros(K * sum(dims) * rc, dtype=torch.float64, device="cuda")
        o = B.default_opts(tol=TOL, max_sweeps=args.max_sweeps, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = B.cp_als_run(h, p.A, p.B, V, U, K, o, traj=traj)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        states = traj_states(traj, K, dims, rc)
        pick = sorted(set(list(range(0, K, max(1, K // 8))) + [K - 1]))
        rhos = [B.cp_residual(h, p.A, p.B, states[s], states[s - 1] if s else V) for s in pick]
        res[name] = (dt, reps, U, rhos)
    dist = rel_distance_dev(h, res["mixed"][2], res["fp64"][2])
    h.close()
    out = {"form": "mixed", "workload": "kinetic_cn d=6 n=128 r=64 (5 Kronecker terms, CN, dt=0.01, tol=1e-8), "
                                        "%d steps" % K}
    for name in ("fp64", "mixed"):
        dt, reps, _, rhos = res[name]
        out[name] = {"steps_per_s": K / dt, "sweeps_total": int(sum(q["sweeps"] for q in reps)),
                     "fp32_sweeps_total": int(sum(q["low_sweeps"] for q in reps)),
                     "converged": "%d/%d" % (sum(1 for q in reps if not (q["flags"] & B.FLAG_NOT_CONVERGED)), K),
                     "rho_sampled": summarize_rho(rhos)}
    conv = all(out[k]["converged"] == "%d/%d" % (K, K) for k in ("fp64", "mixed"))
    out["speedup"] = res["fp64"][0] / res["mixed"][0] if conv else None
    out["rel_distance_final_state"] = dist
    log("mixed: fp64 %.2f steps/s, mixed %.2f steps/s, final distance %.2e" % (
        out["fp64"]["steps_per_s"], out["mixed"]["steps_per_s"], dist))
    return out


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


def _at_point(U, x, b, z):
    """A CP tensor (host factors) at (z, ..., z) by trigonometric interpolation of its
    periodic factor columns."""
    n = U[0].shape[0]
    k = np.fft.fftfreq(n, 1.0 / n)
    ph = np.exp(1j * k * np.pi * (z - x[0]) / b)
    vals = np.ones(U[0].shape[1])
    for u in U:
        vals = vals * np.real(ph @ (np.fft.fft(u, axis=0) / n))
    return float(vals.sum())


def bench_next(args, log):
    """The paper's other steps and experiments, each timed on one MI355X:
      jacobi  the headline workload with damped Jacobi sweeps (Appendix B, damping 1/4)
              against Gauss-Seidel, same tolerance;
      bgk     the linearised BGK equation with a fixed equilibrium (Section 4.2), d = 6,
              n = 64, rank cap 8, Crank-Nicolson with the source dt nu f_eq, 20 steps; the grid
              mass against its exact relaxation;
      spiral  the linear-velocity advection of Section 4.1 at N = 6 (37-term implicit step),
              n = 64, rank 4, 10 Crank-Nicolson steps; the relative error at z* against the
              exact solution;
      ab2     the same generator (36 terms) stepped explicitly by AB2 (Section 3.2), rank cap
              8 (the applied generator L w has a far higher rank than the solution), 20 steps
              of dt = 0.005 from the Crank-Nicolson first level."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    h = B.Handle()
    out = {}
    # --- Jacobi vs Gauss-Seidel on the headline workload
    p = W.advection_ie_variable(seed=args.seed)
    K = 3
    res = {}
    for name, mode in (("gauss_seidel", B.SWEEP_GAUSS_SEIDEL), ("jacobi", B.SWEEP_JACOBI)):
        V, U = B.to_device(p.f0), B.to_device(p.guess)
        o = B.default_opts(tol=TOL, max_sweeps=4000, sweep_mode=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = B.cp_als_run(h, p.A, p.B, V, U, K, o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"steps_per_s": K / dt, "sweeps": [q["sweeps"] for q in reps],
                     "converged": "%d/%d" % (sum(1 for q in reps if not (q["flags"] & B.FLAG_NOT_CONVERGED)), K)}
        res[name]["_U"] = U
    res["rel_distance_final_states"] = rel_distance_dev(h, res["jacobi"].pop("_U"), res["gauss_seidel"].pop("_U"))
    out["jacobi"] = dict(workload="advection_ie_variable d=6 n=256 r=32, %d steps, tol 1e-8" % K, **res)
    log("next: jacobi %.2f steps/s (%s sweeps) vs gauss-seidel %.2f (%s)" % (
        res["jacobi"]["steps_per_s"], res["jacobi"]["sweeps"], res["gauss_seidel"]["steps_per_s"],
        res["gauss_seidel"]["sweeps"]))
    # --- linearised BGK, fixed equilibrium
    p = W.bgk_linear_cn(seed=args.seed, n=64, cap=8, field_rank=3, eps=0.3, dt=0.01)
    K = 20
    src = B.to_device(p.meta["source"])
    U = B.to_device(p.f0)
    G = B.to_device(p.guess)
    o = B.default_opts(tol=TOL, max_sweeps=args.max_sweeps)
    nu, dtb = p.meta["nu"], p.dt
    gam = (1 - 0.5 * nu * dtb) / (1 + 0.5 * nu * dtb)
    mass = lambda F: float(np.sum(np.prod([f.sum(axis=0) for f in F], axis=0)))
    Meq, M0 = mass(p.meta["feq"]), mass(p.f0)
    reps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(K):
        nxt = [g.clone() for g in G]
        reps.append(B.cp_als_step_source(h, p.A, p.B, U, src, nxt, o))
        U, G = nxt, nxt
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    Mk = mass(B.to_host(U))
    out["bgk"] = {"workload": "bgk_linear_cn d=6 (3x+3v) n=64 rank 8, CN dt=0.01, nu=1, %d steps" % K,
                  "steps_per_s": K / dt, "mean_sweeps": float(np.mean([q["sweeps"] for q in reps])),
                  "converged": "%d/%d" % (sum(1 for q in reps if not (q["flags"] & B.FLAG_NOT_CONVERGED)), K),
                  "mass_rel_error_vs_exact_relaxation": abs(Mk - (Meq + gam ** K * (M0 - Meq))) / abs(Meq)}
    log("next: bgk %.2f steps/s" % out["bgk"]["steps_per_s"])
    # --- spiral advection, implicit (37 terms) and explicit AB2 (36 terms)
    zs = 0.698835274542439
    p = W.spiral_advection_cn(seed=args.seed, N=6, n=64, cap=4)
    x, b, C = p.meta["x"], p.meta["b"], p.meta["C"]
    K = 10
    V, U = B.to_device(p.f0), B.to_device(p.guess)
    o = B.default_opts(tol=TOL, max_sweeps=args.max_sweeps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = B.cp_als_run(h, p.A, p.B, V, U, K, o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fe = W.spiral_exact(C, np.full(6, zs), K * p.dt)
    out["spiral"] = {"workload": "spiral advection N=6 n=64 on [-6,6)^6, 37-term CN, rank 4, dt=0.01, %d steps" % K,
                     "steps_per_s": K / dt, "mean_sweeps": float(np.mean([q["sweeps"] for q in reps])),
                     "converged": "%d/%d" % (sum(1 for q in reps if not (q["flags"] & B.FLAG_NOT_CONVERGED)), K),
                     "rel_error_at_zstar": abs(_at_point(B.to_host(U), x, b, zs) - fe) / fe}
    log("next: spiral %.2f steps/s" % out["spiral"]["steps_per_s"])
    dta, K = 0.005, 20
    pa = W.spiral_advection_cn(seed=args.seed, N=6, n=64, dt=dta, cap=8)
    L = pa.meta["L"]
    g1 = B.to_device(pa.guess)
    B.cp_als_step(h, pa.A, pa.B, B.to_device(pa.f0), g1, B.default_opts(tol=1e-12, max_sweeps=300))
    Fp, Fc = B.to_device(pa.f0), [u.clone() for u in g1]
    oa = B.default_opts(tol=1e-12, max_sweeps=300)
    sweeps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        outp = [torch.zeros((8, 64), dtype=torch.float64, device="cuda") for _ in range(6)]
        rank, reps = B.cp_ab2_step(h, L, dta, Fp, Fc, outp, oa)
        sweeps.append(sum(q["sweeps"] for q in reps))
        Fp, Fc = Fc, [u[:rank].contiguous() for u in outp]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fe = W.spiral_exact(C, np.full(6, zs), (K + 1) * dta)
    out["ab2"] = {"workload": "spiral advection N=6 n=64, explicit AB2 with 36-term generator, rank cap 8, "
                              "dt=0.005, %d steps" % K,
                  "steps_per_s": K / dt, "mean_reduction_sweeps": float(np.mean(sweeps)),
                  "rel_error_at_zstar": abs(_at_point(B.to_host(Fc), x, b, zs) - fe) / fe}
    log("next: ab2 %.2f steps/s" % out["ab2"]["steps_per_s"])
    h.close()
    return out


def bench_calibrate(log):
    """A device-to-device copy of 1 GiB (torch): the load whose FETCH_SIZE and WRITE_SIZE
    counters, against the bytes it must move, give the factors that turn the counters into
    HBM bytes."""
    import torch
    n = (1 << 30) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    log("calibrate: copied %d bytes" % (n * 8))
    return {"form": "calibrate", "bytes_read": n * 8, "bytes_written": n * 8}


def bench_plain(args, log):
    """The headline: W untimed warm-up steps, then K steps in one launch timed with HIP events
    on the handle's stream (torch's current stream) and the host clock."""
    import torch
    from paper_1803_10270_amd import binding as B
    from paper_1803_10270_amd import workloads as W
    p = W.advection_ie_variable(seed=args.seed)
    h = B.Handle()
    opts = B.default_opts(tol=p.tol, max_sweeps=args.max_sweeps)
    V = B.to_device(p.f0)
    U = B.to_device(p.guess)
    dims, rc = p.A.dims(), p.rank_cap
    t_w = time.perf_counter()
    if args.warmup > 0:
        B.cp_als_run(h, p.A, p.B, V, U, args.warmup, opts)
    torch.cuda.synchronize()
    log("warmup %d steps: %.2f s" % (args.warmup, time.perf_counter() - t_w))
    V2 = [u.clone() for u in U]
    traj = torch.zeros(args.steps * sum(dims) * rc, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    reports = B.cp_als_run(h, p.A, p.B, V2, U, args.steps, opts, traj=traj)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log("timed %d steps: %.3f s wall, %.3f ms events" % (args.steps, wall, gpu_ms))
    rhos = step_residuals(h, p.A, p.B, V2, traj_states(traj, args.steps, dims, rc))
    h.close()
    return p, reports, wall, gpu_ms, rhos


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--max-sweeps", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the learned, batched and mixed forms")
    ap.add_argument("--form", default="plain",
                    choices=["plain", "learned", "batched", "mixed", "next", "streaming", "calibrate"],
                    help="plain: the headline line; otherwise that leg alone")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-max-sweeps", type=int, default=6000)
    ap.add_argument("--plain-sample", type=int, default=8)
    ap.add_argument("--mixed-steps", type=int, default=50)
    ap.add_argument("--learned-train-trajs", type=int, default=100)
    ap.add_argument("--learned-train-steps", type=int, default=100)
    ap.add_argument("--learned-adam", type=int, default=6000)
    ap.add_argument("--learned-eval-seeds", type=int, default=5)
    ap.add_argument("--learned-eval-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only (sharding the step across GPUs is not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    single = {"learned": bench_learned, "batched": bench_batched, "mixed": bench_mixed, "next": bench_next}
    if args.form in single:
        print(json.dumps(single[args.form](args, log)), flush=True)
        return
    if args.form == "streaming":
        print(json.dumps(bench_streaming(log)), flush=True)
        return
    if args.form == "calibrate":
        print(json.dumps(bench_calibrate(log)), flush=True)
        return
    from paper_1803_10270_amd import binding as B
    p, reports, wall, gpu_ms, rhos = bench_plain(args, log)
    sweeps = [r["sweeps"] for r in reports]
    flops = flop_model(p, reports)
    achieved = flops / (gpu_ms * 1e-3) / 1e12
    conv = int(sum(1 for r in reports if not (r["flags"] & B.FLAG_NOT_CONVERGED)))
    out = {
        "metric": METRIC,
        "value": args.steps / wall,
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
        "config": {"workload": "advection_ie_variable d=6 n=256 r=32 (13 Kronecker terms, implicit Euler, dt=1e-3, "
                               "tol=1e-8, max_sweeps=%d, seed %d)" % (args.max_sweeps, args.seed),
                   "d": 6, "n": 256, "r": 32, "form": "plain", "precision": "fp64"},
        "sweeps_per_step": float(np.mean(sweeps)),
        "pcg_iters_per_update": float(sum(r["pcg_iters"] for r in reports) / max(1, 6 * sum(sweeps))),
        "converged": "%d/%d" % (conv, args.steps),
        "eps_conv_last": reports[-1]["eps_conv"],
        "rho": summarize_rho(rhos),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "als_persistent", "flops_per_launch": flops, "launch_ms": gpu_ms,
                     "source_hash": kernel_source_hash()},
    }
    tr = committed_traffic()
    if tr is not None:
        out["roofline"]["traffic"] = tr["bytes_per_step"] * args.steps
    if not args.no_forms:
        forms = {}
        for name, fn in (("learned", bench_learned), ("batched", bench_batched), ("mixed", bench_mixed),
                         ("next", bench_next)):
            try:
                forms[name] = fn(args, log)
            except Exception as e:   # a form that cannot run is reported, the headline stands
                forms[name] = {"error": repr(e)}
        out["forms"] = forms
        try:
            out["streaming"] = bench_streaming(log)
        except Exception as e:
            out["streaming"] = {"error": repr(e)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
