"""ctypes binding of libcpals.so (C ABI in include/cpals.h).

Argument marshalling only: every step of the method runs in the HIP library.  Device
memory comes from PyTorch tensors; a CP factor panel U_k (n_k x r, column-major) is a
contiguous float64 CUDA tensor of shape (r, n_k).

If the library has not been built, loading raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpals.so")

CP_MAX_DIMS = 8
CP_MAX_OPS = 4

CP_OK, CP_ERR_INVALID_ARG, CP_ERR_SHAPE, CP_ERR_UNSUPPORTED, CP_ERR_HIP, CP_ERR_NOT_CONVERGED, CP_ERR_WORKSPACE = range(7)
FLAG_NOT_CONVERGED, FLAG_PCG_MAXITER, FLAG_REGULARIZED, FLAG_NONFINITE, FLAG_SYNC_TIMEOUT = 1, 2, 4, 8, 16
PREC_FP64, PREC_MIXED = 0, 1
RANK_FIXED, RANK_ADAPTIVE = 0, 1
SWEEP_GAUSS_SEIDEL, SWEEP_JACOBI = 0, 1
OP_KIND = {"identity": 0, "diag": 1, "band": 2, "rank1": 3}


class cp_tensor(C.Structure):
    _fields_ = [("d", C.c_int32), ("r", C.c_int32), ("n", C.c_int32 * CP_MAX_DIMS),
                ("ld", C.c_int32 * CP_MAX_DIMS), ("U", C.c_void_p * CP_MAX_DIMS)]


class cp_op1d(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("half_bw", C.c_int32), ("data", C.c_void_p)]


class cp_operator(C.Structure):
    _fields_ = [("d", C.c_int32), ("n_terms", C.c_int32), ("coef", C.c_void_p), ("op_index", C.c_void_p),
                ("n_ops", C.c_int32 * CP_MAX_DIMS), ("ops", C.c_void_p * CP_MAX_DIMS)]


class cp_als_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_sweeps", C.c_int32), ("precision", C.c_int32),
                ("eps_reg", C.c_double), ("pcg_tol", C.c_double), ("pcg_max_iter", C.c_int32),
                ("rank_mode", C.c_int32), ("tau_rank", C.c_double), ("rank_cap", C.c_int32),
                ("replay_rank", C.c_int32), ("seed", C.c_uint64), ("report_residual", C.c_int32),
                ("sweep_mode", C.c_int32), ("damping", C.c_double)]


class cp_als_report(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("pcg_iters", C.c_int32), ("eps_conv", C.c_double),
                ("fnorm", C.c_double), ("rel_residual", C.c_double), ("flags", C.c_uint32),
                ("final_rank", C.c_int32), ("grown_rank", C.c_int32), ("low_sweeps", C.c_int32)]

    def as_dict(self):
        return {"sweeps": self.sweeps, "pcg_iters": self.pcg_iters, "eps_conv": self.eps_conv,
                "fnorm": self.fnorm, "rel_residual": self.rel_residual, "flags": self.flags,
                "final_rank": self.final_rank, "grown_rank": self.grown_rank, "low_sweeps": self.low_sweeps}


class CpalsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("cpals status %d: %s" % (status, msg))
        self.status = status


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcpals.so is not built (python -m paper_1803_10270_amd.build)")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        P = C.POINTER
        sigs = {
            "cp_create": [P(H), C.c_void_p], "cp_destroy": [H], "cp_set_stream": [H, C.c_void_p],
            "cp_set_workspace": [H, C.c_void_p, C.c_size_t],
            "cp_workspace_size_step": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), P(cp_tensor),
                                       C.c_int32, P(cp_als_opts), P(C.c_size_t)],
            "cp_workspace_size_batched": [H, C.c_int32, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor),
                                          C.c_int32, P(cp_als_opts), P(C.c_size_t)],
            "cp_workspace_size_inner": [H, P(cp_tensor), P(cp_tensor), P(C.c_size_t)],
            "cp_workspace_size_apply": [H, P(cp_operator), P(cp_tensor), P(C.c_size_t)],
            "cp_set_cluster": [H, C.c_int32],
            "cp_inner": [H, P(cp_tensor), P(cp_tensor), C.c_void_p],
            "cp_norm": [H, P(cp_tensor), C.c_void_p],
            "cp_inner_noalloc": [H, P(cp_tensor), P(cp_tensor), C.c_void_p],
            "cp_apply_operator": [H, P(cp_operator), P(cp_tensor), P(cp_tensor)],
            "cp_als_step": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), P(cp_als_opts),
                            P(cp_als_report)],
            "cp_als_run": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), C.c_int32,
                           P(cp_als_opts), P(cp_als_report), C.c_void_p],
            "cp_truncate": [H, P(cp_tensor), P(cp_tensor), P(cp_als_opts), P(cp_als_report)],
            "cp_ab2_step": [H, P(cp_operator), C.c_double, P(cp_tensor), P(cp_tensor), P(cp_tensor), P(cp_als_opts),
                            P(cp_als_report)],
            "cp_workspace_size_ab2": [H, P(cp_operator), P(cp_tensor), P(cp_tensor), P(cp_tensor), P(cp_als_opts),
                                      P(C.c_size_t)],
            "cp_als_run_batched": [H, C.c_int32, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor),
                                   C.c_int32, P(cp_als_opts), P(cp_als_report), C.c_void_p],
            "cp_als_default_opts": [P(cp_als_opts)],
            "cp_residual": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), P(C.c_double)],
            "cp_als_step_adaptive": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), C.c_int32,
                                     C.c_double, P(cp_als_opts), P(cp_als_report), P(C.c_int32), P(C.c_double)],
            "cp_als_step_source": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), P(cp_tensor),
                                   P(cp_als_opts), P(cp_als_report)],
            "cp_batch_plan_create": [H, C.c_int32, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor),
                                     C.c_int32, P(cp_als_opts), P(H)],
            "cp_batch_plan_run": [H, H, P(cp_als_report)],
            "cp_batch_plan_destroy": [H],
            "cp_tune_cluster": [H, P(cp_operator), P(cp_operator), P(cp_tensor), P(cp_tensor), P(cp_als_opts),
                                C.c_int32, P(C.c_int32), P(C.c_float)],
            "cp_tune_save": [H, C.c_char_p], "cp_tune_load": [H, C.c_char_p], "cp_tune_clear": [H],
            # learned warm start (include/cpals_ws.h)
            "cp_ws_create": [H, C.c_void_p, C.c_int32, C.c_int32, P(H)],
            "cp_ws_destroy": [H],
            "cp_ws_get_params": [H, H, C.c_void_p],
            "cp_ws_forward": [H, H, C.c_void_p, C.c_int32, C.c_void_p],
            "cp_ws_gradients": [H, H, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, P(C.c_float)],
            "cp_ws_train_step": [H, H, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.c_float, P(C.c_float)],
            "cp_ws_predict": [H, H, P(cp_tensor), P(cp_tensor), C.c_void_p, P(cp_tensor)],
        }
        for name, argt in sigs.items():
            f = getattr(L, name)
            f.argtypes = argt
            f.restype = C.c_int
        L.cp_last_error.argtypes = [H]
        L.cp_last_error.restype = C.c_char_p
        L.cp_version.argtypes = []
        L.cp_version.restype = C.c_char_p
        L.cp_ws_num_params.argtypes = []
        L.cp_ws_num_params.restype = C.c_int32
        _LIB = L
    return _LIB


# ----------------------------------------------------------------------------------------
# marshalling helpers
# ----------------------------------------------------------------------------------------

def to_device(U: Sequence[np.ndarray], device="cuda"):
    """numpy factor panels (n_k, r) -> list of contiguous float64 (r, n_k) CUDA tensors."""
    import torch
    return [torch.from_numpy(np.ascontiguousarray(np.asarray(u, dtype=np.float64).T)).to(device) for u in U]


def to_host(T) -> List[np.ndarray]:
    return [t.detach().cpu().numpy().T.copy() for t in T]


def tensor_desc(T, rank: Optional[int] = None) -> cp_tensor:
    """List of (r, n_k) float64 CUDA tensors -> cp_tensor (column-major n_k x r panels);
    `rank` (<= r) describes only the first `rank` columns."""
    import torch
    desc = cp_tensor()
    desc.d = len(T)
    desc.r = int(T[0].shape[0])
    for k, t in enumerate(T):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
            raise ValueError("factor panels must be contiguous float64 CUDA tensors of shape (r, n)")
        if int(t.shape[0]) != desc.r:
            raise ValueError("all panels must have the same rank")
        desc.n[k] = int(t.shape[1])
        desc.ld[k] = int(t.shape[1])
        desc.U[k] = t.data_ptr()
    if rank is not None:
        if not 1 <= rank <= desc.r:
            raise ValueError("rank must be in 1..%d" % desc.r)
        desc.r = int(rank)
    return desc


class OperatorDesc:
    """Keeps the host arrays of a separable operator alive for the duration of a call."""

    def __init__(self, L):
        self.coef = np.ascontiguousarray(L.coef, dtype=np.float64)
        self.idx = np.ascontiguousarray(L.op_index, dtype=np.int32)
        self.datas = []
        self.op_arrays = []
        self.desc = cp_operator()
        self.desc.d = L.d
        self.desc.n_terms = L.n_terms
        self.desc.coef = self.coef.ctypes.data
        self.desc.op_index = self.idx.ctypes.data
        for k, ops_k in enumerate(L.ops):
            arr = (cp_op1d * len(ops_k))()
            for a, op in enumerate(ops_k):
                arr[a].kind = OP_KIND[op.kind]
                arr[a].n = op.n
                arr[a].half_bw = op.half_bw
                if op.data is not None:
                    dat = np.ascontiguousarray(op.data, dtype=np.float64).reshape(-1)
                    self.datas.append(dat)
                    arr[a].data = dat.ctypes.data
                else:
                    arr[a].data = None
            self.op_arrays.append(arr)
            self.desc.n_ops[k] = len(ops_k)
            self.desc.ops[k] = C.cast(arr, C.c_void_p)


def default_opts(**kw) -> cp_als_opts:
    o = cp_als_opts()
    lib().cp_als_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Handle:
    """A library handle bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = C.c_void_p()
        st = lib().cp_create(C.byref(self.h), C.c_void_p(stream.cuda_stream))
        if st != CP_OK:
            raise CpalsError(st, "cp_create failed")

    def set_cluster(self, max_workgroups: int) -> None:
        """Workgroups that may share one problem (1 = one workgroup per problem)."""
        self.check(lib().cp_set_cluster(self.h, int(max_workgroups)))

    def set_workspace(self, buf) -> None:
        """Use the caller's device buffer (a CUDA tensor, kept alive here) as the workspace;
        None returns to the library's own."""
        self._ws = buf
        if buf is None:
            self.check(lib().cp_set_workspace(self.h, None, 0))
        else:
            self.check(lib().cp_set_workspace(self.h, C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()))

    def close(self):
        if self.h:
            lib().cp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st, allow_not_converged=False):
        if st == CP_OK or (allow_not_converged and st == CP_ERR_NOT_CONVERGED):
            return st
        raise CpalsError(st, lib().cp_last_error(self.h).decode())


# ----------------------------------------------------------------------------------------
# the C ABI, one Python function per entry point
# ----------------------------------------------------------------------------------------

def cp_inner(h: Handle, x, y, out) -> None:
    """out (1-element float64 CUDA tensor) <- <x, y>."""
    xd, yd = tensor_desc(x), tensor_desc(y)
    h.check(lib().cp_inner(h.h, C.byref(xd), C.byref(yd), C.c_void_p(out.data_ptr())))


def cp_inner_noalloc(h: Handle, x, y, out) -> None:
    """out (1-element float64 CUDA tensor) <- <x, y> without allocating device memory."""
    xd, yd = tensor_desc(x), tensor_desc(y)
    h.check(lib().cp_inner_noalloc(h.h, C.byref(xd), C.byref(yd), C.c_void_p(out.data_ptr())))


def cp_norm(h: Handle, x, out) -> None:
    xd = tensor_desc(x)
    h.check(lib().cp_norm(h.h, C.byref(xd), C.c_void_p(out.data_ptr())))


def cp_apply_operator(h: Handle, L, x, y) -> None:
    """y (rank n_terms * x.r panels) <- L x."""
    Ld = OperatorDesc(L)
    xd, yd = tensor_desc(x), tensor_desc(y)
    h.check(lib().cp_apply_operator(h.h, C.byref(Ld.desc), C.byref(xd), C.byref(yd)))


def cp_als_step(h: Handle, A, B, f_n, f_next, opts: Optional[cp_als_opts] = None, rank: Optional[int] = None,
                f_n_rank: Optional[int] = None) -> dict:
    """One implicit step; f_next is in/out (guess in, solution out).  Returns the report.
    Adaptive rank: f_next's panels hold opts.rank_cap columns and the first `rank` are the
    guess; the report's final_rank says how many hold the result."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, gd = tensor_desc(f_n, f_n_rank), tensor_desc(f_next, rank)
    rep = cp_als_report()
    h.check(lib().cp_als_step(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(gd), C.byref(opts),
                              C.byref(rep)), allow_not_converged=True)
    return rep.as_dict()


def cp_als_run(h: Handle, A, B, f_init, f_io, n_steps: int, opts: Optional[cp_als_opts] = None,
               traj=None, rank: Optional[int] = None, f_init_rank: Optional[int] = None) -> List[dict]:
    """n_steps implicit steps in one launch; f_io in/out.  traj: optional float64 CUDA buffer of
    n_steps * sum_k n_k r elements receiving every step's factors (r = the panels' columns).
    rank / f_init_rank: the guess and f_init use only their first columns (adaptive rank)."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, gd = tensor_desc(f_init, f_init_rank), tensor_desc(f_io, rank)
    reps = (cp_als_report * n_steps)()
    if traj is not None:
        import torch
        need = n_steps * sum(int(t.shape[1]) * int(f_io[0].shape[0]) for t in f_io)
        if traj.dtype != torch.float64 or not traj.is_cuda or not traj.is_contiguous() or traj.numel() < need:
            raise ValueError("traj must be a contiguous float64 CUDA buffer of at least %d elements" % need)
    tp = C.c_void_p(traj.data_ptr()) if traj is not None else C.c_void_p()
    h.check(lib().cp_als_run(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(gd), n_steps,
                             C.byref(opts), reps, tp), allow_not_converged=True)
    return [r.as_dict() for r in reps]


def cp_truncate(h: Handle, g, f, opts: Optional[cp_als_opts] = None) -> dict:
    opts = default_opts() if opts is None else opts
    gd, fd = tensor_desc(g), tensor_desc(f)
    rep = cp_als_report()
    h.check(lib().cp_truncate(h.h, C.byref(gd), C.byref(fd), C.byref(opts), C.byref(rep)), allow_not_converged=True)
    return rep.as_dict()


def _opts_array(opts, count):
    """One cp_als_opts per problem from None, a single struct or a list of them."""
    if opts is None:
        opts = default_opts()
    if isinstance(opts, cp_als_opts):
        opts = [opts] * count
    if len(opts) != count:
        raise ValueError("need one cp_als_opts per problem")
    return (cp_als_opts * count)(*opts)


def cp_ab2_step(h: Handle, L, dt: float, f_prev, f_cur, f_next, opts: Optional[cp_als_opts] = None):
    """One explicit AB2 step (apply, add, rank-reduce) into f_next (panels of cap columns).
    Returns (rank of the result, the three reductions' reports)."""
    opts = default_opts() if opts is None else opts
    Ld = OperatorDesc(L)
    pd, cd, nd = tensor_desc(f_prev), tensor_desc(f_cur), tensor_desc(f_next)
    reps = (cp_als_report * 3)()
    h.check(lib().cp_ab2_step(h.h, C.byref(Ld.desc), float(dt), C.byref(pd), C.byref(cd), C.byref(nd), C.byref(opts),
                              reps), allow_not_converged=True)
    return int(nd.r), [r.as_dict() for r in reps]


def cp_als_run_batched(h: Handle, As, Bs, f_inits, f_ios, n_steps: int, opts=None,
                       ranks: Optional[Sequence[int]] = None, trajs=None) -> List[List[dict]]:
    """opts: one cp_als_opts for all problems or a list (one each); ranks: guess ranks
    (adaptive rank: the panels hold opts[i].rank_cap columns); trajs: None or one float64
    CUDA buffer (or None) per problem receiving its steps' factors as cp_als_run's traj."""
    count = len(As)
    o_arr = _opts_array(opts, count)
    Ads = [OperatorDesc(a) for a in As]
    Bds = [OperatorDesc(b) for b in Bs]
    A_arr = (cp_operator * count)(*[a.desc for a in Ads])
    B_arr = (cp_operator * count)(*[b.desc for b in Bds])
    fi = (cp_tensor * count)(*[tensor_desc(f) for f in f_inits])
    fo = (cp_tensor * count)(*[tensor_desc(f, None if ranks is None else ranks[i]) for i, f in enumerate(f_ios)])
    reps = (cp_als_report * (count * n_steps))()
    tp = None
    if trajs is not None:
        if len(trajs) != count:
            raise ValueError("need one trajectory buffer (or None) per problem")
        tp = (C.c_void_p * count)(*[t.data_ptr() if t is not None else None for t in trajs])
    h.check(lib().cp_als_run_batched(h.h, count, A_arr, B_arr, fi, fo, n_steps, o_arr, reps, tp),
            allow_not_converged=True)
    return [[reps[i * n_steps + s].as_dict() for s in range(n_steps)] for i in range(count)]


def cp_als_step_source(h: Handle, A, B, f_n, source, f_next, opts: Optional[cp_als_opts] = None) -> dict:
    """One implicit step A f_{n+1} = B f_n + source; f_next is in/out (guess in, solution out)."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, sd, gd = tensor_desc(f_n), tensor_desc(source), tensor_desc(f_next)
    rep = cp_als_report()
    h.check(lib().cp_als_step_source(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(sd), C.byref(gd),
                                     C.byref(opts), C.byref(rep)), allow_not_converged=True)
    return rep.as_dict()


def cp_residual(h: Handle, A, B, f, f_n, f_rank: Optional[int] = None, f_n_rank: Optional[int] = None) -> float:
    """||A f - B f_n|| / ||B f_n|| on the device (double-double)."""
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, nd = tensor_desc(f, f_rank), tensor_desc(f_n, f_n_rank)
    out = C.c_double(0.0)
    h.check(lib().cp_residual(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(nd), C.byref(out)))
    return float(out.value)


def cp_als_step_adaptive(h: Handle, A, B, f_n, f_next, r_start: int, tau: float,
                         opts: Optional[cp_als_opts] = None) -> dict:
    """Implicit step growing the rank from r_start (f_next holds cap = f_next rank columns;
    its first r_start are the guess) until the relative residual is <= tau.  Returns the
    report with 'final_rank' and 'rel_residual'."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, gd = tensor_desc(f_n), tensor_desc(f_next)
    rep = cp_als_report()
    fr, rho = C.c_int32(0), C.c_double(0.0)
    h.check(lib().cp_als_step_adaptive(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(gd), r_start, tau,
                                       C.byref(opts), C.byref(rep), C.byref(fr), C.byref(rho)),
            allow_not_converged=True)
    out = rep.as_dict()
    out.update(final_rank=int(fr.value), rel_residual=float(rho.value))
    return out


def cp_tune_cluster(h: Handle, A, B, f_n, guess, opts: Optional[cp_als_opts] = None, sweeps: int = 3):
    """Times every admissible cluster size on this problem, records the fastest in the
    handle's table and returns (W, milliseconds for `sweeps` sweeps)."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, gd = tensor_desc(f_n), tensor_desc(guess)
    w, ms = C.c_int32(0), C.c_float(0.0)
    h.check(lib().cp_tune_cluster(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd), C.byref(gd), C.byref(opts),
                                  sweeps, C.byref(w), C.byref(ms)))
    return int(w.value), float(ms.value)


def workspace_size_step(h: Handle, A, B, f_init, f_io, n_steps: int = 1, opts: Optional[cp_als_opts] = None,
                        source=None, rank: Optional[int] = None) -> int:
    """Bytes of workspace cp_als_run / cp_als_step (/ cp_als_step_source with `source`) need."""
    opts = default_opts() if opts is None else opts
    Ad, Bd = OperatorDesc(A), OperatorDesc(B)
    fd, gd = tensor_desc(f_init), tensor_desc(f_io, rank)
    sd = tensor_desc(source) if source is not None else None
    out = C.c_size_t(0)
    h.check(lib().cp_workspace_size_step(h.h, C.byref(Ad.desc), C.byref(Bd.desc), C.byref(fd),
                                         C.byref(sd) if sd is not None else None, C.byref(gd), n_steps, C.byref(opts),
                                         C.byref(out)))
    return int(out.value)


def workspace_size_inner(h: Handle, x, y) -> int:
    out = C.c_size_t(0)
    xd, yd = tensor_desc(x), tensor_desc(y)
    h.check(lib().cp_workspace_size_inner(h.h, C.byref(xd), C.byref(yd), C.byref(out)))
    return int(out.value)


def workspace_size_apply(h: Handle, L, x) -> int:
    out = C.c_size_t(0)
    Ld = OperatorDesc(L)
    xd = tensor_desc(x)
    h.check(lib().cp_workspace_size_apply(h.h, C.byref(Ld.desc), C.byref(xd), C.byref(out)))
    return int(out.value)


def cp_tune_save(h: Handle, path: str):
    h.check(lib().cp_tune_save(h.h, path.encode()))


def cp_tune_load(h: Handle, path: str):
    h.check(lib().cp_tune_load(h.h, path.encode()))


def cp_tune_clear(h: Handle):
    h.check(lib().cp_tune_clear(h.h))


class BatchPlan:
    """A batched run captured once in a HIP graph (cp_batch_plan_*): the tensors given here
    must stay allocated while the plan lives; run() replays the captured run on their current
    contents (results into f_ios) and returns the reports."""

    def __init__(self, h: Handle, As, Bs, f_inits, f_ios, n_steps: int, opts=None):
        self.h, self.count, self.n_steps = h, len(As), n_steps
        o_arr = _opts_array(opts, self.count)
        self._keep = (list(f_inits), list(f_ios))
        Ads = [OperatorDesc(a) for a in As]
        Bds = [OperatorDesc(b) for b in Bs]
        A_arr = (cp_operator * self.count)(*[a.desc for a in Ads])
        B_arr = (cp_operator * self.count)(*[b.desc for b in Bds])
        fi = (cp_tensor * self.count)(*[tensor_desc(f) for f in f_inits])
        fo = (cp_tensor * self.count)(*[tensor_desc(f) for f in f_ios])
        self.plan = C.c_void_p()
        h.check(lib().cp_batch_plan_create(h.h, self.count, A_arr, B_arr, fi, fo, n_steps, o_arr,
                                           C.byref(self.plan)))

    def run(self) -> List[List[dict]]:
        reps = (cp_als_report * (self.count * self.n_steps))()
        self.h.check(lib().cp_batch_plan_run(self.h.h, self.plan, reps), allow_not_converged=True)
        return [[reps[i * self.n_steps + s].as_dict() for s in range(self.n_steps)] for i in range(self.count)]

    def close(self):
        if self.plan:
            lib().cp_batch_plan_destroy(self.plan)
            self.plan = C.c_void_p()


# ----------------------------------------------------------------------------------------
# learned warm start (include/cpals_ws.h)
# ----------------------------------------------------------------------------------------

def ws_num_params() -> int:
    return int(lib().cp_ws_num_params())


class WarmStartNet:
    """The per-column CNN of include/cpals_ws.h (device memory owned by the library)."""

    def __init__(self, h: Handle, params: np.ndarray, n: int, max_batch: int):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != ws_num_params():
            raise ValueError("expected %d parameters, got %d" % (ws_num_params(), p.size))
        self.h = h
        self.n = n
        self.max_batch = max_batch
        self.net = C.c_void_p()
        h.check(lib().cp_ws_create(h.h, p.ctypes.data_as(C.c_void_p), n, max_batch, C.byref(self.net)))

    def close(self):
        if self.net:
            lib().cp_ws_destroy(self.net)
            self.net = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(ws_num_params(), dtype=np.float32)
        self.h.check(lib().cp_ws_get_params(self.h.h, self.net, out.ctypes.data_as(C.c_void_p)))
        return out

    def forward(self, x, y) -> None:
        """y[B, n] (float32 CUDA) <- network(x[B, 3, n] float32 CUDA)."""
        _check_f32(x, 3)
        _check_f32(y, 2)
        B = x.shape[0]
        if x.shape[1:] != (3, self.n) or tuple(y.shape) != (B, self.n):
            raise ValueError("shapes must be x [B, 3, n], y [B, n]")
        self.h.check(lib().cp_ws_forward(self.h.h, self.net, C.c_void_p(x.data_ptr()), B, C.c_void_p(y.data_ptr())))

    def gradients(self, x, target, grad) -> float:
        """grad (float32 CUDA, n_params) <- d loss / d params; returns the loss."""
        _check_f32(x, 3)
        _check_f32(target, 2)
        _check_f32(grad, 1)
        B = x.shape[0]
        if x.shape[1:] != (3, self.n) or tuple(target.shape) != (B, self.n) or grad.numel() != ws_num_params():
            raise ValueError("shapes must be x [B, 3, n], target [B, n], grad [n_params]")
        loss = C.c_float()
        self.h.check(lib().cp_ws_gradients(self.h.h, self.net, C.c_void_p(x.data_ptr()), C.c_void_p(target.data_ptr()),
                                           B, C.c_void_p(grad.data_ptr()), C.byref(loss)))
        return float(loss.value)

    def train_step(self, traj, samples: np.ndarray, coef: np.ndarray, lr: float) -> float:
        """One Adam step; traj float64 CUDA [T, C, n]; samples int32 [B, 2] of (t, c); coef [C]."""
        import torch
        if traj.dtype != torch.float64 or not traj.is_cuda or not traj.is_contiguous() or traj.dim() != 3:
            raise ValueError("traj must be a contiguous float64 CUDA tensor [T, C, n]")
        T, Cc, n = traj.shape
        if n != self.n:
            raise ValueError("traj has n=%d, network n=%d" % (n, self.n))
        smp = np.ascontiguousarray(samples, dtype=np.int32).reshape(-1, 2)
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        if cf.size != Cc:
            raise ValueError("coef needs one value per column")
        loss = C.c_float()
        self.h.check(lib().cp_ws_train_step(self.h.h, self.net, C.c_void_p(traj.data_ptr()), T, Cc,
                                            smp.ctypes.data_as(C.c_void_p), cf.ctypes.data_as(C.c_void_p), smp.shape[0],
                                            float(lr), C.byref(loss)))
        return float(loss.value)

    def predict(self, f_prev, f_cur, coef: np.ndarray, f_guess) -> None:
        """f_guess <- the network's prediction of the next factors from (f_prev, f_cur)."""
        cf = np.ascontiguousarray(coef, dtype=np.float64)
        tp, tc, tg = tensor_desc(f_prev), tensor_desc(f_cur), tensor_desc(f_guess)
        if cf.size != tc.d:
            raise ValueError("coef needs one value per dimension")
        self.h.check(lib().cp_ws_predict(self.h.h, self.net, C.byref(tp), C.byref(tc), cf.ctypes.data_as(C.c_void_p),
                                         C.byref(tg)))


def _check_f32(t, ndim):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != ndim:
        raise ValueError("expected a contiguous float32 CUDA tensor with %d dimensions" % ndim)
