"""Host-side checks of the C ABI (no GPU needed): the built library loads, exports every
function that include/cpals.h declares, and the ctypes structures of the binding have the
same layout as the C structures."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1803_10270_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cpals.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("cp_inner", "cp_norm", "cp_apply_operator", "cp_als_step", "cp_truncate", "cp_als_run",
                     "cp_als_run_batched", "cp_create", "cp_destroy", "cp_set_workspace", "cp_residual",
                     "cp_workspace_size_step", "cp_workspace_size_batched", "cp_workspace_size_inner",
                     "cp_workspace_size_apply"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.cp_version().startswith(b"cpals")


def test_default_options():
    o = B.default_opts()
    assert o.tol == 1e-8 and o.max_sweeps == 200 and o.eps_reg == 1e-10 and o.precision == B.PREC_FP64
    assert o.rank_mode == B.RANK_FIXED and o.replay_rank == -1 and o.rank_cap == 64 and o.report_residual == 0
    assert o.tau_rank == 1e-6 and o.seed == 0 and o.sweep_mode == B.SWEEP_GAUSS_SEIDEL and o.damping == 0.25


def test_struct_layouts_match_c():
    """Compile a tiny C program against the header and compare sizeof/offsetof."""
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "cpals.h"
#define P(T, F) printf(#T "." #F " %zu\n", offsetof(T, F));
int main(void) {
  printf("cp_tensor %zu\ncp_op1d %zu\ncp_operator %zu\ncp_als_opts %zu\ncp_als_report %zu\n",
         sizeof(cp_tensor), sizeof(cp_op1d), sizeof(cp_operator), sizeof(cp_als_opts), sizeof(cp_als_report));
  P(cp_tensor, U) P(cp_tensor, ld) P(cp_operator, ops) P(cp_operator, n_ops) P(cp_als_opts, precision)
  P(cp_als_opts, pcg_tol) P(cp_als_report, flags) P(cp_als_report, fnorm) P(cp_op1d, data)
  P(cp_als_opts, rank_mode) P(cp_als_opts, tau_rank) P(cp_als_opts, rank_cap) P(cp_als_opts, replay_rank)
  P(cp_als_opts, seed) P(cp_als_opts, report_residual) P(cp_als_report, rel_residual)
  P(cp_als_opts, sweep_mode) P(cp_als_opts, damping)
  P(cp_als_report, final_rank) P(cp_als_report, grown_rank) P(cp_als_report, low_sweeps)
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "t.c")
        exe = os.path.join(td, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I" + os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    vals = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    vals = {k: int(v) for k, v in vals.items()}
    assert vals["cp_tensor"] == C.sizeof(B.cp_tensor)
    assert vals["cp_op1d"] == C.sizeof(B.cp_op1d)
    assert vals["cp_operator"] == C.sizeof(B.cp_operator)
    assert vals["cp_als_opts"] == C.sizeof(B.cp_als_opts)
    assert vals["cp_als_report"] == C.sizeof(B.cp_als_report)
    assert vals["cp_tensor.U"] == B.cp_tensor.U.offset
    assert vals["cp_tensor.ld"] == B.cp_tensor.ld.offset
    assert vals["cp_operator.ops"] == B.cp_operator.ops.offset
    assert vals["cp_operator.n_ops"] == B.cp_operator.n_ops.offset
    assert vals["cp_als_opts.precision"] == B.cp_als_opts.precision.offset
    assert vals["cp_als_opts.pcg_tol"] == B.cp_als_opts.pcg_tol.offset
    assert vals["cp_als_report.flags"] == B.cp_als_report.flags.offset
    assert vals["cp_als_report.fnorm"] == B.cp_als_report.fnorm.offset
    assert vals["cp_op1d.data"] == B.cp_op1d.data.offset
    for f in ("rank_mode", "tau_rank", "rank_cap", "replay_rank", "seed", "report_residual", "sweep_mode", "damping"):
        assert vals["cp_als_opts." + f] == getattr(B.cp_als_opts, f).offset, f
    for f in ("rel_residual", "final_rank", "grown_rank", "low_sweeps"):
        assert vals["cp_als_report." + f] == getattr(B.cp_als_report, f).offset, f


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(B, "_LIB", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libcpals.so")
    with pytest.raises(RuntimeError):
        B.lib()
