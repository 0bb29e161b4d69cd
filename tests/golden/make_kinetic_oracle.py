"""Writes kinetic_cn_n128_r64_2sweeps.npz: the FP64 oracle's result of two ALS sweeps (tol 0)
of the first Crank-Nicolson step of the linearised kinetic workload at d = 6 (3 space + 3
velocity dimensions), n = 128, rank 64, seed 0 -- the shape of the mixed-precision
benchmark.  The oracle needs minutes for it on the host, so the GPU test reads the stored
result.  Calls only the seeded input generator and oracle/.

    python tests/golden/make_kinetic_oracle.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cpals_oracle as O  # noqa: E402
from paper_1803_10270_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "kinetic_cn_n128_r64_2sweeps.npz")


def main():
    p = W.kinetic_cn(seed=0, n=128, cap=64)
    U, rep = O.als_step(p.A, p.B, p.f0, p.guess, tol=0.0, max_sweeps=2)
    np.savez_compressed(OUT, **{"U%d" % k: u for k, u in enumerate(U)}, sweep_eps=np.array(rep["sweep_eps"]))
    print(OUT, rep["sweep_eps"])


if __name__ == "__main__":
    main()
