"""Calibration load for hardware byte counters: one device-to-device copy of a known size.

    python paper_1803_10270_amd/copy_probe.py [MiB]

Under rocprofv3 --pmc FETCH_SIZE (or WRITE_SIZE) the counter value of this copy, compared
with the bytes it must move, gives the factor that converts the counter into HBM bytes."""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print("copied %d bytes" % (n * 8), flush=True)


if __name__ == "__main__":
    main()
