"""Calibration workload for HBM byte counters: a plain device copy of known size.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (and separately ``WRITE_SIZE``); the
counter values of these copies divided by the bytes they must move give the
scale factor applied to the stencil kernel's counters (pmc_summary.py).
"""
import sys

import torch

BYTES = 1 << 30          # 1 GiB read + 1 GiB written per copy
REPEATS = 3


def main():
    n = BYTES // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(REPEATS):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {REPEATS} x {BYTES} bytes", file=sys.stderr)


if __name__ == "__main__":
    main()
