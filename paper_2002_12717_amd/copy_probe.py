"""Calibration program for HBM traffic counters: copies a 1 GiB device buffer
(torch copy kernel) a fixed number of times.  A counter run over this program
gives the counter reading that corresponds to a known number of bytes read
(1 GiB per copy) and written (1 GiB per copy)."""
import sys

import torch


def main(reps: int = 4, nbytes: int = 1 << 30):
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {reps} x {nbytes} bytes", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
