"""A plain device-to-device copy of known size, used to calibrate HBM byte
counters (rocprofv3 FETCH_SIZE / WRITE_SIZE) against algorithmic bytes.

    python -m paper_1812_05711_amd.hbm_copy [--mib 1024] [--reps 5]

Each repetition copies --mib MiB: it reads and writes that many bytes.
"""

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.reps} x {a.mib} MiB", flush=True)


if __name__ == "__main__":
    main()
