"""Single launches of the library's kernels at the benchmark's sizes, for
hardware-counter profiles (rocprofv3 --pmc), next to a plain copy of known
size that calibrates the byte counters.

    python3 -m paper_1503_05464_amd.profile_kernels [--n 65536] [--ncols 64]

runs, in order:
* an elementwise copy of 4 GiB (torch multiply by one, a kernel rather
  than a DMA copy) -- reads 4 GiB, writes 4 GiB;
* hss_sample on the N = n FP32 Gaussian-kernel matrix of the benchmark
  (k-d ordered points, leaf 256, leaf blocks masked), ncols FP64 random
  columns, both products (S^r and S^c: two sample_kernel launches), the
  configuration of one growth step of the benchmark's compression.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--ncols", type=int, default=64)
    ap.add_argument("--leaf", type=int, default=256)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1503_05464_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    print("[profile] copy of 4 GiB", flush=True)
    src = torch.ones(1 << 29, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()

    n = args.n
    p = W.cube_points(n, 4)
    p = p[W.kd_order(p, args.leaf)]
    A = W.device_kernel_matrix("gauss", p, torch.float32, dev)
    lo = np.arange(0, n, args.leaf)
    leaf_of = torch.from_numpy((np.arange(n) // args.leaf).astype(np.int32)).to(dev)
    assert len(lo) == (n + args.leaf - 1) // args.leaf
    Rr = P.hss_random_normal(0, 0, n, 0, args.ncols)
    Rc = P.hss_random_normal(0, 1, n, 0, args.ncols)
    torch.cuda.synchronize()
    print(f"[profile] hss_sample n={n} ncols={args.ncols} (two sample_kernel launches)", flush=True)
    P.hss_sample(A, Rr, Rc, leaf_of)
    torch.cuda.synchronize()
    print("[profile] done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
