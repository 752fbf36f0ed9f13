"""Tile autotuner of the batched FP64 GEMM (the kernel of every per-node
product: local samples and R_tau in compression, the sweeps of the matvec,
the ULV factor and solve updates).

A launch's size class is its widest N and its largest M, bucketed (N <= 16,
<= 32, <= 64, > 64; M <= 32, <= 128, > 128).  For every class this script
builds seeded synthetic batches of that class -- many problems with sizes
drawn inside the class's buckets, K of the order of M as in the library's
products -- times each tile shape of the kernel (hss_gemm_batched with a
forced variant; HIP events on the stream around launches queued behind a
long product, so that only device time is measured), checks
each result against the default shape's, and writes the fastest shape of
each class into csrc/gemm_tiles.inc together with the measured times.
Rebuild the library afterwards (build.py).

    python -m paper_1503_05464_amd.autotune [--reps 20] [--dry-run] [--out FILE]

Runs on the GPU.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "gemm_tiles.inc")
N_BUCKETS = [(1, 16), (17, 32), (33, 64), (65, 256)]
M_BUCKETS = [(4, 32), (33, 128), (129, 600)]
SHAPES = ["64 x 64", "64 x 16", "128 x 16", "32 x 32", "64 x 32", "128 x 32", "16 x 64"]


def _batches(cls: int, seed: int):
    """Two batches of one class: many problems (a level of many nodes) and a
    few larger ones (the top of a tree)."""
    import numpy as np
    import torch

    nb, mb = divmod(cls, 3)
    (n_lo, n_hi), (m_lo, m_hi) = N_BUCKETS[nb], M_BUCKETS[mb]
    g = np.random.default_rng(seed)
    out = []
    for count in (384, 6):
        As, Bs, Cs, tr = [], [], [], []
        for q in range(count):
            M = int(g.integers(m_lo, m_hi + 1)) if q else m_hi  # the largest M of the class
            N = int(g.integers(n_lo, n_hi + 1)) if q else n_hi
            K = int(g.integers(max(4, M // 2), M + 33))
            t = bool(g.integers(0, 2))
            A = torch.randn((K, M) if t else (M, K), dtype=torch.float64, device="cuda")
            As.append(A)
            Bs.append(torch.randn((K, N), dtype=torch.float64, device="cuda"))
            Cs.append(torch.randn((M, N), dtype=torch.float64, device="cuda"))
            tr.append(t)
        out.append((As, Bs, Cs, tr))
    return out


def _args(P, batch):
    """The C arguments of hss_gemm_batched for a batch, marshalled once."""
    import ctypes as C

    import numpy as np

    As, Bs, Cs, tr = batch
    arr = [np.array([c.shape[0] for c in Cs], dtype=np.int32), np.array([c.shape[1] for c in Cs], dtype=np.int32),
           np.array([b.shape[0] for b in Bs], dtype=np.int32),
           np.array([a.data_ptr() for a in As], dtype=np.uint64), np.array([a.stride(0) for a in As], dtype=np.int64),
           np.array(tr, dtype=np.int32),
           np.array([b.data_ptr() for b in Bs], dtype=np.uint64), np.array([b.stride(0) for b in Bs], dtype=np.int64),
           np.array([c.data_ptr() for c in Cs], dtype=np.uint64), np.array([c.stride(0) for c in Cs], dtype=np.int64)]
    return arr, [C.c_void_p(a.ctypes.data) for a in arr]


def _time(P, batch, variant: int, reps: int, blocker) -> float:
    """Device time of one launch (with its descriptor copy): the launches are
    queued behind a long product on the stream, so the time the host takes to
    issue them does not show between the events."""
    import ctypes as C

    import torch

    keep, a = _args(P, batch)
    n = len(batch[0])
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib = P.lib()

    def call():
        st = lib.hss_gemm_batched(n, *a, 1.0, 0.5, variant, stream)
        if st != 0:
            raise RuntimeError(lib.hss_last_error().decode())

    s = torch.cuda.current_stream()
    for _ in range(3):
        call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(6):
        blocker = blocker @ blocker
        blocker /= blocker.abs().max()
    e0.record(s)
    for _ in range(reps):
        call()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps  # us per launch


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--dry-run", action="store_true", help="print the table, do not write it")
    ap.add_argument("--out", default=TABLE, help="where to write the table (default: csrc/gemm_tiles.inc)")
    args = ap.parse_args()

    import torch

    import paper_1503_05464_amd as P

    nvar = P.hss_gemm_variants()
    blocker = torch.randn((6144, 6144), dtype=torch.float64, device="cuda")
    best, lines = [], []
    for cls in range(len(N_BUCKETS) * len(M_BUCKETS)):
        batches = _batches(cls, 100 + cls)
        # every shape computes the same products (checked on the first batch)
        As, Bs, Cs0, tr = batches[0]
        ref = [c.clone() for c in Cs0]
        P.hss_gemm_batched(As, Bs, ref, tr, 1.0, 0.5, 0)
        for v in range(1, nvar):
            got = [c.clone() for c in Cs0]
            P.hss_gemm_batched(As, Bs, got, tr, 1.0, 0.5, v)
            for a, b in zip(got, ref):
                if not torch.allclose(a, b, rtol=1e-12, atol=1e-12 * float(b.abs().max()) + 1e-300):
                    raise RuntimeError(f"class {cls}: shape {SHAPES[v]} disagrees with 64 x 64")
        # time: the sum over the class's two batches
        us = [sum(_time(P, b, v, args.reps, blocker) for b in batches) for v in range(nvar)]
        v_best = min(range(nvar), key=lambda v: us[v])
        best.append(v_best)
        nb, mb = divmod(cls, 3)
        desc = f"N {N_BUCKETS[nb][0]}..{N_BUCKETS[nb][1]}, M {M_BUCKETS[mb][0]}..{M_BUCKETS[mb][1]}"
        line = f"class {cls:2d} ({desc}): " + ", ".join(f"{SHAPES[v]} {us[v]:.1f}" for v in range(nvar)) + \
               f" -> {SHAPES[v_best]}"
        print(line, flush=True)
        lines.append(line)
    props = torch.cuda.get_device_properties(0)
    dev = f"{getattr(props, 'gcnArchName', '').split(':')[0] or props.name} ({props.name})"
    text = (
        "// Tile shape of the batched FP64 GEMM per size class of a launch, written by\n"
        "// paper_1503_05464_amd/autotune.py from measured launch times.\n"
        "// class = 3 * (N bucket) + (M bucket), N = the widest problem's columns\n"
        "// (<= 16, <= 32, <= 64, > 64), M = the largest problem's rows (<= 32, <= 128,\n"
        "// > 128).  Entries index kGVariants in kernels_gemm.hip:\n"
        "//   " + ", ".join(f"{v}: {SHAPES[v]}" for v in range(nvar)) + ".\n"
        f"// Measured on {dev}: microseconds per launch, summed over a batch of 384\n"
        "// problems and a batch of 6 (synthetic sizes inside the class), per shape:\n"
        + "".join(f"//   {ln}\n" for ln in lines)
        + f"constexpr int kGemmClasses = {len(best)};\n"
        + "constexpr int kGemmTileTable[kGemmClasses] = {" + ", ".join(str(b) for b in best) + "};\n"
    )
    if args.dry_run:
        print(text)
    else:
        with open(args.out, "w") as f:
            f.write(text)
        print(f"wrote {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
