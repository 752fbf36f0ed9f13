"""Writes the oracle's results for workloads too slow to recompute inside a
GPU test: the 3-D Gaussian kernel (as in the N=65536 workload) at N=4096,
leaf 256, FP32 storage, d0=128, dd=64.  Calls only oracle/ and workloads/.

    python tests/golden/make_oracle_golden.py [p_margin ...]

Output: tests/golden/oracle_gauss4096_rtol1e-06_pm<p>.json with the
number of passes, d_final, per-node ranks (kr, kc) and the relative
Frobenius error of the oracle's HSS form.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import hss  # noqa: E402


def main(margins):
    n, leaf, rtol = 4096, 256, 1e-6
    p = W.cube_points(n, 4)
    p = p[W.kd_order(p, leaf)]
    A = W.gaussian_kernel(p).astype(np.float32)
    for pm in margins:
        t0 = time.time()
        H = hss.compress(A, hss.Options(rtol=rtol, d0=128, dd=64, d_max=4096, leaf_size=leaf,
                                        p_margin=pm, seed=0))
        kr = [0] * H.tree.n_nodes
        kc = [0] * H.tree.n_nodes
        for t, (a, b) in H.ranks().items():
            kr[t], kc[t] = int(a), int(b)
        out = dict(n=n, leaf=leaf, rtol=rtol, d0=128, dd=64, p_margin=pm, seed=0, storage="f32",
                   points="cube_points(4096, 4), kd_order leaf 256", passes=H.passes,
                   d_final=H.d_final, converged=H.converged, kr=kr, kc=kc,
                   rel_error=hss.relative_error(A.astype(np.float64), H),
                   oracle_seconds=round(time.time() - t0, 1))
        path = os.path.join(HERE, f"oracle_gauss4096_rtol1e-06_pm{pm}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(path, out["passes"], out["d_final"], out["rel_error"], flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [10])
