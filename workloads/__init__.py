"""Seeded synthetic inputs for randomized HSS compression.

This module only builds *inputs*: point clouds, their ordering, the dense
kernel matrices assembled from them, right-hand sides and plain random test
matrices.  It holds none of the compression method's arithmetic (no tree,
no sampling, no interpolative decomposition), so that both the FP64 oracle
and the GPU library can be fed the same data without sharing any code.

Workloads (all seeded, NumPy ``default_rng`` / PCG64):

* ``toeplitz_inverse_distance`` -- A_ij = 1/(1+|i-j|), A_ii = 2 (natural
  order; a smooth Toeplitz matrix in the spirit of the paper's Toeplitz test
  matrices, Sec. 4.1).
* ``simple_toeplitz`` -- the paper's SimpleToeplitz: a_ii = n^2,
  a_ij = i - j (Sec. 4.1); its off-diagonal blocks have rank <= 2.
* ``circle_points`` + ``log_kernel`` -- N points on the unit circle with a
  radial jitter of 1e-3*U(-1,1), ordered by angle; A_ij = -ln|x_i - x_j|,
  A_ii = 1 + ln N (a 2-D BEM-like kernel standing in for the paper's BEM
  matrices, Sec. 4.1).
* ``cube_points`` + ``kd_order`` + ``gaussian_kernel`` -- p ~ U[0,1]^3 ordered
  by recursive k-d bisection; A_ij = exp(-|p_i-p_j|^2 / (2 sigma^2)) +
  1e-2 delta_ij with sigma = 0.1 (a covariance-like kernel standing in for
  the paper's covariance matrices, Sec. 4.1).
* ``planar_points`` + ``laplace_kernel`` -- points in the unit square (z=0),
  A_ij = 1/(4 pi |p_i - p_j|), A_ii = sqrt(N) (a frontal-like separator
  matrix standing in for the paper's root fronts, Sec. 4.6).
* ``low_rank_plus_identity`` -- A = c I + X Y^T with X, Y n x k, so every
  off-diagonal block has rank <= k exactly.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "toeplitz_inverse_distance",
    "simple_toeplitz",
    "circle_points",
    "log_kernel",
    "cube_points",
    "planar_points",
    "kd_order",
    "gaussian_kernel",
    "laplace_kernel",
    "low_rank_plus_identity",
    "uniform_rhs",
    "normal_rhs",
    "gaussian_matrix",
    "kernel_rows",
    "device_kernel_matrix",
    "CONFIGS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# plain matrices
# --------------------------------------------------------------------------
def toeplitz_inverse_distance(n: int) -> np.ndarray:
    """A_ij = 1/(1+|i-j|) for i != j, A_ii = 2, float64, natural order."""
    i = np.arange(n, dtype=np.float64)
    a = 1.0 / (1.0 + np.abs(i[:, None] - i[None, :]))
    np.fill_diagonal(a, 2.0)
    return a


def simple_toeplitz(n: int) -> np.ndarray:
    """The paper's SimpleToeplitz: a_ii = n^2, a_ij = i - j (1-based or
    0-based gives the same matrix since only differences appear)."""
    i = np.arange(n, dtype=np.float64)
    a = i[:, None] - i[None, :]
    np.fill_diagonal(a, float(n) * float(n))
    return a


def low_rank_plus_identity(n: int, k: int, c: float = 1.0, seed: int = 0) -> np.ndarray:
    """A = c I + X Y^T, X and Y n x k standard normal: every block A(I, J)
    with I and J disjoint has rank <= k."""
    g = _rng(seed)
    x = g.standard_normal((n, k))
    y = g.standard_normal((n, k))
    return c * np.eye(n) + x @ y.T


def gaussian_matrix(rows: int, cols: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    return g.standard_normal((rows, cols))


def uniform_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """x ~ U(-1, 1), n x nrhs, row-major."""
    return _rng(seed).uniform(-1.0, 1.0, size=(n, nrhs))


def normal_rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    return _rng(seed).standard_normal((n, nrhs))


# --------------------------------------------------------------------------
# point clouds and their ordering
# --------------------------------------------------------------------------
def circle_points(n: int, seed: int, jitter: float = 1e-3) -> np.ndarray:
    """theta_i = 2 pi (i + 1/2)/n, r_i = 1 + jitter*u_i, u_i ~ U(-1, 1).
    Already ordered by angle.  Returns n x 2."""
    u = _rng(seed).uniform(-1.0, 1.0, size=n)
    th = 2.0 * math.pi * (np.arange(n) + 0.5) / n
    r = 1.0 + jitter * u
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def cube_points(n: int, seed: int) -> np.ndarray:
    """p ~ U[0,1]^3, n x 3 (unordered)."""
    return _rng(seed).uniform(0.0, 1.0, size=(n, 3))


def planar_points(n: int, seed: int) -> np.ndarray:
    """p ~ U[0,1]^2 x {0}, n x 3 (unordered)."""
    p = np.zeros((n, 3))
    p[:, :2] = _rng(seed).uniform(0.0, 1.0, size=(n, 2))
    return p


def kd_order(points: np.ndarray, leaf_size: int) -> np.ndarray:
    """Permutation ordering the points by recursive k-d bisection.

    A set of m > leaf_size points is split at its median along the axis of
    largest extent (stable sort), the lower floor(m/2) points first, then
    each half is ordered recursively.  Sets of at most leaf_size points keep
    their incoming order.  The interval sizes therefore follow the same
    floor/ceil halving as the cluster tree built on [0, n)."""
    n = points.shape[0]
    perm = np.arange(n)
    stack = [(0, n)]
    while stack:
        lo, hi = stack.pop()
        m = hi - lo
        if m <= leaf_size:
            continue
        idx = perm[lo:hi]
        sub = points[idx]
        ext = sub.max(axis=0) - sub.min(axis=0)
        axis = int(np.argmax(ext))
        order = np.argsort(sub[:, axis], kind="stable")
        perm[lo:hi] = idx[order]
        half = m // 2
        stack.append((lo + half, hi))
        stack.append((lo, lo + half))
    return perm


# --------------------------------------------------------------------------
# kernel matrices (host, float64; rows may be a subset)
# --------------------------------------------------------------------------
def _sqdist(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    d = np.zeros((p.shape[0], q.shape[0]))
    for a in range(p.shape[1]):
        diff = p[:, a][:, None] - q[:, a][None, :]
        d += diff * diff
    return d


def log_kernel(points: np.ndarray, rows: np.ndarray | None = None) -> np.ndarray:
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    d2 = _sqdist(points[rows], points)
    with np.errstate(divide="ignore"):
        a = -0.5 * np.log(d2)
    a[np.arange(rows.size), rows] = 1.0 + math.log(n)
    return a


def gaussian_kernel(points: np.ndarray, rows: np.ndarray | None = None,
                    sigma: float = 0.1, shift: float = 1e-2) -> np.ndarray:
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    d2 = _sqdist(points[rows], points)
    a = np.exp(-d2 / (2.0 * sigma * sigma))
    a[np.arange(rows.size), rows] += shift
    return a


def laplace_kernel(points: np.ndarray, rows: np.ndarray | None = None) -> np.ndarray:
    n = points.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    d2 = _sqdist(points[rows], points)
    with np.errstate(divide="ignore"):
        a = 1.0 / (4.0 * math.pi * np.sqrt(d2))
    a[np.arange(rows.size), rows] = math.sqrt(n)
    return a


_KERNELS = {"log": log_kernel, "gauss": gaussian_kernel, "laplace": laplace_kernel}


def kernel_rows(kind: str, points: np.ndarray, rows, dtype=np.float64) -> np.ndarray:
    """Rows `rows` of the kernel matrix, rounded to `dtype` (the storage
    type), returned as float64."""
    a = _KERNELS[kind](points, np.asarray(rows))
    return a.astype(dtype).astype(np.float64)


def device_kernel_matrix(kind: str, points: np.ndarray, dtype, device, block: int = 2048):
    """Assemble the kernel matrix on the GPU with PyTorch, block of rows by
    block of rows (float64 arithmetic, rounded to ``dtype`` for storage).
    Used for the large workloads whose host assembly would take minutes;
    the arithmetic matches ``kernel_rows`` up to the last bit of exp/log."""
    import torch

    n = points.shape[0]
    p = torch.as_tensor(points, dtype=torch.float64, device=device)
    out = torch.empty((n, n), dtype=dtype, device=device)
    for lo in range(0, n, block):
        hi = min(n, lo + block)
        q = p[lo:hi]
        d2 = torch.zeros((hi - lo, n), dtype=torch.float64, device=device)
        for a in range(p.shape[1]):
            diff = q[:, a][:, None] - p[:, a][None, :]
            d2 += diff * diff
        r = torch.arange(hi - lo, device=device)
        if kind == "gauss":
            blk = torch.exp(-d2 / (2.0 * 0.1 * 0.1))
            blk[r, r + lo] += 1e-2
        elif kind == "log":
            blk = -0.5 * torch.log(d2)
            blk[r, r + lo] = 1.0 + math.log(n)
        elif kind == "laplace":
            blk = 1.0 / (4.0 * math.pi * torch.sqrt(d2))
            blk[r, r + lo] = math.sqrt(n)
        else:
            raise ValueError(kind)
        out[lo:hi] = blk.to(dtype)
        del d2, blk
    return out


def batch_instances(count: int, n_lo: int, n_hi: int, seed: int, leaf_size: int):
    """`count` planar point sets for a batch of independent matrices: sizes
    N = floor(exp(U(ln n_lo, ln n_hi))), points p ~ U[0,1]^2 x {0}, each set
    ordered by k-d bisection with `leaf_size`.  One seeded generator draws
    the sizes, then the point sets in order."""
    g = _rng(seed)
    sizes = np.floor(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    sets = []
    for n in sizes:
        p = np.zeros((int(n), 3))
        p[:, :2] = g.uniform(0.0, 1.0, size=(int(n), 2))
        sets.append(p[kd_order(p, leaf_size)])
    return sets


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
CONFIGS = {
    # small FP64 Toeplitz, runs in seconds on the CPU
    "toeplitz1024": dict(n=1024, kind="toeplitz", leaf=64, rtol=1e-6, d0=64, dd=32,
                         storage="f64", rhs_seed=1),
    # 2-D log kernel on a perturbed circle, FP64, then ULV solve
    "circle16384": dict(n=16384, kind="log", leaf=128, rtol=1e-8, d0=128, dd=64,
                        storage="f64", point_seed=2, rhs_seed=3),
    # 3-D Gaussian kernel, k-d ordered, FP32 storage
    "gauss65536": dict(n=65536, kind="gauss", leaf=256, rtol=1e-6, d0=128, dd=64,
                       storage="f32", point_seed=4, rhs_seed=1),
    # 512 independent planar 1/(4 pi r) matrices (frontal-matrix stand-ins),
    # N log-uniform in [256, 4096], FP32 storage, BF16x3 sampling
    "batched512": dict(count=512, n_lo=256, n_hi=4096, kind="laplace", leaf=64, rtol=1e-4,
                       d0=64, dd=32, d_max=1024, p_margin=32, storage="f32", sample_prec="bf16x3",
                       point_seed=5),
}


def config_points(name: str, n: int | None = None) -> np.ndarray | None:
    cfg = CONFIGS[name]
    n = cfg["n"] if n is None else n
    if cfg["kind"] == "log":
        return circle_points(n, cfg["point_seed"])
    if cfg["kind"] == "gauss":
        p = cube_points(n, cfg["point_seed"])
        return p[kd_order(p, cfg["leaf"])]
    return None
