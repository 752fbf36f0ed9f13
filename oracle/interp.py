"""Interpolative decomposition to a relative tolerance (Sec. 2.2, Sec. 3.2).

[X, J] = ID(Y, eps) expresses the columns of Y (d x m) as combinations of a
subset J of its columns, Y ~ Y(:, J) X, computed from a QR factorization
with column pivoting Y Pi = Q [R1 R2] (R1: k x k), which gives
X = [I  R1^{-1} R2] Pi^{-1}.  The pivoted QR stops as soon as the next
pivot's R_ii satisfies |R_ii| / |R_11| <= eps; the number of pivots taken is
the eps-rank k.

Readings taken where the paper is silent:

* the pivot is the column with the largest 2-norm of its not yet
  eliminated part, recomputed exactly at every step; equal norms are broken
  by the lowest original column index;
* k = 0 when Y is zero (R_11 = 0);
* the generator stored is U = X^T = Pi [I; E] (Sec. 2.2): J holds the
  selected columns in pivot order, `rest` the others in increasing index
  order, and E = (R1^{-1} R2)^T with its rows in that same order.

Pins: pivots equal LAPACK's column-pivoted QR (scipy.linalg.qr) on inputs
with well separated norms; U(J, :) = I; the residual
||Y(:, rest) - Y(:, J) E^T||_F <= sqrt(m-k) eps |R_11| (up to rounding), which
also bounds the number of singular values above that level by k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_triangular


@dataclass
class IDResult:
    k: int            # eps-rank
    J: np.ndarray     # selected columns, pivot order (int64, length k)
    rest: np.ndarray  # other columns, increasing (length m-k)
    E: np.ndarray     # (m-k) x k, U = Pi [I; E]
    r11: float        # |R_11| (largest column norm of Y)

    @property
    def m(self) -> int:
        return self.k + self.rest.size

    def U(self) -> np.ndarray:
        """Dense m x k generator with U[J] = I and U[rest] = E."""
        u = np.zeros((self.m, self.k))
        u[self.J, np.arange(self.k)] = 1.0
        u[self.rest, :] = self.E
        return u


def interpolative_decomposition(Y: np.ndarray, eps: float) -> IDResult:
    Y = np.array(Y, dtype=np.float64, copy=True)
    d, m = Y.shape
    kmax = min(d, m)
    cols = np.arange(m)  # cols[p] = original column now at position p
    k = 0
    r11 = 0.0
    for i in range(kmax):
        nrm = np.linalg.norm(Y[i:, i:], axis=0)
        best = nrm.max()
        if i == 0:
            r11 = float(best)
        if best == 0.0 or best <= eps * r11:
            break
        ties = np.flatnonzero(nrm == best)
        p = i + ties[np.argmin(cols[i + ties])]
        if p != i:
            Y[:, [i, p]] = Y[:, [p, i]]
            cols[[i, p]] = cols[[p, i]]
        # Householder reflector H = I - 2 v v^T / (v^T v) with H x = alpha e1
        x = Y[i:, i]
        alpha = -np.copysign(np.linalg.norm(x), x[0])
        v = x.copy()
        v[0] -= alpha
        vv = float(v @ v)
        if i + 1 < m and vv > 0.0:
            tail = Y[i:, i + 1:]
            tail -= np.outer(v, (2.0 / vv) * (v @ tail))
        Y[i, i] = alpha
        Y[i + 1:, i] = 0.0
        k = i + 1
    R1 = np.triu(Y[:k, :k])
    R2 = Y[:k, k:]
    T = solve_triangular(R1, R2, lower=False) if k > 0 else np.zeros((0, m - k))
    rest_pos = np.argsort(cols[k:], kind="stable")
    rest = cols[k:][rest_pos]
    E = np.ascontiguousarray(T[:, rest_pos].T)
    return IDResult(k=k, J=cols[:k].copy(), rest=rest, E=E, r11=r11)


def apply_transpose(idr: IDResult, x: np.ndarray) -> np.ndarray:
    """U^T x = x[J] + E^T x[rest]  (x has m rows)."""
    return x[idr.J] + idr.E.T @ x[idr.rest]


def apply(idr: IDResult, z: np.ndarray) -> np.ndarray:
    """U z: rows J get z, rows `rest` get E z  (z has k rows)."""
    out = np.zeros((idr.m,) + z.shape[1:])
    out[idr.J] = z
    out[idr.rest] = idr.E @ z
    return out
