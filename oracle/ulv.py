"""ULV-like factorization (Alg. 3, Sec. 2.4) and solve (Alg. 4, Sec. 2.5,
App. A) of an HSS form whose U generators have the ID structure
U = Pi [I; E].

Factorization, children before parents:

* D_tau = D at a leaf; at an inner node
  D_tau = [Dt_a, B_ab Vt_{b;b}^T ; B_ba Vt_{a;b}^T, Dt_b];
  Vh_tau = V at a leaf, diag(Vt_{a;b}, Vt_{b;b}) V_tau at an inner node;
* Omega = [-E I; I 0] Pi^T gives Omega U = [0; I];
  W = Omega D_tau = [W_t; W_b] with W_b the k^r rows Pi^T selects first,
  i.e. W_t = D_tau(rest, :) - E D_tau(J, :) and W_b = D_tau(J, :);
* LQ factorization W_t = [L 0] Q (Q square orthogonal, Q_t its first
  m - k rows, Q_b the rest), Vt = Q Vh = [Vt_t; Vt_b], Dt = W_b Q_b^T;
* at the root D_tau is factored by LU with partial pivoting.

Solve, bottom-up then top-down (Alg. 4):

* b_tau = b(I) at a leaf; at an inner node
  b_tau = [bt_{a;b} - W_{a;b} Q_{a;t}^T y_a - B_ab z_b ;
           bt_{b;b} - B_ba z_a - W_{b;b} Q_{b;t}^T y_b];
* bt = Omega b_tau = [b_tau(rest) - E b_tau(J) ; b_tau(J)],
  y = L^{-1} bt_t, z = Vt_t^T y (+ V^T [z_a; z_b] at an inner node);
* root: x_root = D_root^{-1} b_root (LU);
* x_a = Q_a^T [y_a; x_tau(top)], x_b = Q_b^T [y_b; x_tau(bottom)].

Pins: the result equals a dense LU solve of the matrix the generators
represent (to_dense); the one-level transform has the zero blocks of
Eq. (1level_ulv_transform).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import lu_factor, lu_solve, solve_triangular

from .hss import HSSForm
from .interp import apply_transpose


@dataclass
class ULVFactors:
    H: HSSForm
    L: dict = field(default_factory=dict)       # (m-k) x (m-k) lower triangular
    Q: dict = field(default_factory=dict)       # m x m orthogonal
    Wb: dict = field(default_factory=dict)      # k x m
    Vt_t: dict = field(default_factory=dict)    # (m-k) x k^c
    Vt_b: dict = field(default_factory=dict)    # k x k^c
    Dt: dict = field(default_factory=dict)      # k x k
    root_lu: tuple | None = None
    root_D: np.ndarray | None = None


def _lq(Wt: np.ndarray):
    """W_t = [L 0] Q with Q orthogonal (from a complete QR of W_t^T)."""
    r, m = Wt.shape
    if r == 0:
        return np.zeros((0, 0)), np.eye(m)
    q, rr = np.linalg.qr(Wt.T, mode="complete")
    return rr[:r, :].T.copy(), q.T.copy()


def _blockdiag(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    out = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]))
    out[:a.shape[0], :a.shape[1]] = a
    out[a.shape[0]:, a.shape[1]:] = b
    return out


def _merged_D(F: ULVFactors, t: int) -> np.ndarray:
    H, tree = F.H, F.H.tree
    a, b = tree.left[t], tree.right[t]
    top = np.hstack([F.Dt[a], H.B12[t] @ F.Vt_b[b].T])
    bot = np.hstack([H.B21[t] @ F.Vt_b[a].T, F.Dt[b]])
    return np.vstack([top, bot])


def factor(H: HSSForm) -> ULVFactors:
    F = ULVFactors(H=H)
    tree = H.tree
    root = 0
    if tree.is_leaf(root):
        F.root_D = H.D[root]
        F.root_lu = lu_factor(H.D[root])
        return F
    for h in range(tree.height[root]):
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                Dtau = H.D[t]
                Vh = H.V[t].U()
            else:
                a, b = tree.left[t], tree.right[t]
                Dtau = _merged_D(F, t)
                Vh = _blockdiag(F.Vt_b[a], F.Vt_b[b]) @ H.V[t].U()
            U = H.U[t]
            Wt = Dtau[U.rest] - U.E @ Dtau[U.J]
            Wb = Dtau[U.J]
            L, Q = _lq(Wt)
            mk = Wt.shape[0]
            Vt = Q @ Vh
            F.L[t], F.Q[t], F.Wb[t] = L, Q, Wb
            F.Vt_t[t], F.Vt_b[t] = Vt[:mk], Vt[mk:]
            F.Dt[t] = Wb @ Q[mk:].T
    F.root_D = _merged_D(F, root)
    F.root_lu = lu_factor(F.root_D)
    return F


def solve(F: ULVFactors, b: np.ndarray) -> np.ndarray:
    H, tree = F.H, F.H.tree
    b = np.asarray(b, dtype=np.float64)
    vec = b.ndim == 1
    if vec:
        b = b[:, None]
    root = 0
    if tree.is_leaf(root):
        x = lu_solve(F.root_lu, b)
        return x[:, 0] if vec else x
    y, z, btb = {}, {}, {}

    def rhs(t):
        if tree.is_leaf(t):
            return b[tree.lo[t]:tree.hi[t]]
        a, c = tree.left[t], tree.right[t]
        ma = F.Q[a].shape[0] - F.Wb[a].shape[0]
        mc = F.Q[c].shape[0] - F.Wb[c].shape[0]
        top = btb[a] - F.Wb[a] @ (F.Q[a][:ma].T @ y[a]) - H.B12[t] @ z[c]
        bot = btb[c] - H.B21[t] @ z[a] - F.Wb[c] @ (F.Q[c][:mc].T @ y[c])
        return np.vstack([top, bot])

    for h in range(tree.height[root]):
        for t in tree.nodes_at_height(h):
            bt = rhs(t)
            U = H.U[t]
            bt_t = bt[U.rest] - U.E @ bt[U.J]
            btb[t] = bt[U.J]
            y[t] = solve_triangular(F.L[t], bt_t, lower=True) if bt_t.shape[0] else bt_t
            z[t] = F.Vt_t[t].T @ y[t]
            if not tree.is_leaf(t):
                z[t] = z[t] + apply_transpose(H.V[t], np.vstack([z[tree.left[t]], z[tree.right[t]]]))
    xs = {root: lu_solve(F.root_lu, rhs(root))}
    x = np.zeros_like(b)
    for h in range(tree.height[root], -1, -1):
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                x[tree.lo[t]:tree.hi[t]] = xs[t]
                continue
            a, c = tree.left[t], tree.right[t]
            ka = H.U[a].k
            xs[a] = F.Q[a].T @ np.vstack([y[a], xs[t][:ka]])
            xs[c] = F.Q[c].T @ np.vstack([y[c], xs[t][ka:]])
    return x[:, 0] if vec else x
