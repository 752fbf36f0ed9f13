"""Randomized HSS compression (Alg. 1) with adaptive sampling (Sec. 3.3,
Alg. 5), HSS matvec (Alg. 2) and the dense matrix an HSS form represents
(Eqs. 1-4, Sec. 2.1).  FP64, node by node.

Compression, in the paper's order:

1. draw R^r, R^c (n x d) and form the samples S^r = A R^r, S^c = A^T R^c;
2. visit the nodes children-before-parents.  At a leaf,
   D = A(I, I), S^r_loc = S^r(I, :) - D R^r(I, :), S^c_loc = S^c(I, :) - D^T R^c(I, :).
   At an inner node with children a, b:
   B_ab = A(I^r_a, I^c_b), B_ba = A(I^r_b, I^c_a),
   S^r_loc = [S^r_a - B_ab R^r_b ; S^r_b - B_ba R^r_a],
   S^c_loc = [S^c_a - B_ba^T R^c_b ; S^c_b - B_ab^T R^c_a];
3. [U^T, J^r] = ID((S^r_loc)^T, eps), [V^T, J^c] = ID((S^c_loc)^T, eps);
4. S^r_tau = S^r_loc(J^r, :), S^c_tau = S^c_loc(J^c, :),
   R^r_tau = V^T R^r_in, R^c_tau = U^T R^c_in with R_in = R(I, :) at a leaf
   and the children's stacked R_a, R_b otherwise;
   I^r_tau = I_in(J^r), I^c_tau = I_in(J^c);
5. at the root only B_ab and B_ba are formed.

Adaptive sampling, late notification (Sec. 3.3), run level-synchronously:
one pass visits the heights 0, 1, ... in order; an inner node whose
children are not both COMPRESSED is skipped (stays UNTOUCHED).  A node that
is UNTOUCHED builds its local samples from column 0; a PARTIALLY_COMPRESSED
node and a COMPRESSED node only build the new columns and append them.  A
node that is not COMPRESSED runs both IDs; if either fails it becomes
PARTIALLY_COMPRESSED and its generators are thrown away.  When a pass ends
with a node not COMPRESSED, dd new columns are drawn and sampled and a new
pass starts.

Readings (where the paper is silent or garbled):

* fail rule: an ID fails when its rank k exceeds d - p_margin while k is
  below m, the number of rows of the local sample (k = m means the basis is
  exact, U = Pi I, so more samples cannot help).  p_margin defaults to the
  oversampling of Alg. 1 (d = r + 10);
* every COMPRESSED node extends its local samples and R_tau with new
  columns; only nodes below an unfinished ancestor ever read them, so this
  gives the same result as extending only those;
* d grows d0, d0+dd, ... up to d_max; when a pass fails at d = d_max a last
  pass accepts every ID regardless of the fail rule and the result is
  flagged not converged;
* the root has no U or V, it only forms B_ab and B_ba (Alg. 1 result).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import philox
from .interp import IDResult, apply, apply_transpose, interpolative_decomposition
from .tree import ClusterTree, bisection_tree

UNTOUCHED, PARTIALLY_COMPRESSED, COMPRESSED = 0, 1, 2


@dataclass
class Options:
    rtol: float = 1e-6
    d0: int = 64
    dd: int = 32
    d_max: int = 4096
    p_margin: int = 10
    seed: int = 0
    leaf_size: int = 64
    # precision of the sampling products: "f64", or "f32" / "bf16x3" (A
    # stored in FP32); in the reduced modes R is rounded once when drawn
    # (see round_random) and the rounded R is used everywhere after that
    sample_prec: str = "f64"


@dataclass
class HSSForm:
    tree: ClusterTree
    n: int
    D: dict = field(default_factory=dict)      # leaf -> |I| x |I|
    U: dict = field(default_factory=dict)      # non-root -> IDResult (row basis)
    V: dict = field(default_factory=dict)      # non-root -> IDResult (column basis)
    B12: dict = field(default_factory=dict)    # inner -> k^r_a x k^c_b
    B21: dict = field(default_factory=dict)    # inner -> k^r_b x k^c_a
    Ir: dict = field(default_factory=dict)     # non-root -> global row skeleton
    Ic: dict = field(default_factory=dict)     # non-root -> global column skeleton
    d_final: int = 0
    passes: int = 0
    converged: bool = True
    history: list = field(default_factory=list)  # per pass: (d, states, ranks)
    samples: dict | None = None

    def ranks(self):
        return {t: (self.U[t].k, self.V[t].k) for t in self.U}

    def max_rank(self) -> int:
        return max([max(kr, kc) for kr, kc in self.ranks().values()], default=0)


def round_random(R, prec: str):
    """R rounded to nearest, ties to even, from its float64 value: to FP32
    ("f32"), or to 8 significant bits, the precision of BF16 ("bf16x3");
    unchanged for "f64".  This is the random matrix the reduced-precision
    sampling modes use in every later step (their products are then exact
    up to the rounding of accumulation, which the oracle does not model: it
    forms the products in float64)."""
    R = np.asarray(R, dtype=np.float64)
    if prec == "f64":
        return R.copy()
    if prec == "f32":
        return R.astype(np.float32).astype(np.float64)
    if prec != "bf16x3":
        raise ValueError(prec)
    # 8 significant bits keep the top 7 of the 52 stored fraction bits: round
    # the low 45 bits away, to nearest, ties to even (a carry may bump the
    # exponent, which is the correct rounding)
    u = np.ascontiguousarray(R).view(np.uint64).copy()
    low = np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    rem = u & low
    keep_odd = (u >> np.uint64(45)) & np.uint64(1)
    up = (rem > half) | ((rem == half) & (keep_odd == np.uint64(1)))
    u = u & ~low
    u = u + np.where(up, np.uint64(1 << 45), np.uint64(0))
    return u.view(np.float64).reshape(R.shape)


class _Sampler:
    """Random matrices and the samples S^r = A R^r, S^c = A^T R^c, grown by
    columns.  A may be float32 (upcast exactly by row panels)."""

    def __init__(self, A, seed, R_r=None, R_c=None, panel=4096, prec="f64"):
        self.A = A
        self.n = A.shape[0]
        self.seed = seed
        self.prec = prec
        self.R_user = (R_r, R_c)
        self.panel = panel
        self.Rr = np.zeros((self.n, 0))
        self.Rc = np.zeros((self.n, 0))
        self.Sr = np.zeros((self.n, 0))
        self.Sc = np.zeros((self.n, 0))

    def grow(self, c0, c1):
        if self.R_user[0] is not None:
            rr = np.asarray(self.R_user[0][:, c0:c1], dtype=np.float64)
            rc = np.asarray(self.R_user[1][:, c0:c1], dtype=np.float64)
        else:
            rr = philox.gaussian_columns(self.seed, 0, self.n, c0, c1)
            rc = philox.gaussian_columns(self.seed, 1, self.n, c0, c1)
        rr = round_random(rr, self.prec)
        rc = round_random(rc, self.prec)
        sr = np.zeros((self.n, c1 - c0))
        sc = np.zeros((self.n, c1 - c0))
        for r0 in range(0, self.n, self.panel):
            r1 = min(self.n, r0 + self.panel)
            sr[r0:r1], part = sample_panel(self.A[r0:r1], rr, rc[r0:r1])
            sc += part
        self.Rr = np.hstack([self.Rr, rr])
        self.Rc = np.hstack([self.Rc, rc])
        self.Sr = np.hstack([self.Sr, sr])
        self.Sc = np.hstack([self.Sc, sc])


def sample_panel(A_rows, R_r, R_c_rows):
    """One row panel P of the sampling products: S^r(P, :) = A(P, :) R^r and
    the panel's share A(P, :)^T R^c(P, :) of S^c = A^T R^c.  A(P, :) may be
    float32; it is widened exactly to float64."""
    blk = np.asarray(A_rows, dtype=np.float64)
    return blk @ R_r, blk.T @ R_c_rows


def _fails(idr: IDResult, d: int, p_margin: int) -> bool:
    return idr.k > d - p_margin and idr.k < idr.m


def compress(A, opts: Options, tree: ClusterTree | None = None, R_r=None, R_c=None,
             keep_samples: bool = False) -> HSSForm:
    """HSS form of the dense n x n matrix A (float64 or float32 array).

    R_r, R_c: optional n x d_max random matrices used instead of the Philox
    columns.  keep_samples: keep the local samples, the R_tau and the global
    R, S in ``H.samples`` (for tests)."""
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    tree = bisection_tree(n, opts.leaf_size) if tree is None else tree
    H = HSSForm(tree=tree, n=n)
    root = 0
    if tree.is_leaf(root):
        H.D[root] = np.asarray(A, dtype=np.float64).copy()
        return H
    height_root = tree.height[root]
    levels = [[t for t in tree.nodes_at_height(h) if t != root] for h in range(height_root)]
    nonroot = [t for t in range(tree.n_nodes) if t != root]

    state = {t: UNTOUCHED for t in nonroot}
    cdone = {t: 0 for t in nonroot}
    Sr_loc, Sc_loc, Rr_t, Rc_t = {}, {}, {}, {}

    def A_sub(rows, cols):
        return np.asarray(A[np.ix_(rows, cols)], dtype=np.float64)

    if opts.sample_prec != "f64" and np.asarray(A).dtype != np.float32:
        raise ValueError("reduced-precision sampling needs A stored in float32")
    smp = _Sampler(A, opts.seed, R_r, R_c, prec=opts.sample_prec)
    d = min(opts.d0, opts.d_max)
    smp.grow(0, d)
    forced = False

    def local_samples(t, c0, c1):
        if tree.is_leaf(t):
            lo, hi = tree.lo[t], tree.hi[t]
            Dt = H.D[t]
            sr = smp.Sr[lo:hi, c0:c1] - Dt @ smp.Rr[lo:hi, c0:c1]
            sc = smp.Sc[lo:hi, c0:c1] - Dt.T @ smp.Rc[lo:hi, c0:c1]
        else:
            a, b = tree.left[t], tree.right[t]
            sr = np.vstack([
                Sr_loc[a][H.U[a].J, c0:c1] - H.B12[t] @ Rr_t[b][:, c0:c1],
                Sr_loc[b][H.U[b].J, c0:c1] - H.B21[t] @ Rr_t[a][:, c0:c1]])
            sc = np.vstack([
                Sc_loc[a][H.V[a].J, c0:c1] - H.B21[t].T @ Rc_t[b][:, c0:c1],
                Sc_loc[b][H.V[b].J, c0:c1] - H.B12[t].T @ Rc_t[a][:, c0:c1]])
        return sr, sc

    def r_update(t, c0, c1):
        if tree.is_leaf(t):
            lo, hi = tree.lo[t], tree.hi[t]
            rr_in, rc_in = smp.Rr[lo:hi, c0:c1], smp.Rc[lo:hi, c0:c1]
        else:
            a, b = tree.left[t], tree.right[t]
            rr_in = np.vstack([Rr_t[a][:, c0:c1], Rr_t[b][:, c0:c1]])
            rc_in = np.vstack([Rc_t[a][:, c0:c1], Rc_t[b][:, c0:c1]])
        return apply_transpose(H.V[t], rr_in), apply_transpose(H.U[t], rc_in)

    def index_sets(t):
        if tree.is_leaf(t):
            base_r = base_c = np.arange(tree.lo[t], tree.hi[t])
        else:
            a, b = tree.left[t], tree.right[t]
            base_r = np.concatenate([H.Ir[a], H.Ir[b]])
            base_c = np.concatenate([H.Ic[a], H.Ic[b]])
        return base_r, base_c

    while True:
        H.passes += 1
        for lvl in levels:
            for t in lvl:
                leaf = tree.is_leaf(t)
                if not leaf:
                    a, b = tree.left[t], tree.right[t]
                    if state[a] != COMPRESSED or state[b] != COMPRESSED:
                        continue
                if state[t] == UNTOUCHED:
                    if leaf:
                        lo, hi = tree.lo[t], tree.hi[t]
                        H.D[t] = A_sub(np.arange(lo, hi), np.arange(lo, hi))
                    else:
                        H.B12[t] = A_sub(H.Ir[a], H.Ic[b])
                        H.B21[t] = A_sub(H.Ir[b], H.Ic[a])
                    Sr_loc[t] = np.zeros((len(index_sets(t)[0]), 0))
                    Sc_loc[t] = np.zeros((len(index_sets(t)[1]), 0))
                    cdone[t] = 0
                c0 = cdone[t]
                if c0 < d:
                    sr, sc = local_samples(t, c0, d)
                    Sr_loc[t] = np.hstack([Sr_loc[t], sr])
                    Sc_loc[t] = np.hstack([Sc_loc[t], sc])
                if state[t] != COMPRESSED:
                    idr = interpolative_decomposition(Sr_loc[t].T, opts.rtol)
                    idc = interpolative_decomposition(Sc_loc[t].T, opts.rtol)
                    if not forced and (_fails(idr, d, opts.p_margin) or _fails(idc, d, opts.p_margin)):
                        state[t] = PARTIALLY_COMPRESSED
                        cdone[t] = d
                        continue
                    H.U[t], H.V[t] = idr, idc
                    base_r, base_c = index_sets(t)
                    H.Ir[t] = base_r[idr.J]
                    H.Ic[t] = base_c[idc.J]
                    Rr_t[t], Rc_t[t] = r_update(t, 0, d)
                    state[t] = COMPRESSED
                elif c0 < d:
                    rr, rc = r_update(t, c0, d)
                    Rr_t[t] = np.hstack([Rr_t[t], rr])
                    Rc_t[t] = np.hstack([Rc_t[t], rc])
                cdone[t] = d
        H.history.append((d, dict(state), {t: (H.U[t].k, H.V[t].k) for t in H.U}))
        if all(state[t] == COMPRESSED for t in nonroot):
            break
        if d >= opts.d_max:
            forced = True
            H.converged = False
            continue
        dn = min(d + opts.dd, opts.d_max)
        smp.grow(d, dn)
        d = dn
    a, b = tree.left[root], tree.right[root]
    H.B12[root] = A_sub(H.Ir[a], H.Ic[b])
    H.B21[root] = A_sub(H.Ir[b], H.Ic[a])
    H.d_final = d
    if keep_samples:
        H.samples = dict(Sr_loc=Sr_loc, Sc_loc=Sc_loc, Rr_t=Rr_t, Rc_t=Rc_t,
                         Rr=smp.Rr, Rc=smp.Rc, Sr=smp.Sr, Sc=smp.Sc)
    return H


# --------------------------------------------------------------------------
# using the HSS form
# --------------------------------------------------------------------------
def matvec(H: HSSForm, x: np.ndarray) -> np.ndarray:
    """Alg. 2: b = A_HSS x for x with one or more columns."""
    tree = H.tree
    x = np.asarray(x, dtype=np.float64)
    vec = x.ndim == 1
    if vec:
        x = x[:, None]
    root = 0
    if tree.is_leaf(root):
        b = H.D[root] @ x
        return b[:, 0] if vec else b
    y, z = {}, {}
    hr = tree.height[root]
    for h in range(hr):  # upward: y = V^T x
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                xin = x[tree.lo[t]:tree.hi[t]]
            else:
                xin = np.vstack([y[tree.left[t]], y[tree.right[t]]])
            y[t] = apply_transpose(H.V[t], xin)
    b = np.zeros_like(x)
    for h in range(hr, -1, -1):  # downward
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                lo, hi = tree.lo[t], tree.hi[t]
                b[lo:hi] = apply(H.U[t], z[t]) + H.D[t] @ x[lo:hi]
                continue
            a, c = tree.left[t], tree.right[t]
            ka = H.U[a].k
            if t == root:
                w = np.zeros((ka + H.U[c].k, x.shape[1]))
            else:
                w = apply(H.U[t], z[t])
            z[a] = H.B12[t] @ y[c] + w[:ka]
            z[c] = H.B21[t] @ y[a] + w[ka:]
    return b[:, 0] if vec else b


def to_dense(H: HSSForm) -> np.ndarray:
    """The matrix the generators represent, assembled from the definition:
    D at the leaves, U^big_tau = diag(U^big_a, U^big_b) U_tau (nested bases),
    and A(I_a, I_b) = U^big_a B_ab (V^big_b)^T for every pair of siblings."""
    tree = H.tree
    out = np.zeros((H.n, H.n))
    root = 0
    if tree.is_leaf(root):
        return H.D[root].copy()
    ubig, vbig = {}, {}
    for h in range(tree.height[root]):
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                ubig[t] = H.U[t].U()
                vbig[t] = H.V[t].U()
            else:
                a, b = tree.left[t], tree.right[t]
                blk_u = np.zeros((ubig[a].shape[0] + ubig[b].shape[0], ubig[a].shape[1] + ubig[b].shape[1]))
                blk_u[:ubig[a].shape[0], :ubig[a].shape[1]] = ubig[a]
                blk_u[ubig[a].shape[0]:, ubig[a].shape[1]:] = ubig[b]
                blk_v = np.zeros((vbig[a].shape[0] + vbig[b].shape[0], vbig[a].shape[1] + vbig[b].shape[1]))
                blk_v[:vbig[a].shape[0], :vbig[a].shape[1]] = vbig[a]
                blk_v[vbig[a].shape[0]:, vbig[a].shape[1]:] = vbig[b]
                ubig[t] = blk_u @ H.U[t].U()
                vbig[t] = blk_v @ H.V[t].U()
    for t in range(tree.n_nodes):
        if tree.is_leaf(t):
            lo, hi = tree.lo[t], tree.hi[t]
            out[lo:hi, lo:hi] = H.D[t]
        else:
            a, b = tree.left[t], tree.right[t]
            out[tree.lo[a]:tree.hi[a], tree.lo[b]:tree.hi[b]] = ubig[a] @ H.B12[t] @ vbig[b].T
            out[tree.lo[b]:tree.hi[b], tree.lo[a]:tree.hi[a]] = ubig[b] @ H.B21[t] @ vbig[a].T
    return out


def relative_error(A, H: HSSForm) -> float:
    A = np.asarray(A, dtype=np.float64)
    return float(np.linalg.norm(A - to_dense(H)) / np.linalg.norm(A))


def sampling_flops(n: int, d: int) -> float:
    """Flops of the two sampling products S^r = A R^r, S^c = A^T R^c with d
    columns each: 2 * (2 n^2 d) (Sec. 2.2 states they dominate)."""
    return 4.0 * n * n * d


def sample(A, R_r, R_c):
    """S^r = A R^r and S^c = A^T R^c (Alg. 1, step 2), FP64."""
    A = np.asarray(A, dtype=np.float64)
    return A @ np.asarray(R_r, dtype=np.float64), A.T @ np.asarray(R_c, dtype=np.float64)


def leaf_local_samples(A, tree: ClusterTree, S_r, S_c, R_r, R_c):
    """Leaf local samples of Alg. 1 stacked in index order:
    S^r_loc = S^r(I,:) - D R^r(I,:), S^c_loc = S^c(I,:) - D^T R^c(I,:)."""
    A = np.asarray(A, dtype=np.float64)
    out_r = np.array(S_r, dtype=np.float64, copy=True)
    out_c = np.array(S_c, dtype=np.float64, copy=True)
    for t in tree.leaves():
        lo, hi = tree.lo[t], tree.hi[t]
        D = A[lo:hi, lo:hi]
        out_r[lo:hi] -= D @ R_r[lo:hi]
        out_c[lo:hi] -= D.T @ R_c[lo:hi]
    return out_r, out_c
