"""Pins of the oracle's sampling helpers (oracle/hss.py ``sample`` and
``leaf_local_samples``), the references of the GPU sampling tests.

Alg. 1 (Sec. 2.2) forms S^r = A R^r and S^c = A^T R^c, and at a leaf with
index set I and diagonal block D = A(I, I) the local samples
S^r_loc = S^r(I,:) - D R^r(I,:) and S^c_loc = S^c(I,:) - D^T R^c(I,:).  By
the strip Hankel definition of the off-diagonal block rows (Sec. 2.2) these
equal A(I, I0\\I) R^r(I0\\I) and A(I0\\I, I)^T R^c(I0\\I).

Independent anchors, all on non-symmetric matrices so that a transposed
operand shows:
* identity random matrices: the samples are A and A^T themselves, and the
  leaf local samples are A and A^T with the leaf diagonal blocks zeroed;
* brute force: every entry as an exactly rounded sum (math.fsum) of the
  products, written out from the definition, on tiny inputs;
* the strip Hankel products on index sets built without the tree's blocks;
* the samples that ``compress`` forms panel by panel from its own Philox
  columns (keep_samples=True).
Each planted mistake (A for A^T, D for D^T, a dropped term, a wrong leaf
block) is run through the same checks and must be caught.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import hss
from oracle.tree import bisection_tree


def _nonsym(n, seed):
    g = np.random.default_rng(seed)
    A = W.toeplitz_inverse_distance(n) + 0.3 * g.standard_normal((n, n))
    assert np.abs(A - A.T).max() > 0.1
    return A


def _fsum_product(X, Y):
    """X @ Y with every entry an exactly rounded sum of its n products."""
    out = np.empty((X.shape[0], Y.shape[1]))
    for i in range(X.shape[0]):
        for j in range(Y.shape[1]):
            out[i, j] = math.fsum(float(X[i, k]) * float(Y[k, j]) for k in range(X.shape[1]))
    return out


# ---------------------------------------------------------------------------
# checks, written once and applied to the oracle and to planted mistakes
# ---------------------------------------------------------------------------
def _sample_ok(sample_fn) -> bool:
    n = 11
    A = _nonsym(n, 1)
    g = np.random.default_rng(2)
    Rr, Rc = g.standard_normal((n, 4)), g.standard_normal((n, 3))
    # identity R: the products are the operands themselves
    Sr, Sc = sample_fn(A, np.eye(n), np.eye(n))
    if not (np.array_equal(Sr, A) and np.array_equal(Sc, A.T)):
        return False
    # brute force, each entry within one rounding of the exact sum (the
    # library product and fsum differ by at most gamma_n |A||R|)
    Sr, Sc = sample_fn(A, Rr, Rc)
    gam = n * 2.0 ** -53 / (1 - n * 2.0 ** -53)
    ok_r = np.all(np.abs(Sr - _fsum_product(A, Rr)) <= gam * (np.abs(A) @ np.abs(Rr)))
    ok_c = np.all(np.abs(Sc - _fsum_product(A.T, Rc)) <= gam * (np.abs(A.T) @ np.abs(Rc)))
    return bool(ok_r and ok_c)


def _leaf_ok(leaf_fn) -> bool:
    n, leaf = 23, 5
    tree = bisection_tree(n, leaf)
    A = _nonsym(n, 3)
    # identity R: A and A^T with the leaf diagonal blocks zeroed
    off = np.ones((n, n))
    for t in tree.leaves():
        off[tree.lo[t]:tree.hi[t], tree.lo[t]:tree.hi[t]] = 0.0
    out_r, out_c = leaf_fn(A, tree, A, A.T, np.eye(n), np.eye(n))
    if not (np.allclose(out_r, A * off, rtol=0, atol=1e-15) and
            np.allclose(out_c, A.T * off, rtol=0, atol=1e-15)):
        return False
    # Gaussian R: the strip Hankel products A(I, I0\I) R(I0\I) and
    # A(I0\I, I)^T R(I0\I), each entry an exactly rounded sum
    g = np.random.default_rng(4)
    Rr, Rc = g.standard_normal((n, 3)), g.standard_normal((n, 3))
    Sr, Sc = _fsum_product(A, Rr), _fsum_product(A.T, Rc)
    out_r, out_c = leaf_fn(A, tree, Sr, Sc, Rr, Rc)
    for t in tree.leaves():
        I = np.arange(tree.lo[t], tree.hi[t])
        C = np.array([j for j in range(n) if j < tree.lo[t] or j >= tree.hi[t]])
        ref_r = _fsum_product(A[np.ix_(I, C)], Rr[C])
        ref_c = _fsum_product(A[np.ix_(C, I)].T, Rc[C])
        sc_r = np.abs(A[I]) @ np.abs(Rr)
        sc_c = np.abs(A[:, I].T) @ np.abs(Rc)
        if not (np.all(np.abs(out_r[I] - ref_r) <= 1e-14 * sc_r) and
                np.all(np.abs(out_c[I] - ref_c) <= 1e-14 * sc_c)):
            return False
    return True


# ---------------------------------------------------------------------------
# the oracle passes
# ---------------------------------------------------------------------------
def test_sample_pinned():
    assert _sample_ok(hss.sample)


def test_leaf_local_samples_pinned():
    assert _leaf_ok(hss.leaf_local_samples)


def test_sample_and_leaf_samples_match_compression_panels():
    """The compression forms its samples panel by panel from its own Philox
    columns; ``sample`` + ``leaf_local_samples`` on those columns must give
    its leaf local samples."""
    n, leaf = 300, 40
    A = _nonsym(n, 5)
    H = hss.compress(A, hss.Options(rtol=1e-6, d0=24, dd=8, leaf_size=leaf), keep_samples=True)
    S = H.samples
    Sr, Sc = hss.sample(A, S["Rr"], S["Rc"])
    scale_r = np.abs(A) @ np.abs(S["Rr"])
    scale_c = np.abs(A.T) @ np.abs(S["Rc"])
    assert np.all(np.abs(Sr - S["Sr"]) <= 1e-13 * scale_r)
    assert np.all(np.abs(Sc - S["Sc"]) <= 1e-13 * scale_c)
    out_r, out_c = hss.leaf_local_samples(A, H.tree, Sr, Sc, S["Rr"], S["Rc"])
    for t in H.tree.leaves():
        lo, hi = H.tree.lo[t], H.tree.hi[t]
        k = S["Sr_loc"][t].shape[1]
        assert np.allclose(out_r[lo:hi, :k], S["Sr_loc"][t], rtol=0, atol=1e-12 * scale_r.max())
        assert np.allclose(out_c[lo:hi, :k], S["Sc_loc"][t], rtol=0, atol=1e-12 * scale_c.max())


# ---------------------------------------------------------------------------
# planted mistakes are caught
# ---------------------------------------------------------------------------
def _sample_AT(A, Rr, Rc):  # A and A^T swapped
    A = np.asarray(A, dtype=np.float64)
    return A.T @ Rr, A @ Rc


def _sample_RT(A, Rr, Rc):  # R^r used for both sides
    A = np.asarray(A, dtype=np.float64)
    return A @ Rr, A.T @ Rr[:, :Rc.shape[1]]


def _leaf_DT(A, tree, S_r, S_c, R_r, R_c):  # D and D^T swapped
    out_r, out_c = np.array(S_r, dtype=float), np.array(S_c, dtype=float)
    for t in tree.leaves():
        lo, hi = tree.lo[t], tree.hi[t]
        D = A[lo:hi, lo:hi]
        out_r[lo:hi] -= D.T @ R_r[lo:hi]
        out_c[lo:hi] -= D @ R_c[lo:hi]
    return out_r, out_c


def _leaf_no_c(A, tree, S_r, S_c, R_r, R_c):  # column side term dropped
    out_r, out_c = np.array(S_r, dtype=float), np.array(S_c, dtype=float)
    for t in tree.leaves():
        lo, hi = tree.lo[t], tree.hi[t]
        out_r[lo:hi] -= A[lo:hi, lo:hi] @ R_r[lo:hi]
    return out_r, out_c


def _leaf_shifted(A, tree, S_r, S_c, R_r, R_c):  # block taken one row too low
    out_r, out_c = np.array(S_r, dtype=float), np.array(S_c, dtype=float)
    n = A.shape[0]
    for t in tree.leaves():
        lo, hi = tree.lo[t], tree.hi[t]
        r0 = min(lo + 1, n - (hi - lo))
        D = A[r0:r0 + hi - lo, lo:hi]
        out_r[lo:hi] -= D @ R_r[lo:hi]
        out_c[lo:hi] -= D.T @ R_c[lo:hi]
    return out_r, out_c


@pytest.mark.parametrize("bad", [_sample_AT, _sample_RT])
def test_sample_pin_catches(bad):
    assert not _sample_ok(bad)


@pytest.mark.parametrize("bad", [_leaf_DT, _leaf_no_c, _leaf_shifted])
def test_leaf_pin_catches(bad):
    assert not _leaf_ok(bad)
