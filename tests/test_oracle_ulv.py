"""Pins of the oracle's ULV factorization and solve (oracle/ulv.py).

* the solution equals a dense LU solve (numpy.linalg.solve) of the matrix
  the HSS generators represent;
* for a one-level tree, diag(Omega_1, Omega_2) A diag(Q_1, Q_2)^T has the
  block structure of Eq. (1level_ulv_transform): [L_i 0] in the t-rows of the
  own block, zeros in the t-rows of the other block, and the reduced matrix
  D_0 of the underlined blocks is what is factored at the root.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hss, ulv


def _omega(idr):
    """Omega = [-E I; I 0] Pi^T as a dense m x m matrix."""
    m, k = idr.m, idr.k
    P = np.zeros((m, m))
    order = np.concatenate([idr.J, idr.rest])
    P[np.arange(m), order] = 1.0  # P x = x[order] = Pi^T x
    top = np.hstack([-idr.E, np.eye(m - k)])
    bot = np.hstack([np.eye(k), np.zeros((k, m - k))])
    return np.vstack([top, bot]) @ P


@pytest.mark.parametrize("case", ["toeplitz", "uneven", "exact", "simple"])
def test_solve_matches_dense_solve(case):
    if case == "toeplitz":
        A = W.toeplitz_inverse_distance(512)
        opts = hss.Options(rtol=1e-8, d0=48, dd=16, leaf_size=32)
    elif case == "uneven":
        A = W.low_rank_plus_identity(129, 5, 3.0, 1)
        opts = hss.Options(rtol=1e-10, d0=16, dd=8, leaf_size=64)
    elif case == "exact":
        A = W.low_rank_plus_identity(300, 7, 2.0, 4)
        opts = hss.Options(rtol=1e-12, d0=20, dd=8, leaf_size=20)
    else:
        A = W.simple_toeplitz(256)
        opts = hss.Options(rtol=1e-10, d0=12, dd=4, leaf_size=16)
    H = hss.compress(A, opts)
    F = ulv.factor(H)
    b = W.normal_rhs(A.shape[0], 3, 9)
    x = ulv.solve(F, b)
    dense = hss.to_dense(H)
    ref = np.linalg.solve(dense, b)
    cond = np.linalg.cond(dense)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-14 * cond * 10
    assert np.linalg.norm(dense @ x - b) / np.linalg.norm(b) < 1e-12
    x1 = ulv.solve(F, b[:, 0])
    assert np.allclose(x1, x[:, 0], rtol=0, atol=1e-12 * np.abs(x).max())


def test_single_leaf_solve():
    A = W.toeplitz_inverse_distance(40)
    H = hss.compress(A, hss.Options(leaf_size=64))
    b = W.normal_rhs(40, 2, 1)
    assert np.allclose(ulv.solve(ulv.factor(H), b), np.linalg.solve(A, b))


def test_one_level_transform_structure():
    n = 128
    A = W.toeplitz_inverse_distance(n) + 0.2 * np.tril(W.toeplitz_inverse_distance(n), -1)
    H = hss.compress(A, hss.Options(rtol=1e-6, d0=40, dd=8, leaf_size=64))
    assert H.tree.n_nodes == 3
    F = ulv.factor(H)
    dense = hss.to_dense(H)
    Om = np.zeros((n, n))
    Qb = np.zeros((n, n))
    m1 = H.tree.size(1)
    Om[:m1, :m1] = _omega(H.U[1])
    Om[m1:, m1:] = _omega(H.U[2])
    Qb[:m1, :m1] = F.Q[1]
    Qb[m1:, m1:] = F.Q[2]
    M = Om @ dense @ Qb.T
    k1, k2 = H.U[1].k, H.U[2].k
    t1 = np.arange(0, m1 - k1)
    b1 = np.arange(m1 - k1, m1)
    t2 = np.arange(m1, n - k2)
    b2 = np.arange(n - k2, n)
    scale = np.abs(dense).max()
    # t-rows: [L_1 0 | 0 0] and [0 0 | L_2 0]
    assert np.allclose(M[np.ix_(t1, t1)], F.L[1], atol=1e-12 * scale)
    assert np.allclose(M[np.ix_(t1, b1)], 0, atol=1e-12 * scale)
    assert np.allclose(M[np.ix_(t1, np.arange(m1, n))], 0, atol=1e-12 * scale)
    assert np.allclose(M[np.ix_(t2, np.arange(0, m1))], 0, atol=1e-12 * scale)
    assert np.allclose(M[np.ix_(t2, t2)], F.L[2], atol=1e-12 * scale)
    assert np.allclose(M[np.ix_(t2, b2)], 0, atol=1e-12 * scale)
    # the underlined blocks form D_0, the matrix LU-factored at the root
    D0 = M[np.ix_(np.concatenate([b1, b2]), np.concatenate([b1, b2]))]
    assert np.allclose(D0, F.root_D, atol=1e-12 * scale)
