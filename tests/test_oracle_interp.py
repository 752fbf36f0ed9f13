"""Pins of the oracle's interpolative decomposition (oracle/interp.py).

What fixes the ID independently of the oracle's own code:
* LAPACK's column-pivoted QR (scipy.linalg.qr(pivoting=True), xGEQP3)
  chooses the same pivots when the column norms are well separated;
* hand-worked 2x2 / 3x3 cases;
* the mathematics of a QR stopped at |R_kk| <= eps |R_11|:
  Y(:, rest) - Y(:, J) E^T = Q2 R22 whose columns all have norm <= eps |R_11|,
  so its Frobenius norm is <= sqrt(m-k) eps |R_11| and sigma_{k+1}(Y) is
  bounded by the same number; exact-rank inputs give exactly their rank.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.interp import apply, apply_transpose, interpolative_decomposition


def _separated(d, m, seed):
    g = np.random.default_rng(seed)
    y = g.standard_normal((d, m))
    # geometric column scaling in a shuffled order: distinct norms at every step
    scale = 2.0 ** (-np.arange(m) * 0.7)
    return y * scale[g.permutation(m)]


@pytest.mark.parametrize("d,m,seed", [(12, 8, 0), (8, 12, 1), (30, 30, 2), (5, 40, 3)])
def test_pivots_match_lapack_qrcp(d, m, seed):
    y = _separated(d, m, seed)
    idr = interpolative_decomposition(y, 0.0)
    _, _, piv = sla.qr(y, pivoting=True, mode="economic")
    k = min(d, m)
    assert idr.k == k
    assert list(idr.J) == list(piv[:k])


def test_hand_worked_cases():
    # one nonzero column of norm 5, one zero column: rank 1
    r = interpolative_decomposition(np.array([[3.0, 0.0], [4.0, 0.0]]), 1e-12)
    assert r.k == 1 and list(r.J) == [0] and list(r.rest) == [1] and r.E[0, 0] == 0.0
    # column 0 = 0.5 * column 1; column 1 has the larger norm
    r = interpolative_decomposition(np.array([[1.0, 2.0], [0.0, 0.0]]), 1e-12)
    assert r.k == 1 and list(r.J) == [1] and list(r.rest) == [0]
    assert r.E[0, 0] == pytest.approx(0.5, abs=1e-15)
    # all norms equal: the lowest index wins every tie
    r = interpolative_decomposition(np.eye(3), 1e-12)
    assert r.k == 3 and list(r.J) == [0, 1, 2] and r.E.shape == (0, 3)
    # eps >= 1 keeps nothing; a zero matrix has rank 0
    assert interpolative_decomposition(np.ones((3, 3)), 1.0).k == 0
    z = interpolative_decomposition(np.zeros((4, 5)), 1e-6)
    assert z.k == 0 and z.E.shape == (5, 0) and list(z.rest) == [0, 1, 2, 3, 4]


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6, 1e-8, 1e-10])
def test_residual_bound_and_svd_rank(eps):
    g = np.random.default_rng(7)
    d, m = 60, 45
    u, _ = np.linalg.qr(g.standard_normal((d, d)))
    v, _ = np.linalg.qr(g.standard_normal((m, m)))
    s = 10.0 ** (-np.linspace(0, 12, min(d, m)))
    y = (u[:, :min(d, m)] * s) @ v.T
    idr = interpolative_decomposition(y, eps)
    k = idr.k
    resid = y[:, idr.rest] - y[:, idr.J] @ idr.E.T
    bound = np.sqrt(m - k) * eps * idr.r11
    slack = 1e-13 * idr.r11 * np.sqrt(m * d)  # rounding
    assert np.linalg.norm(resid) <= bound + slack
    sv = np.linalg.svd(y, compute_uv=False)
    assert np.sum(sv > bound + slack) <= k
    # U(J,:) = I exactly and U reproduces Y^T from the skeleton rows
    U = idr.U()
    assert np.array_equal(U[idr.J], np.eye(k))
    assert np.linalg.norm(y.T - U @ y[:, idr.J].T) <= bound + slack


@pytest.mark.parametrize("rank", [0, 1, 3, 9])
def test_exact_rank_recovered(rank):
    g = np.random.default_rng(rank)
    y = g.standard_normal((40, rank)) @ g.standard_normal((rank, 25))
    idr = interpolative_decomposition(y, 1e-10)
    assert idr.k == rank
    assert np.allclose(y[:, idr.J] @ idr.U().T, y, atol=1e-11 * max(1.0, np.abs(y).max()))


def test_apply_helpers_match_dense():
    g = np.random.default_rng(5)
    y = g.standard_normal((10, 16))
    idr = interpolative_decomposition(y, 0.3)
    U = idr.U()
    x = g.standard_normal((16, 3))
    z = g.standard_normal((idr.k, 3))
    assert np.allclose(apply_transpose(idr, x), U.T @ x)
    assert np.allclose(apply(idr, z), U @ z)
