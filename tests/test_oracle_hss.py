"""Pins of the oracle's compression and matvec (oracle/hss.py).

Independent anchors:
* the strip Hankel definition of the local samples (Sec. 2.2): at a leaf
  S^r_loc = A(I, I0\\I) R^r(I0\\I) and S^c_loc = A(I0\\I, I)^T R^c(I0\\I); at an
  inner node with exact-rank off-diagonal blocks the same holds with the
  rows restricted to the children's row skeletons;
* nested bases (Eq. 4): R^r_tau = (V^big_tau)^T R^r(I_tau);
* exact-rank inputs (A = cI + XY^T, every off-diagonal block of rank <= k)
  give ranks <= k and a reconstruction at rounding level; rtol = 0 gives an
  exact HSS form;
* the paper's SimpleToeplitz ranks and sampling flops (Table 3);
* the adaptive rule's restart count, predicted in closed form for
  exact-rank inputs, and the late-notification state invariant (Sec. 3.3);
* Alg. 2 against the dense matrix assembled from the HSS definition.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import hss
from oracle.tree import bisection_tree

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _asym(n, k, seed):
    return W.low_rank_plus_identity(n, k, c=3.0, seed=seed)


def _descendants(tree, t):
    out, st = [], [t]
    while st:
        v = st.pop()
        if tree.left[v] >= 0:
            out += [tree.left[v], tree.right[v]]
            st += [tree.left[v], tree.right[v]]
    return out


def _ancestors(tree, t):
    out = []
    while tree.parent[t] >= 0:
        t = tree.parent[t]
        out.append(t)
    return out


def test_leaf_local_samples_are_strip_hankel_products():
    n = 200
    A = W.toeplitz_inverse_distance(n)
    A = A + np.triu(A, 1) * 0.37  # make it non-symmetric
    H = hss.compress(A, hss.Options(rtol=1e-7, d0=40, dd=8, leaf_size=25), keep_samples=True)
    S = H.samples
    d = H.d_final
    for t in H.tree.leaves():
        I = np.arange(H.tree.lo[t], H.tree.hi[t])
        C = np.setdiff1d(np.arange(n), I)
        ref_r = A[np.ix_(I, C)] @ S["Rr"][C, :d]
        ref_c = A[np.ix_(C, I)].T @ S["Rc"][C, :d]
        assert np.allclose(S["Sr_loc"][t][:, :d], ref_r, rtol=0, atol=1e-12 * np.abs(ref_r).max())
        assert np.allclose(S["Sc_loc"][t][:, :d], ref_c, rtol=0, atol=1e-12 * np.abs(ref_c).max())


def test_inner_local_samples_and_nested_R_exact_rank():
    n, k = 256, 6
    A = _asym(n, k, 1)
    H = hss.compress(A, hss.Options(rtol=1e-12, d0=24, dd=8, leaf_size=32), keep_samples=True)
    S, tree, d = H.samples, H.tree, H.d_final
    vbig, ubig = {}, {}
    for h in range(tree.height[0]):
        for t in tree.nodes_at_height(h):
            if tree.is_leaf(t):
                vbig[t] = H.V[t].U()
                ubig[t] = H.U[t].U()
            else:
                a, b = tree.left[t], tree.right[t]
                bd = np.zeros((vbig[a].shape[0] + vbig[b].shape[0], vbig[a].shape[1] + vbig[b].shape[1]))
                bd[:vbig[a].shape[0], :vbig[a].shape[1]] = vbig[a]
                bd[vbig[a].shape[0]:, vbig[a].shape[1]:] = vbig[b]
                vbig[t] = bd @ H.V[t].U()
                bu = np.zeros((ubig[a].shape[0] + ubig[b].shape[0], ubig[a].shape[1] + ubig[b].shape[1]))
                bu[:ubig[a].shape[0], :ubig[a].shape[1]] = ubig[a]
                bu[ubig[a].shape[0]:, ubig[a].shape[1]:] = ubig[b]
                ubig[t] = bu @ H.U[t].U()
            I = np.arange(tree.lo[t], tree.hi[t])
            # nested bases: R_tau = (V^big)^T R(I)
            assert np.allclose(S["Rr_t"][t][:, :d], vbig[t].T @ S["Rr"][I, :d], atol=1e-10)
            assert np.allclose(S["Rc_t"][t][:, :d], ubig[t].T @ S["Rc"][I, :d], atol=1e-10)
            if not tree.is_leaf(t):
                a, b = tree.left[t], tree.right[t]
                C = np.setdiff1d(np.arange(n), I)
                rows_r = np.concatenate([H.Ir[a], H.Ir[b]])
                rows_c = np.concatenate([H.Ic[a], H.Ic[b]])
                ref_r = A[np.ix_(rows_r, C)] @ S["Rr"][C, :d]
                ref_c = A[np.ix_(C, rows_c)].T @ S["Rc"][C, :d]
                scale = max(np.abs(ref_r).max(), 1.0)
                assert np.allclose(S["Sr_loc"][t][:, :d], ref_r, atol=1e-9 * scale)
                assert np.allclose(S["Sc_loc"][t][:, :d], ref_c, atol=1e-9 * scale)
    assert H.max_rank() <= k
    assert hss.relative_error(A, H) < 1e-12


@pytest.mark.parametrize("n,leaf,k", [(129, 64, 5), (300, 40, 3), (512, 32, 8)])
def test_exact_rank_inputs(n, leaf, k):
    A = _asym(n, k, n)
    H = hss.compress(A, hss.Options(rtol=1e-12, d0=k + 12, dd=8, leaf_size=leaf))
    assert H.converged and H.max_rank() <= k
    assert hss.relative_error(A, H) < 1e-12


def test_rtol_zero_is_exact():
    n = 96
    g = np.random.default_rng(3)
    A = g.standard_normal((n, n))
    H = hss.compress(A, hss.Options(rtol=0.0, d0=n, dd=8, leaf_size=12, d_max=n))
    assert H.converged
    assert hss.relative_error(A, H) < 1e-13
    # full-rank blocks give U = Pi I: no E entries
    for t in H.U:
        assert H.U[t].E.size == 0 and H.V[t].E.size == 0


def _golden_table3():
    rows = []
    with open(os.path.join(GOLDEN, "paper_table3_simple_toeplitz.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                eps, r, gf = line.split()
                rows.append((float(eps), int(r), float(gf)))
    return rows


def test_simple_toeplitz_against_table3():
    rows = _golden_table3()
    # the printed flops are those of sampling with d = r + 10 = 12 at n = 80000
    for eps, r, gflop in rows:
        model = hss.sampling_flops(80_000, 12) / 1e9
        assert abs(model - gflop) / gflop < 1e-3
    # off-diagonal blocks of a_ij = i - j have rank 2: ranks never exceed the
    # printed maximum ranks (2 at 1e-8 and 1e-6, 3 at 1e-4 and 1e-2)
    A = W.simple_toeplitz(1024)
    for eps, r, _ in rows:
        H = hss.compress(A, hss.Options(rtol=eps, d0=12, dd=4, leaf_size=64))
        assert H.converged and H.max_rank() <= r
        assert hss.relative_error(A, H) <= 10 * eps


@pytest.mark.parametrize("k,d0,dd", [(6, 8, 4), (6, 16, 4), (9, 4, 8), (12, 40, 8)])
def test_adaptive_restart_count(k, d0, dd):
    n, leaf, p = 256, 32, 10
    A = _asym(n, k, 11)
    H = hss.compress(A, hss.Options(rtol=1e-11, d0=d0, dd=dd, leaf_size=leaf, p_margin=p))
    restarts = max(0, math.ceil((k + p - d0) / dd))
    assert H.passes == restarts + 1
    assert H.d_final == d0 + restarts * dd
    assert H.max_rank() <= k


def test_late_notification_invariants():
    A = W.toeplitz_inverse_distance(1024)
    H = hss.compress(A, hss.Options(rtol=1e-6, d0=12, dd=6, leaf_size=64))
    assert H.passes >= 3
    tree = H.tree
    saw_partial = False
    for d, states, _ in H.history:
        for t, s in states.items():
            if s == hss.PARTIALLY_COMPRESSED:
                saw_partial = True
                assert all(states[c] == hss.COMPRESSED for c in _descendants(tree, t))
                assert all(states.get(a, hss.UNTOUCHED) == hss.UNTOUCHED for a in _ancestors(tree, t) if a != 0)
            if s == hss.UNTOUCHED and not tree.is_leaf(t):
                kids = (states[tree.left[t]], states[tree.right[t]])
                assert kids != (hss.COMPRESSED, hss.COMPRESSED)
    assert saw_partial
    assert hss.relative_error(A, H) <= 10 * 1e-6


def test_not_converged_at_d_max():
    A = _asym(256, 20, 2)
    H = hss.compress(A, hss.Options(rtol=1e-12, d0=8, dd=8, d_max=16, leaf_size=32))
    assert not H.converged and H.d_final == 16
    assert len(H.U) == H.tree.n_nodes - 1


def test_matvec_matches_definition():
    for A, opts in [
        (W.toeplitz_inverse_distance(1024), hss.Options(rtol=1e-6, d0=64, dd=32, leaf_size=64)),
        (_asym(129, 4, 5), hss.Options(rtol=1e-10, d0=20, dd=8, leaf_size=64)),
        (W.simple_toeplitz(300), hss.Options(rtol=1e-8, d0=12, dd=4, leaf_size=20)),
    ]:
        H = hss.compress(A, opts)
        x = W.uniform_rhs(A.shape[0], 3, 1)
        dense = hss.to_dense(H)
        assert np.allclose(hss.matvec(H, x), dense @ x, rtol=0, atol=1e-12 * np.abs(dense @ x).max())
        assert np.allclose(hss.matvec(H, x[:, 0]), dense @ x[:, 0], rtol=0,
                           atol=1e-12 * np.abs(dense @ x).max())


def test_toeplitz1024_acceptance():
    cfg = W.CONFIGS["toeplitz1024"]
    A = W.toeplitz_inverse_distance(cfg["n"])
    H = hss.compress(A, hss.Options(rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"]))
    assert H.converged
    assert hss.relative_error(A, H) <= 10 * cfg["rtol"]
    x = W.uniform_rhs(cfg["n"], 8, cfg["rhs_seed"])
    b = hss.matvec(H, x)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(A @ x) <= 10 * cfg["rtol"]


def test_single_leaf_tree():
    A = W.toeplitz_inverse_distance(50)
    H = hss.compress(A, hss.Options(leaf_size=64))
    assert np.array_equal(hss.to_dense(H), A)
    x = W.uniform_rhs(50, 2, 0)
    assert np.allclose(hss.matvec(H, x), A @ x)


def test_float32_storage_is_upcast_exactly():
    A = W.toeplitz_inverse_distance(256).astype(np.float32)
    opts = hss.Options(rtol=1e-6, d0=40, dd=8, leaf_size=32)
    H32 = hss.compress(A, opts)
    H64 = hss.compress(A.astype(np.float64), opts)
    assert H32.ranks() == H64.ranks()
    assert hss.relative_error(A.astype(np.float64), H32) == hss.relative_error(A.astype(np.float64), H64)
    assert bisection_tree(256, 32).n_nodes == H32.tree.n_nodes


def test_full_rank_blocks_never_fail():
    # leaves of 4 rows are full rank (k = m) at any d: the fail rule must not
    # fire for them; the root's children (16 rows, full rank) need d >= 16.
    g = np.random.default_rng(8)
    A = g.standard_normal((32, 32))
    H = hss.compress(A, hss.Options(rtol=1e-12, d0=12, dd=4, leaf_size=4))
    assert H.passes == 2 and H.d_final == 16 and H.converged
    first_pass_states = H.history[0][1]
    assert all(first_pass_states[t] == hss.COMPRESSED for t in H.tree.leaves())
    assert hss.relative_error(A, H) < 1e-12
