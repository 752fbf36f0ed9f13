"""End-to-end GPU compression and matvec against the oracle (C ABI).

Several results are correct at once for a randomized, pivoted method: near
ties between column norms may pick different pivots after rounding.  So the
unique parts are compared exactly -- the tree, the number of passes, d_final
(the adaptive schedule) -- the per-node ranks must agree except for at most
one node by at most one, and the rest is checked for validity: the
reconstruction error ||A - A_HSS||_F / ||A||_F <= 10 rtol, the GPU matvec
against a dense A x to 10 rtol, and the GPU matvec applied to the oracle's
own generators (imported through hss_import) to 1e-13 against the oracle's
Alg. 2 on those generators.
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W
from oracle import hss as ohss
from oracle.tree import bisection_tree

pytestmark = pytest.mark.gpu


def _gpu(A, **kw):
    return P.hss_compress(torch.from_numpy(np.ascontiguousarray(A)).cuda(), **kw)


def _gpu_dense(h, n):
    eye = torch.eye(n, dtype=torch.float64, device="cuda")
    return P.hss_matvec(h, eye).cpu().numpy()


def _rank_arrays_oracle(H):
    nn = H.tree.n_nodes
    kr = np.zeros(nn, dtype=int)
    kc = np.zeros(nn, dtype=int)
    for t, (a, b) in H.ranks().items():
        kr[t], kc[t] = a, b
    return kr, kc


def _compare(A, rtol, d0, dd, leaf, d_max=4096, max_mismatch=1, seed=0):
    n = A.shape[0]
    print(f"compress n={n} rtol={rtol} d0={d0} dd={dd} leaf={leaf}", flush=True)
    Ho = ohss.compress(A, ohss.Options(rtol=rtol, d0=d0, dd=dd, d_max=d_max, leaf_size=leaf, seed=seed))
    h = _gpu(A, rtol=rtol, d0=d0, dd=dd, d_max=d_max, leaf_size=leaf, seed=seed)
    st = P.hss_stats(h)
    assert st["n_nodes"] == Ho.tree.n_nodes
    assert st["passes"] == Ho.passes
    assert st["d_final"] == Ho.d_final
    assert bool(st["converged"]) == Ho.converged
    kr, kc, mr, mc = P.hss_ranks(h)
    okr, okc = _rank_arrays_oracle(Ho)
    diff = np.flatnonzero((kr != okr) | (kc != okc))
    assert len(diff) <= max_mismatch, (diff, kr[diff], okr[diff], kc[diff], okc[diff])
    assert np.all(np.abs(kr - okr) <= 1) and np.all(np.abs(kc - okc) <= 1)
    return Ho, h


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_toeplitz1024_acceptance(storage):
    cfg = W.CONFIGS["toeplitz1024"]
    A = W.toeplitz_inverse_distance(cfg["n"])
    if storage == "f32":
        A = A.astype(np.float32)
    A64 = A.astype(np.float64)
    Ho, h = _compare(A, cfg["rtol"], cfg["d0"], cfg["dd"], cfg["leaf"])
    dense = _gpu_dense(h, cfg["n"])
    err = np.linalg.norm(A64 - dense) / np.linalg.norm(A64)
    assert err <= 10 * cfg["rtol"], err
    for nrhs in (1, 8):
        x = W.uniform_rhs(cfg["n"], nrhs, cfg["rhs_seed"])
        b = P.hss_matvec(h, torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.linalg.norm(b - A64 @ x) / np.linalg.norm(A64 @ x) <= 10 * cfg["rtol"]
    xv = torch.from_numpy(W.uniform_rhs(cfg["n"], 1, 2)[:, 0]).cuda()
    bv = P.hss_matvec(h, xv)
    assert bv.shape == (cfg["n"],)


def test_adaptive_schedule_matches_oracle():
    A = W.toeplitz_inverse_distance(1024)
    Ho, h = _compare(A, 1e-6, 12, 6, 64)
    assert Ho.passes >= 3
    dense = _gpu_dense(h, 1024)
    assert np.linalg.norm(A - dense) / np.linalg.norm(A) <= 1e-5


@pytest.mark.parametrize("n,leaf,k,d0,dd", [(129, 64, 5, 8, 4), (1000, 64, 7, 16, 8), (2051, 100, 9, 24, 8)])
def test_exact_rank_uneven(n, leaf, k, d0, dd):
    A = W.low_rank_plus_identity(n, k, 3.0, n)
    Ho, h = _compare(A, 1e-12, d0, dd, leaf, max_mismatch=0)
    kr, kc, _, _ = P.hss_ranks(h)
    assert kr.max() <= k and kc.max() <= k
    dense = _gpu_dense(h, n)
    assert np.linalg.norm(A - dense) / np.linalg.norm(A) < 1e-12


def test_user_tree_and_single_leaf():
    A = W.toeplitz_inverse_distance(300)
    # uneven user tree: [0,300) -> [0,40) leaf, [40,300) -> [40,170), [170,300)
    tree = ([0, 0, 40, 40, 170], [300, 40, 300, 170, 300], [-1, -1, -1, -1, -1], [-1] * 5)
    left = [1, -1, 3, -1, -1]
    right = [2, -1, 4, -1, -1]
    tree = (tree[0], tree[1], left, right)
    h = _gpu(A, tree=tree, rtol=1e-8, d0=40, dd=8)
    dense = _gpu_dense(h, 300)
    assert np.linalg.norm(A - dense) / np.linalg.norm(A) <= 1e-7
    h1 = _gpu(A[:50, :50], leaf_size=64)
    assert np.allclose(_gpu_dense(h1, 50), A[:50, :50], rtol=0, atol=1e-15)


def test_not_converged_is_usable():
    A = W.low_rank_plus_identity(256, 20, 3.0, 2)
    h = _gpu(A, rtol=1e-12, d0=8, dd=8, d_max=16, leaf_size=32)
    assert h.status == P.HSS_NOT_CONVERGED and not P.hss_stats(h)["converged"]
    Ho = ohss.compress(A, ohss.Options(rtol=1e-12, d0=8, dd=8, d_max=16, leaf_size=32))
    assert not Ho.converged and P.hss_stats(h)["d_final"] == Ho.d_final == 16
    x = torch.ones(256, 1, dtype=torch.float64, device="cuda")
    assert torch.isfinite(P.hss_matvec(h, x)).all()


def test_release_cached_memory_keeps_live_handles():
    """Releasing the library's cached blocks leaves a live handle usable and
    changes no result: the same compression after the release (fresh
    blocks) gives bit-identical products."""
    cfg = W.CONFIGS["toeplitz1024"]
    A = W.toeplitz_inverse_distance(cfg["n"])
    kw = dict(rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"])
    x = torch.from_numpy(W.uniform_rhs(cfg["n"], 4, cfg["rhs_seed"])).cuda()
    h0 = _gpu(A, **kw)
    b0 = P.hss_matvec(h0, x).cpu().numpy()
    h1 = _gpu(A, **kw)
    P.hss_destroy(h1)  # its blocks go to the cache
    P.hss_release_cached_memory()
    assert np.array_equal(P.hss_matvec(h0, x).cpu().numpy(), b0)
    h2 = _gpu(A, **kw)
    assert np.array_equal(P.hss_matvec(h2, x).cpu().numpy(), b0)
    P.hss_release_cached_memory()  # nothing cached but the blocks of h0, h2: both stay live
    assert np.array_equal(P.hss_matvec(h2, x).cpu().numpy(), b0)


def _oracle_to_import(Ho):
    tree = Ho.tree
    nodes = []
    kr = np.zeros(tree.n_nodes, dtype=np.int32)
    kc = np.zeros(tree.n_nodes, dtype=np.int32)
    for t in range(tree.n_nodes):
        nd = {}
        if t != 0:
            nd.update(Jr=Ho.U[t].J, Jc=Ho.V[t].J, Er=Ho.U[t].E, Ec=Ho.V[t].E)
            kr[t], kc[t] = Ho.U[t].k, Ho.V[t].k
        if tree.is_leaf(t):
            nd["D"] = Ho.D[t]
        else:
            nd["B12"], nd["B21"] = Ho.B12[t], Ho.B21[t]
        nodes.append(nd)
    return (tree.lo, tree.hi, tree.left, tree.right), kr, kc, nodes


@pytest.mark.parametrize("case", ["toeplitz", "uneven", "simple"])
def test_matvec_on_oracle_generators(case):
    if case == "toeplitz":
        A, opts = W.toeplitz_inverse_distance(1024), ohss.Options(rtol=1e-6, d0=64, dd=32, leaf_size=64)
    elif case == "uneven":
        A, opts = W.low_rank_plus_identity(129, 5, 3.0, 1), ohss.Options(rtol=1e-10, d0=16, dd=8, leaf_size=64)
    else:
        A, opts = W.simple_toeplitz(700), ohss.Options(rtol=1e-8, d0=12, dd=4, leaf_size=50)
    Ho = ohss.compress(A, opts)
    tree, kr, kc, nodes = _oracle_to_import(Ho)
    h = P.hss_import(A.shape[0], tree, kr, kc, nodes)
    for nrhs in (1, 5):
        x = W.uniform_rhs(A.shape[0], nrhs, 4)
        ref = ohss.matvec(Ho, x)
        got = P.hss_matvec(h, torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_export_structure():
    A = W.toeplitz_inverse_distance(512)
    h = _gpu(A, rtol=1e-8, d0=48, dd=16, leaf_size=32)
    tree = bisection_tree(512, 32)
    kr, kc, mr, mc = P.hss_ranks(h)
    for t in range(1, tree.n_nodes):
        g = P.hss_export_node(h, t, (tree.left[t], tree.right[t]))
        lo, hi = tree.lo[t], tree.hi[t]
        assert len(set(g["Jr"].tolist())) == kr[t] and np.all((g["Jr"] >= 0) & (g["Jr"] < mr[t]))
        assert np.all((g["Ir"] >= lo) & (g["Ir"] < hi)) and np.all((g["Ic"] >= lo) & (g["Ic"] < hi))
        if not tree.is_leaf(t):
            a, b = tree.left[t], tree.right[t]
            assert np.array_equal(g["B12"], A[np.ix_(P.hss_export_node(h, a, (tree.left[a], tree.right[a]))["Ir"],
                                                     P.hss_export_node(h, b, (tree.left[b], tree.right[b]))["Ic"])])
        else:
            assert np.array_equal(g["D"], A[lo:hi, lo:hi])


def test_small_ids_in_two_phases_skip_failed_nodes(monkeypatch, capfd):
    """Small IDs run in two phases when forced (the first side of every node,
    then the second side where the first passed the rule): the compression is
    the one-phase compression exactly (a node with a failing side fails
    either way, Sec. 3.3), bit for bit in the matvec, and second sides were
    skipped."""
    A = W.toeplitz_inverse_distance(2048)
    kw = dict(rtol=1e-8, d0=16, dd=8, leaf_size=64)
    monkeypatch.setenv("HSS_QRCP_SMALL_SPLIT", "0")
    h0 = _gpu(A, **kw)
    monkeypatch.setenv("HSS_QRCP_SMALL_SPLIT", "1")
    monkeypatch.setenv("HSS_VERBOSE", "2")
    capfd.readouterr()
    print("compress with small IDs in two phases", flush=True)
    h1 = _gpu(A, **kw)
    err = capfd.readouterr().err
    skipped = [int(line.split(":")[1].split()[0]) for line in err.splitlines() if "two phases" in line]
    assert skipped and sum(skipped) > 0, err
    s0, s1 = P.hss_stats(h0), P.hss_stats(h1)
    assert (s0["passes"], s0["d_final"]) == (s1["passes"], s1["d_final"]) and s0["passes"] >= 3
    for a, b in zip(P.hss_ranks(h0), P.hss_ranks(h1)):
        assert np.array_equal(a, b)
    x = torch.from_numpy(W.uniform_rhs(2048, 3, 5)).cuda()
    assert torch.equal(P.hss_matvec(h0, x), P.hss_matvec(h1, x))
    Ho = ohss.compress(A, ohss.Options(**kw))
    assert (s1["passes"], s1["d_final"]) == (Ho.passes, Ho.d_final)
