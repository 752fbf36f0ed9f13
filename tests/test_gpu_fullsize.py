"""GPU checks at the benchmark sizes, in the launch configuration bench.py
times.

* N = 65536 sampling products: sampled rows of S^r and sampled rows of S^c
  against the oracle's panel product on the same rows of A (read back from
  the device: A is an input) and the same R, within 2 gamma_N |A||R|;
* N = 65536 compression: properties that hold at any size -- every node
  compressed, ranks below the local sample sizes, skeleton indices inside the
  node interval, B_ab = A(I^r_a, I^c_b) exactly, and the acceptance bounds
  ||A - A_HSS||_F <= 10 rtol ||A||_F, ||A_HSS x - A x|| <= 10 rtol ||A x||;
* N = 16384 log kernel at rtol 1e-8, same acceptance bounds;
* N = 4096 Gaussian kernel against the oracle's stored results
  (tests/golden/oracle_gauss4096_*.json, written by make_oracle_golden.py).
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W
from oracle import hss as ohss
from oracle.tree import bisection_tree

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gauss(n, leaf=256):
    p = W.cube_points(n, 4)
    p = p[W.kd_order(p, leaf)]
    return W.device_kernel_matrix("gauss", p, torch.float32, torch.device("cuda:0"))


def _frob(h, A, panel=4096):
    n = A.shape[0]
    num = den = 0.0
    for c0 in range(0, n, panel):
        w = min(panel, n - c0)
        E = torch.zeros((n, w), dtype=torch.float64, device="cuda")
        E[c0:c0 + w] = torch.eye(w, dtype=torch.float64, device="cuda")
        Hp = P.hss_matvec(h, E)
        Ap = A[:, c0:c0 + w].double()
        num += float(torch.linalg.norm(Hp - Ap)) ** 2
        den += float(torch.linalg.norm(Ap)) ** 2
    return (num / den) ** 0.5


def _dense_mv(A, x, block=4096):
    out = torch.empty((A.shape[0], x.shape[1]), dtype=torch.float64, device=A.device)
    for r0 in range(0, A.shape[0], block):
        out[r0:r0 + block] = A[r0:r0 + block].double() @ x
    return out


@pytest.fixture(scope="module")
def gauss65536():
    print("assembling the N=65536 Gaussian kernel matrix", flush=True)
    A = _gauss(65536)
    torch.cuda.synchronize()
    yield A
    del A
    torch.cuda.empty_cache()


def test_sampling_rows_at_full_size(gauss65536):
    A = gauss65536
    n, nc = A.shape[0], 64
    Rr = P.hss_random_normal(0, 0, n, 0, nc)
    Rc = P.hss_random_normal(0, 1, n, 0, nc)
    tree = bisection_tree(n, 256)
    leaf_of = torch.arange(n, device="cuda", dtype=torch.int32) // 256
    print("sample n=65536 ncols=64 masked", flush=True)
    Sr, Sc = P.hss_sample(A, Rr, Rc, leaf_of)
    torch.cuda.synchronize()
    rows = np.random.default_rng(5).choice(n, 12, replace=False)
    rows = np.concatenate([rows, [0, n - 1, 255, 256]])
    Ar = A[torch.from_numpy(rows).cuda()].double().cpu().numpy()       # rows of A
    Ac = A[:, torch.from_numpy(rows).cuda()].double().T.cpu().numpy()  # columns of A, as rows
    Rr_h, Rc_h = Rr.cpu().numpy(), Rc.cpu().numpy()
    for q, i in enumerate(rows):  # S^(leaf) = (A - D^(leaf)) R
        lo = (i // 256) * 256
        Ar[q, lo:lo + 256] = 0.0
        Ac[q, lo:lo + 256] = 0.0
    unused = np.zeros((len(rows), nc))
    ref_r, _ = ohss.sample_panel(Ar, Rr_h, unused)
    ref_c, _ = ohss.sample_panel(Ac, Rc_h, unused)
    g = 2 * n * U / (1 - n * U)
    bnd_r = g * (np.abs(Ar) @ np.abs(Rr_h))
    bnd_c = g * (np.abs(Ac) @ np.abs(Rc_h))
    assert np.all(np.abs(Sr.cpu().numpy()[rows] - ref_r) <= bnd_r)
    assert np.all(np.abs(Sc.cpu().numpy()[rows] - ref_c) <= bnd_c)
    assert tree.n_nodes == 511


def test_compress_gauss65536_acceptance(gauss65536):
    A = gauss65536
    n, rtol = A.shape[0], 1e-6
    print("compress n=65536 rtol=1e-6 p_margin=256", flush=True)
    h = P.hss_compress(A, rtol=rtol, d0=128, dd=64, d_max=4096, leaf_size=256, p_margin=256)
    st = P.hss_stats(h)
    assert st["converged"] and st["n_nodes"] == 511 and st["height"] == 8
    kr, kc, mr, mc = P.hss_ranks(h)
    assert np.all(kr <= mr) and np.all(kc <= mc) and st["max_rank"] < st["d_final"]
    tree = bisection_tree(n, 256)
    for t in (1, 2, 5, 100, 300, 510):
        g = P.hss_export_node(h, t, (tree.left[t], tree.right[t]))
        assert np.all((g["Ir"] >= tree.lo[t]) & (g["Ir"] < tree.hi[t]))
        assert np.all((g["Ic"] >= tree.lo[t]) & (g["Ic"] < tree.hi[t]))
        if tree.left[t] >= 0:
            a, b = tree.left[t], tree.right[t]
            ga = P.hss_export_node(h, a, (tree.left[a], tree.right[a]))
            gb = P.hss_export_node(h, b, (tree.left[b], tree.right[b]))
            sub = A[torch.from_numpy(ga["Ir"].astype(np.int64)).cuda()][:, torch.from_numpy(gb["Ic"].astype(np.int64)).cuda()]
            assert np.array_equal(g["B12"], sub.double().cpu().numpy())
    x = torch.from_numpy(np.random.default_rng(1).uniform(-1, 1, (n, 2))).cuda()
    b = P.hss_matvec(h, x)
    ref = _dense_mv(A, x)
    assert float(torch.linalg.norm(b - ref) / torch.linalg.norm(ref)) <= 10 * rtol
    assert _frob(h, A) <= 10 * rtol


def test_compress_circle16384_acceptance():
    cfg = W.CONFIGS["circle16384"]
    pts = W.circle_points(cfg["n"], cfg["point_seed"])
    A = W.device_kernel_matrix("log", pts, torch.float64, torch.device("cuda:0"))
    print("compress circle n=16384 rtol=1e-8", flush=True)
    h = P.hss_compress(A, rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"])
    st = P.hss_stats(h)
    assert st["converged"] and st["height"] == 7
    x = torch.from_numpy(W.normal_rhs(cfg["n"], 1, 3)).cuda()
    b = P.hss_matvec(h, x)
    ref = A @ x
    assert float(torch.linalg.norm(b - ref) / torch.linalg.norm(ref)) <= 10 * cfg["rtol"]
    assert _frob(h, A) <= 10 * cfg["rtol"]


@pytest.mark.parametrize("pm", [10, 200, 256])
def test_gauss4096_against_stored_oracle(pm):
    path = os.path.join(GOLDEN, f"oracle_gauss4096_rtol1e-06_pm{pm}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    ref = json.load(open(path))
    A = _gauss(ref["n"], ref["leaf"])
    print(f"compress gauss n=4096 p_margin={pm} vs stored oracle", flush=True)
    h = P.hss_compress(A, rtol=ref["rtol"], d0=ref["d0"], dd=ref["dd"], leaf_size=ref["leaf"], p_margin=pm)
    st = P.hss_stats(h)
    assert st["passes"] == ref["passes"] and st["d_final"] == ref["d_final"]
    kr, kc, _, _ = P.hss_ranks(h)
    okr, okc = np.array(ref["kr"]), np.array(ref["kc"])
    diff = np.flatnonzero((kr != okr) | (kc != okc))
    assert len(diff) <= 2 and np.all(np.abs(kr - okr) <= 2) and np.all(np.abs(kc - okc) <= 2)
    err = _frob(h, A)
    assert err <= 1.5 * ref["rel_error"] + 1e-9


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_compress_gauss65536_reduced_precision(gauss65536, prec):
    """The N = 65536 Gaussian kernel at rtol 1e-4 with the sampling products
    in FP32 or in BF16x3 (the precision sweep): converged, with the
    acceptance bounds 10 rtol on the matvec and the Frobenius error, and
    the final d within one growth step of FP64 sampling's."""
    A = gauss65536
    n, rtol = A.shape[0], 1e-4
    kw = dict(rtol=rtol, d0=128, dd=64, d_max=4096, leaf_size=256, p_margin=256)
    print(f"compress n=65536 rtol=1e-4 prec={prec}", flush=True)
    h64 = P.hss_compress(A, **kw)
    d64 = P.hss_stats(h64)["d_final"]
    del h64
    h = P.hss_compress(A, sample_prec=prec, **kw)
    st = P.hss_stats(h)
    assert st["converged"] and abs(st["d_final"] - d64) <= 64, (st["d_final"], d64)
    x = torch.from_numpy(np.random.default_rng(3).uniform(-1, 1, (n, 2))).cuda()
    b = P.hss_matvec(h, x)
    ref = _dense_mv(A, x)
    assert float(torch.linalg.norm(b - ref) / torch.linalg.norm(ref)) <= 10 * rtol
    assert _frob(h, A) <= 10 * rtol


def test_gauss4096_split_launches_skip_failed_nodes(monkeypatch, capfd):
    """Persistent QRCP launches held to 40 workgroups each, so a level's IDs
    need several launches: the second side of a node whose first side
    failed the rule is not factored (the node fails either way, Sec. 3.3),
    and the compression still follows the oracle's schedule (stored result,
    p_margin 256)."""
    path = os.path.join(GOLDEN, "oracle_gauss4096_rtol1e-06_pm256.json")
    ref = json.load(open(path))
    A = _gauss(ref["n"], ref["leaf"])
    monkeypatch.setenv("HSS_QRCP_PATH", "persistent")
    monkeypatch.setenv("HSS_QRCP_PERSIST_WG", "40")
    monkeypatch.setenv("HSS_VERBOSE", "2")
    capfd.readouterr()
    print("compress gauss n=4096 with 40-workgroup persistent launches", flush=True)
    h = P.hss_compress(A, rtol=ref["rtol"], d0=ref["d0"], dd=ref["dd"], leaf_size=ref["leaf"], p_margin=256)
    err_txt = capfd.readouterr().err
    assert "second sides skipped" in err_txt
    st = P.hss_stats(h)
    assert st["passes"] == ref["passes"] and st["d_final"] == ref["d_final"]
    kr, kc, _, _ = P.hss_ranks(h)
    okr, okc = np.array(ref["kr"]), np.array(ref["kc"])
    diff = np.flatnonzero((kr != okr) | (kc != okc))
    assert len(diff) <= 2 and np.all(np.abs(kr - okr) <= 2) and np.all(np.abs(kc - okc) <= 2)
    assert _frob(h, A) <= 1.5 * ref["rel_error"] + 1e-9
