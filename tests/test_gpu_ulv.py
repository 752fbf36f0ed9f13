"""GPU ULV factorization and solve (Alg. 3/4) through the C ABI.

* On the oracle's own generators (imported with hss_import) the GPU solve
  equals the oracle's ULV solve, which is pinned to a dense LU solve of the
  represented matrix: |x_gpu - x_oracle| <= 1e-14 cond(A_HSS) |x|.
* After a GPU compression: A_HSS x = b to 1e-11 relative (the GPU matvec of
  the same handle), and the original A x = b to the compression accuracy.
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W
from oracle import hss as ohss
from oracle import ulv as oulv

pytestmark = pytest.mark.gpu


def _import(Ho):
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
    return P.hss_import(Ho.n, (tree.lo, tree.hi, tree.left, tree.right), kr, kc, nodes)


CASES = {
    "toeplitz": (lambda: W.toeplitz_inverse_distance(512), dict(rtol=1e-8, d0=48, dd=16, leaf_size=32)),
    "uneven": (lambda: W.low_rank_plus_identity(129, 5, 3.0, 1), dict(rtol=1e-10, d0=16, dd=8, leaf_size=64)),
    "exact": (lambda: W.low_rank_plus_identity(300, 7, 2.0, 4), dict(rtol=1e-12, d0=20, dd=8, leaf_size=20)),
    "simple": (lambda: W.simple_toeplitz(256), dict(rtol=1e-10, d0=12, dd=4, leaf_size=16)),
    "wide_leaves": (lambda: W.toeplitz_inverse_distance(1500), dict(rtol=1e-10, d0=100, dd=50, leaf_size=300)),
}


@pytest.mark.parametrize("path", ["auto", "step", "persistent"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_ulv_on_oracle_generators(case, path, monkeypatch, capfd):
    """The LQ factorizations of the ULV factor (Householder QR without
    pivoting) on each large-problem path: one launch per step, or the
    persistent kernel (which writes to a workspace and copies back, and must
    not give up its bounded waits)."""
    if path != "auto":
        monkeypatch.setenv("HSS_QRCP_PATH", path)
    monkeypatch.setenv("HSS_VERBOSE", "1")
    make, kw = CASES[case]
    A = make()
    Ho = ohss.compress(A, ohss.Options(**kw))
    F = oulv.factor(Ho)
    h = _import(Ho)
    print(f"ulv {case}: n={A.shape[0]}, path {path}", flush=True)
    capfd.readouterr()
    P.hss_factor(h)
    assert "persistent wait gave up" not in capfd.readouterr().err
    cond = np.linalg.cond(ohss.to_dense(Ho))
    for nrhs in (1, 3, 64, 300):  # up to 64 columns: one wavefront each; 300: one thread each
        b = W.normal_rhs(A.shape[0], nrhs, 7)
        ref = oulv.solve(F, b)
        got = P.hss_solve(h, torch.from_numpy(b).cuda()).cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-14 * cond * np.linalg.norm(ref) * 10


def test_solve_requires_factor_and_single_leaf():
    A = W.toeplitz_inverse_distance(50)
    h = P.hss_compress(torch.from_numpy(A).cuda(), leaf_size=64)
    b = torch.from_numpy(W.normal_rhs(50, 2, 1)).cuda()
    with pytest.raises(P.HSSError) as e:
        P.hss_solve(h, b)
    assert e.value.status == P.HSS_ERR_STATE
    P.hss_factor(h)
    x = P.hss_solve(h, b).cpu().numpy()
    assert np.allclose(x, np.linalg.solve(A, b.cpu().numpy()), rtol=0, atol=1e-12)


def test_compress_factor_solve_toeplitz1024():
    cfg = W.CONFIGS["toeplitz1024"]
    A = W.toeplitz_inverse_distance(cfg["n"])
    h = P.hss_compress(torch.from_numpy(A).cuda(), rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"])
    P.hss_factor(h)
    b = torch.from_numpy(W.normal_rhs(cfg["n"], 4, 3)).cuda()
    x = P.hss_solve(h, b)
    r_hss = P.hss_matvec(h, x) - b
    assert float(torch.linalg.norm(r_hss) / torch.linalg.norm(b)) < 1e-11
    xn = x.cpu().numpy()
    assert np.linalg.norm(A @ xn - b.cpu().numpy()) / (np.linalg.norm(A, 2) * np.linalg.norm(xn)) <= 10 * cfg["rtol"]


def test_compress_factor_solve_circle16384():
    cfg = W.CONFIGS["circle16384"]
    pts = W.circle_points(cfg["n"], cfg["point_seed"])
    A = W.device_kernel_matrix("log", pts, torch.float64, torch.device("cuda:0"))
    print("circle16384: compress, factor, solve", flush=True)
    h = P.hss_compress(A, rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"])
    P.hss_factor(h)
    b = torch.from_numpy(W.normal_rhs(cfg["n"], 1, cfg["rhs_seed"])).cuda()
    x = P.hss_solve(h, b)
    r_hss = P.hss_matvec(h, x) - b
    assert float(torch.linalg.norm(r_hss) / torch.linalg.norm(b)) < 1e-10
    r = A @ x - b
    # ||A||_2 from 30 power iterations (a lower bound: the check is at least as strict)
    v = torch.ones((cfg["n"], 1), dtype=torch.float64, device="cuda")
    for _ in range(30):
        v = A @ v
        v = v / torch.linalg.norm(v)
    anorm = float(torch.linalg.norm(A @ v))
    assert float(torch.linalg.norm(r)) / (anorm * float(torch.linalg.norm(x))) <= 10 * cfg["rtol"]


@pytest.mark.parametrize("path", ["auto", "step", "persistent"])
@pytest.mark.parametrize("n", [1500, 3000])
def test_large_root_lu(n, path, monkeypatch, capfd):
    """A matrix without low-rank structure (random plus a diagonal shift):
    the off-diagonal ranks are full, so the root block has about n rows and
    its partial-pivoting LU takes the register panel kernel with one, two
    and four rows per thread (panels of more than 1024 and 2048 rows).  The
    solve must reproduce x with the accuracy of a dense LU."""
    g = np.random.default_rng(n)
    A = torch.from_numpy(g.standard_normal((n, n)) / np.sqrt(n) + 3.0 * np.eye(n)).cuda()
    print(f"large root LU: n={n}, path {path}", flush=True)
    h = P.hss_compress(A, rtol=1e-13, d0=n // 2 + 128, dd=64, d_max=n + 256, leaf_size=n // 4, p_margin=16)
    st = P.hss_stats(h)
    assert st["converged"]
    if path != "auto":  # the factor's QRs (leaves of n/4 rows: the large-problem paths)
        monkeypatch.setenv("HSS_QRCP_PATH", path)
    monkeypatch.setenv("HSS_VERBOSE", "1")
    capfd.readouterr()
    P.hss_factor(h)
    assert "persistent wait gave up" not in capfd.readouterr().err
    xs = torch.from_numpy(g.uniform(-1, 1, (n, 3))).cuda()
    b = A @ xs
    x = P.hss_solve(h, b)
    assert float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs)) < 1e-9


def test_nopiv_register_kernel_matches_pivoting_kernel(monkeypatch):
    """The circle16384 factor runs LQs of up to 128 rows and 129-256 columns
    on the 64-lane register kernel.  Its specialization for factorizations
    without pivoting (one barrier per step, no candidate search) must give
    the same factor as the pivoting kernel run in its no-pivot mode: the
    solves of two identical compressions agree bit for bit."""
    cfg = W.CONFIGS["circle16384"]
    pts = W.circle_points(cfg["n"], cfg["point_seed"])
    A = W.device_kernel_matrix("log", pts, torch.float64, torch.device("cuda:0"))
    b = torch.from_numpy(W.normal_rhs(cfg["n"], 3, 11)).cuda()
    xs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("HSS_REG_NOPIV", flag)
        print(f"circle16384 factor, HSS_REG_NOPIV={flag}", flush=True)
        h = P.hss_compress(A, rtol=cfg["rtol"], d0=cfg["d0"], dd=cfg["dd"], leaf_size=cfg["leaf"])
        P.hss_factor(h)
        xs.append(P.hss_solve(h, b))
    assert torch.equal(xs[0], xs[1])



@pytest.mark.parametrize("n", [8192, 16384])
def test_persistent_slot_ring_matches_exchange_every_step(n, monkeypatch, capfd):
    """The ULV factor of a serving-mix matrix (3-D Gaussian kernel, BF16x3
    sampling, leaves of 128, ranks up to 1024) runs its large QRs without
    pivoting on the persistent kernel, with 4 or 8 column slots per
    workgroup: the workgroups wait for every record only every 2 or 4 steps
    and for the column owner's record in between.  Every other record says
    "no candidate", so the factor must equal, bit for bit, the one whose
    launches exchange all records at every step."""
    pts = W.cube_points(n, 7)
    A = W.device_kernel_matrix("gauss", pts[W.kd_order(pts, 128)], torch.float32, torch.device("cuda:0"))
    b = torch.from_numpy(W.normal_rhs(n, 3, 5)).cuda()
    monkeypatch.setenv("HSS_VERBOSE", "2")
    xs, slots = [], []
    for flag in ("1", "0"):
        monkeypatch.setenv("HSS_QRCP_RING2", flag)
        print(f"persistent ring: n={n}, HSS_QRCP_RING2={flag}", flush=True)
        h = P.hss_compress(A, rtol=1e-6, d0=64, dd=32, d_max=1024, leaf_size=128, sample_prec="bf16x3",
                           p_margin=32)
        capfd.readouterr()
        P.hss_factor(h)
        err = capfd.readouterr().err
        assert "persistent wait gave up" not in err
        slots.append([int(l.split(" workgroups, ")[1].split(" ")[0]) for l in err.splitlines()
                      if "persistent launch:" in l])
        xs.append(P.hss_solve(h, b))
    print(f"column slots per launch: {slots}", flush=True)
    assert slots[0] and set(slots[0]) == {2}
    assert slots[1] and max(slots[1]) >= 4
    assert torch.equal(xs[0], xs[1])
