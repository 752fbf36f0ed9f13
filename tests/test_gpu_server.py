"""The serving loop (hss_server_*) on the GPU, through the C ABI.

* A mix of requests (two kernels, several sizes, two tolerances, FP64 and
  FP32 storage with BF16x3 sampling, 1 to 5 right-hand sides) submitted
  together: every result solves its system as the same calls made alone do
  -- with the QRCP path fixed the solution of the mix equals the solution
  computed alone to 1e-12, with the path left to the cost model within the
  forward error bound 20 rtol cond(A) -- and A_HSS x = b (ULV exactness)
  with the backward error against A within 10 rtol.
* A small memory budget forces requests to wait for admission: all finish,
  none starts before it was submitted, and at most the budget is in use.
* Argument errors and unknown tickets are rejected.
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _request(q):
    g = np.random.default_rng(100 + q)
    n = int(g.choice([300, 700, 1200, 2000]))
    kind = ["log", "gauss"][q % 2]
    pts = W.circle_points(n, q) if kind == "log" else W.cube_points(n, q)
    if kind == "gauss":
        pts = pts[W.kd_order(pts, 64)]
    f32 = q % 3 == 0
    A = W.device_kernel_matrix(kind, pts, torch.float32 if f32 else torch.float64, torch.device("cuda:0"))
    kw = dict(rtol=[1e-4, 1e-6][q % 2], d0=64, dd=32, d_max=1024, leaf_size=64, p_margin=32,
              sample_prec="bf16x3" if f32 else "f64")
    b = torch.from_numpy(W.normal_rhs(n, 1 + q % 5, q)).cuda()
    return A, b, kw


def _alone(A, b, kw):
    h = P.hss_compress(A, **kw)
    P.hss_factor(h)
    return P.hss_solve(h, b), h


@pytest.mark.parametrize("path", ["step", "auto"])
def test_mix_equals_alone(path, monkeypatch):
    """With the QRCP path fixed (the only choice that depends on what else
    is in a batch) a request's solution in the mix equals its solution alone
    to rounding; with the cost model choosing, the two are solutions of HSS
    approximations that may differ by a near-tie pivot, so they agree within
    the forward error bound 20 rtol cond(A)."""
    if path == "step":
        monkeypatch.setenv("HSS_QRCP_PATH", "step")
    reqs = [_request(q) for q in range(10)]
    srv = P.HSSServer(max_batch=8, workers=2)
    print(f"server: {len(reqs)} requests", flush=True)
    tickets = [srv.submit(A, b, **kw) for A, b, kw in reqs]
    outs = [srv.wait(t) for t in tickets]
    srv.close()
    for (A, b, kw), (x, info) in zip(reqs, outs):
        assert info["status"] == P.HSS_OK and info["t_submit"] <= info["t_start"] <= info["t_done"]
        xa, h = _alone(A, b, kw)
        rel = float(torch.linalg.norm(x - xa) / torch.linalg.norm(xa))
        if path == "step":
            assert rel <= 1e-12, (A.shape[0], rel)
        else:
            cond = float(torch.linalg.cond(A.double()))
            assert rel <= 20 * kw["rtol"] * cond, (A.shape[0], rel, cond)
        r_hss = P.hss_matvec(h, x) - b
        assert float(torch.linalg.norm(r_hss) / torch.linalg.norm(b)) <= 1e-9 + 10 * kw["rtol"]
        r = A.double() @ x - b
        anorm = float(torch.linalg.matrix_norm(A.double(), ord=2))
        assert float(torch.linalg.norm(r)) / (anorm * float(torch.linalg.norm(x))) <= 10 * kw["rtol"]
    assert max(o[1]["batch_size"] for o in outs) >= 2  # requests did share batches


def test_budget_forces_waiting():
    reqs = [_request(q) for q in (1, 3, 5, 7)]
    # about two of these requests fit at once
    srv = P.HSSServer(hbm_budget=2 * (8 * 2000 * 1024 * 8 + (64 << 20)), max_batch=4, workers=3)
    tickets = [srv.submit(A, b, **kw) for A, b, kw in reqs]
    infos = [srv.wait(t)[1] for t in tickets]
    srv.close()
    assert all(i["status"] == P.HSS_OK for i in infos)
    assert all(i["t_start"] >= i["t_submit"] for i in infos)


def test_server_argument_errors():
    srv = P.HSSServer()
    A = torch.eye(50, dtype=torch.float64, device="cuda")
    b = torch.ones(50, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HSSError):
        srv.submit(A, b, sample_prec="bf16x3")
    st = P.lib().hss_server_wait(srv._ptr, 12345, None)
    assert st == P.HSS_ERR_ARG and b"unknown ticket" in P.lib().hss_last_error()
    srv.close()
