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


def test_resident_handle_solve_only_requests():
    """A compress request with keep=True leaves its factored handle resident
    in the server; solve-only requests on it (1 to 64 right-hand sides, Alg.
    4) equal hss_solve on the same handle bit for bit; the handle's bytes
    count against the budget until it is released, and a released handle
    takes no more requests."""
    A, b, kw = _request(2)
    n = A.shape[0]
    srv = P.HSSServer(max_batch=8, workers=2)
    print(f"server: keep-resident compress n={n}", flush=True)
    t = srv.submit(A, b, keep=True, **kw)
    x0, info = srv.wait(t)
    h = info["handle"]
    assert info["status"] == P.HSS_OK and h is not None and h.n == n
    rhs = [torch.from_numpy(W.normal_rhs(n, k, 50 + k)).cuda() for k in (1, 7, 64, 33)]
    print("server: solve-only requests on the resident handle", flush=True)
    tickets = [srv.solve(h, r) for r in rhs]
    outs = [srv.wait(q) for q in tickets]
    for r, (x, inf) in zip(rhs, outs):
        assert inf["status"] == P.HSS_OK and inf["handle"] is None
        direct = P.hss_solve(h, r)
        torch.cuda.synchronize()
        assert torch.equal(x, direct)
        res = P.hss_matvec(h, x) - r  # the ULV solve is exact for A_HSS
        assert float(torch.linalg.norm(res) / torch.linalg.norm(r)) <= 1e-9
    # the first request's own solution equals a later solve-only one with the same b
    x1, _ = srv.wait(srv.solve(h, b))
    assert torch.equal(x1, x0)
    srv.release(h)
    with pytest.raises(P.HSSError):
        srv.solve(h, b)
    srv.close()


def test_served_results_against_oracle():
    """Each served solution against the oracle's compress -> ULV factor ->
    solve of the same matrix with the same options (Alg. 1, 3, 4; BF16x3
    requests through the oracle's rounding of R): the two HSS forms are
    approximations of A within rtol, so their solutions agree within the
    forward error bound 20 rtol cond(A)."""
    from oracle import hss as ohss
    from oracle import ulv as oulv

    reqs = [_request(q) for q in (0, 1, 4, 6)]
    reqs = [(A, b, kw) for A, b, kw in reqs if A.shape[0] <= 1200] or [_request(0)]
    srv = P.HSSServer(max_batch=8, workers=2)
    print(f"server vs oracle: {len(reqs)} requests", flush=True)
    tickets = [srv.submit(A, b, **kw) for A, b, kw in reqs]
    outs = [srv.wait(t) for t in tickets]
    srv.close()
    for (A, b, kw), (x, info) in zip(reqs, outs):
        assert info["status"] == P.HSS_OK
        An = A.cpu().numpy()
        opts = ohss.Options(rtol=kw["rtol"], d0=kw["d0"], dd=kw["dd"], d_max=kw["d_max"],
                            leaf_size=kw["leaf_size"], p_margin=kw["p_margin"],
                            sample_prec=kw["sample_prec"])
        print(f"oracle n={An.shape[0]} {kw['sample_prec']} rtol={kw['rtol']}", flush=True)
        Ho = ohss.compress(An, opts)
        xo = oulv.solve(oulv.factor(Ho), b.cpu().numpy())
        cond = float(np.linalg.cond(An.astype(np.float64)))
        rel = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
        assert rel <= 20 * kw["rtol"] * cond, (An.shape[0], rel, cond)
        assert info["d_final"] == Ho.d_final or kw["sample_prec"] != "f64", (info["d_final"], Ho.d_final)
