"""The C ABI's stream and memory contract, on the GPU:

* hss_matvec and hss_solve are stream-ordered (Alg. 2, Alg. 4): queued
  behind long work on a stream, they return before their own work has run,
  and the result, once the stream is synchronised, equals the result of the
  same call made on an idle stream bit for bit;
* hss_set_allocator: compression (Alg. 1 with the adaptive sampling of
  Sec. 3.3), matvec, ULV factor and solve with every device block taken from
  PyTorch's caching allocator give results bit-identical to the library's own
  pool, also from the serving loop's worker threads.
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _busy(stream, n=4096, reps=12):
    """Queue tens of milliseconds of work on `stream`."""
    with torch.cuda.stream(stream):
        a = torch.randn((n, n), dtype=torch.float64, device="cuda")
        for _ in range(reps):
            a = a @ a
            a = a / a.abs().max()
    return a


def _toeplitz(n=1024):
    return torch.from_numpy(W.toeplitz_inverse_distance(n)).cuda()


def test_matvec_and_solve_are_stream_ordered():
    A = _toeplitz()
    n = A.shape[0]
    h = P.hss_compress(A, rtol=1e-6, d0=64, dd=32, leaf_size=64)
    P.hss_factor(h)
    x = torch.from_numpy(W.uniform_rhs(n, 8, 1)).cuda()
    ref_b = P.hss_matvec(h, x)
    ref_x = P.hss_solve(h, x)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    for name, call in (("matvec", lambda: P.hss_matvec(h, x, stream=s)),
                       ("solve", lambda: P.hss_solve(h, x, stream=s))):
        print(f"{name}: queued behind busy work on a side stream", flush=True)
        keep = _busy(s)
        with torch.cuda.stream(s):
            out = call()
        ev = torch.cuda.Event()
        ev.record(s)
        pending = not ev.query()
        s.synchronize()
        assert pending, f"{name} returned after its work had run"
        ref = ref_b if name == "matvec" else ref_x
        assert torch.equal(out, ref), name
        del keep
    # back to back on two streams: the second call is ordered after the first
    s2 = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b1 = P.hss_matvec(h, x, stream=s)
    with torch.cuda.stream(s2):
        b2 = P.hss_matvec(h, x, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(b1, ref_b) and torch.equal(b2, ref_b)
    # destroying the handle waits for queued work
    keep = _busy(s)
    with torch.cuda.stream(s):
        b3 = P.hss_matvec(h, x, stream=s)
    P.hss_destroy(h)
    torch.cuda.synchronize()
    assert torch.equal(b3, ref_b)
    del keep


def _run_all(A, x, batch):
    h = P.hss_compress(A, rtol=1e-6, d0=64, dd=32, leaf_size=64)
    P.hss_factor(h)
    b = P.hss_matvec(h, x)
    sol = P.hss_solve(h, x)
    hs = P.hss_compress_batched(batch, rtol=1e-4, d0=32, dd=16, leaf_size=64, sample_prec="bf16x3")
    bb = P.hss_matvec_batched(hs, [x[: B.shape[0]] for B in batch])
    torch.cuda.synchronize()
    out = dict(b=b.cpu(), sol=sol.cpu(), ranks=[r.copy() for r in P.hss_ranks(h)],
               stats=P.hss_stats(h)["d_final"], bb=[t.cpu() for t in bb],
               branks=[P.hss_ranks(q)[0].copy() for q in hs])
    del h, hs
    return out


def test_torch_allocator_bit_identical():
    A = _toeplitz()
    n = A.shape[0]
    x = torch.from_numpy(W.uniform_rhs(n, 3, 2)).cuda()
    batch = []
    for q, m in enumerate((300, 517, 1000)):
        p = W.planar_points(m, 40 + q)
        p = p[W.kd_order(p, 64)]
        batch.append(W.device_kernel_matrix("laplace", p, torch.float32, torch.device("cuda:0")))
    print("default allocator", flush=True)
    ref = _run_all(A, x, batch)
    P.use_torch_allocator()
    try:
        print("torch caching allocator", flush=True)
        before = torch.cuda.memory_allocated()
        h = P.hss_compress(A, rtol=1e-6, d0=64, dd=32, leaf_size=64)
        assert torch.cuda.memory_allocated() > before  # the handle's generators live in torch's pool
        P.hss_destroy(h)
        got = _run_all(A, x, batch)
        # the serving loop's worker threads allocate through the same callbacks
        srv = P.HSSServer(hbm_budget=1 << 30, max_batch=4, workers=2)
        tickets = [srv.submit(A, x, rtol=1e-6, d0=64, dd=32, leaf_size=64) for _ in range(3)]
        served = [srv.wait(t) for t in tickets]
        srv.close()
    finally:
        P.use_torch_allocator(False)
    torch.cuda.synchronize()
    assert got["stats"] == ref["stats"]
    for a, b in zip(got["ranks"], ref["ranks"]):
        assert np.array_equal(a, b)
    assert torch.equal(got["b"], ref["b"]) and torch.equal(got["sol"], ref["sol"])
    for a, b in zip(got["bb"], ref["bb"]):
        assert torch.equal(a, b)
    for a, b in zip(got["branks"], ref["branks"]):
        assert np.array_equal(a, b)
    for xs, info in served:  # a batch of the same request: the solution of the request alone
        assert info["status"] == P.HSS_OK
        err = float(torch.linalg.norm(xs.cpu() - ref["sol"]) / torch.linalg.norm(ref["sol"]))
        assert err <= 1e-12, err
