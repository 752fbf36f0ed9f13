"""GPU parity of the building blocks against the oracle, through the C ABI.

Tolerances (FP64, u = 2^-53):
* random matrices: the same Philox words on both sides; the Box-Muller
  log/sqrt/cos/sin may differ by a few ulps -> |diff| <= 1e-14 max(1, |z|);
* sampling: a dot product of length K has error <= gamma_K |A||R| with
  gamma_K = K u / (1 - K u) in any summation order, so two correct
  implementations differ by at most 2 gamma_K (|A||R|) entrywise;
* ID: inputs with well separated column norms have unique pivots -> J and k
  equal exactly; E = (R1^{-1} R2)^T agrees to 1e-10 relative (the QR
  factors differ by rounding, amplified by cond(R1)).
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W
from oracle import hss as ohss
from oracle import interp, philox
from oracle.tree import bisection_tree

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _gamma(k):
    return k * U / (1 - k * U)


@pytest.mark.parametrize("n,c0,c1", [(1, 0, 1), (1001, 3, 70), (4096, 0, 128), (777, 64, 96)])
def test_random_normal_matches_oracle(n, c0, c1):
    print(f"random_normal n={n} cols=[{c0},{c1})", flush=True)
    for which in (0, 1):
        g = P.hss_random_normal(7, which, n, c0, c1).cpu().numpy()
        ref = philox.gaussian_columns(7, which, n, c0, c1)
        assert np.all(np.abs(g - ref) <= 1e-14 * np.maximum(1.0, np.abs(ref)))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,ncols,masked", [(1000, 64, False), (1000, 100, True), (2048, 128, True),
                                            (300, 7, True), (4500, 64, False)])
def test_sample_matches_oracle(dtype, n, ncols, masked):
    print(f"sample n={n} ncols={ncols} masked={masked} dtype={dtype}", flush=True)
    g = np.random.default_rng(n + ncols)
    A = W.toeplitz_inverse_distance(n) + 0.3 * g.standard_normal((n, n)) / np.sqrt(n)
    A = A.astype(np.float32 if dtype == torch.float32 else np.float64)
    A64 = A.astype(np.float64)
    Rr = g.standard_normal((n, ncols))
    Rc = g.standard_normal((n, ncols))
    Ad = torch.from_numpy(A).cuda()
    tree = bisection_tree(n, 64)
    leaf_of = None
    if masked:
        lo = np.zeros(n, dtype=np.int32)
        for q, t in enumerate(sorted(tree.leaves(), key=lambda t: tree.lo[t])):
            lo[tree.lo[t]:tree.hi[t]] = q
        leaf_of = torch.from_numpy(lo).cuda()
    Sr, Sc = P.hss_sample(Ad, torch.from_numpy(Rr).cuda(), torch.from_numpy(Rc).cuda(), leaf_of)
    torch.cuda.synchronize()
    ref_r, ref_c = ohss.sample(A64, Rr, Rc)
    absA = np.abs(A64)
    if masked:
        ref_r, ref_c = ohss.leaf_local_samples(A64, tree, ref_r, ref_c, Rr, Rc)
    bound_r = 2 * _gamma(n) * (absA @ np.abs(Rr)) + 1e-300
    bound_c = 2 * _gamma(n) * (absA.T @ np.abs(Rc)) + 1e-300
    # the masked oracle subtracts D R afterwards: add that product's error too
    if masked:
        bound_r *= 2
        bound_c *= 2
    assert np.all(np.abs(Sr.cpu().numpy() - ref_r) <= bound_r)
    assert np.all(np.abs(Sc.cpu().numpy() - ref_c) <= bound_c)


def _separated(d, m, seed, rank=None):
    g = np.random.default_rng(seed)
    y = g.standard_normal((d, m))
    if rank is not None:
        y = g.standard_normal((d, rank)) @ g.standard_normal((rank, m))
    scale = 2.0 ** (-np.arange(m) * 0.37)
    return y * scale[g.permutation(m)]


@pytest.mark.parametrize("rtol", [1e-2, 1e-6, 1e-12])
def test_id_batched_matches_oracle(rtol):
    cases = [(12, 8, None), (8, 12, None), (64, 300, None), (130, 257, None), (1, 5, None),
             (5, 1, None), (40, 25, 6), (200, 64, None), (3, 3, 0)]
    Ys, refs = [], []
    for q, (d, m, rank) in enumerate(cases):
        y = _separated(d, m, 100 + q, rank) if rank != 0 else np.zeros((d, m))
        refs.append(interp.interpolative_decomposition(y, rtol))
        Ys.append(torch.from_numpy(np.ascontiguousarray(y.T)).cuda())  # rows = columns of Y
    print(f"id_batched rtol={rtol} problems={len(cases)}", flush=True)
    got = P.hss_id_batched(Ys, rtol)
    for (k, perm, E), ref, (d, m, rank) in zip(got, refs, cases):
        assert k == ref.k, (d, m, rank)
        assert list(perm[:k]) == list(ref.J)
        assert list(perm[k:]) == list(ref.rest)
        if E.size:
            assert np.allclose(E, ref.E, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(ref.E).max()))


def test_id_ties_take_lowest_index():
    y = np.eye(6)[:, [3, 1, 5, 0, 2, 4]] * 2.0
    got = P.hss_id_batched([torch.from_numpy(np.ascontiguousarray(y.T)).cuda()], 1e-8)[0]
    ref = interp.interpolative_decomposition(y, 1e-8)
    assert got[0] == ref.k == 6 and list(got[1]) == list(ref.J) == [0, 1, 2, 3, 4, 5]


def _slow_decay(d, m, seed, rate):
    g = np.random.default_rng(seed)
    return g.standard_normal((d, m)) * (2.0 ** (-rate * np.arange(m)))[g.permutation(m)]


@pytest.mark.parametrize("cases", [[(2400, 700, 0.37, 11), (2350, 500, 0.0, 12)],
                                   [(900, 1100, 0.37, 15), (1000, 700, 0.0, 16)],
                                   [(700, 900, 0.37, 13), (650, 600, 0.0, 14)]], ids=["d2400", "d1000", "d700"])
@pytest.mark.parametrize("path", ["auto", "persistent"])
def test_id_batched_variant_problems(path, cases, monkeypatch, capfd):
    """The batch's largest d picks the persistent variant: above 2304 rows
    the one with the most rows per lane, at 1000 rows the 16-rows-per-lane
    one, at 700 rows the 12-rows-per-lane one.  Same checks as below, and
    no bounded wait of a persistent launch gave up (the results would then
    come from the per-step rerun)."""
    if path != "auto":
        monkeypatch.setenv("HSS_QRCP_PATH", path)
    monkeypatch.setenv("HSS_VERBOSE", "1")
    rtol = 1e-6
    Ys, refs, mats = [], [], []
    for d, m, rate, seed in cases:
        y = _slow_decay(d, m, seed, rate)
        mats.append(y)
        refs.append(interp.interpolative_decomposition(y, rtol))
        Ys.append(torch.from_numpy(np.ascontiguousarray(y.T)).cuda())
    print(f"id_batched variant: {len(cases)} problems, d max {max(c[0] for c in cases)}, path {path}", flush=True)
    capfd.readouterr()
    got = P.hss_id_batched(Ys, rtol)
    assert "persistent wait gave up" not in capfd.readouterr().err
    for (k, perm, E), ref, y, (d, m, rate, seed) in zip(got, refs, mats, cases):
        assert abs(k - ref.k) <= 1, (d, m, rate, k, ref.k)
        if rate >= 0.3:
            assert k == ref.k and list(perm[:k]) == list(ref.J)
            assert np.allclose(E, ref.E, rtol=1e-8, atol=1e-8 * max(1.0, np.abs(ref.E).max()))
        J, rest = perm[:k], perm[k:]
        X = np.zeros((k, m))
        X[:, J] = np.eye(k)
        if len(rest):
            X[:, rest] = E.T
        nu1 = np.linalg.norm(y, axis=0).max()
        err = np.linalg.norm(y - y[:, J] @ X, 2)
        assert err <= 10 * np.sqrt(max(1, m - k)) * rtol * nu1, (d, m, err)


_TALL_CASES = [(3300, 600, 0.37, 21), (4300, 400, 0.0, 22), (2700, 600, 0.02, 23)]


@pytest.fixture(scope="module")
def tall_refs():
    mats = [_slow_decay(d, m, seed, rate) for d, m, rate, seed in _TALL_CASES]
    return mats, [interp.interpolative_decomposition(y, 1e-6) for y in mats]


@pytest.mark.parametrize("path", ["auto", "step"])
def test_id_batched_tall_problems(path, tall_refs, monkeypatch):
    """Problems taller than the persistent kernel holds (d above 2560 rows)
    run one launch per pivot step.  While more than 4096 rows are active
    the general loop runs, after that the register variants up to 64 rows
    per lane; the 4300-row full-rank case crosses from one to the other.
    Same checks as above."""
    if path != "auto":
        monkeypatch.setenv("HSS_QRCP_PATH", path)
    rtol = 1e-6
    mats, refs = tall_refs
    Ys = [torch.from_numpy(np.ascontiguousarray(y.T)).cuda() for y in mats]
    print(f"id_batched tall: {len(mats)} problems, path {path}", flush=True)
    got = P.hss_id_batched(Ys, rtol)
    for (k, perm, E), ref, y, (d, m, rate, seed) in zip(got, refs, mats, _TALL_CASES):
        assert abs(k - ref.k) <= 1, (d, m, rate, k, ref.k)
        if rate >= 0.3:  # separated norms: the same pivots and interpolation matrix
            assert k == ref.k and list(perm[:k]) == list(ref.J)
            assert np.allclose(E, ref.E, rtol=1e-8, atol=1e-8 * max(1.0, np.abs(ref.E).max()))
        J, rest = perm[:k], perm[k:]
        X = np.zeros((k, m))
        X[:, J] = np.eye(k)
        if len(rest):
            X[:, rest] = E.T
        nu1 = np.linalg.norm(y, axis=0).max()
        err = np.linalg.norm(y - y[:, J] @ X, 2)
        assert err <= 10 * np.sqrt(max(1, m - k)) * rtol * nu1, (d, m, err)


@pytest.mark.parametrize("path", ["auto", "step", "persistent"])
def test_id_batched_large_problems(path, monkeypatch, capfd):
    """Problems on the large-problem paths (one launch per pivot step, or
    persistent launches with the columns in registers; "auto" lets the cost
    model choose): d up to 2100 rows, several workgroups per problem, more
    problems than are resident at once, and one full-rank factorization of 900
    pivot steps.  Pivots agree with the oracle while the norms are well
    separated; everywhere the rank agrees and the ID reproduces Y to its
    tolerance; no bounded wait of a persistent launch gave up."""
    if path != "auto":
        monkeypatch.setenv("HSS_QRCP_PATH", path)
    monkeypatch.setenv("HSS_VERBOSE", "1")
    rtol = 1e-6
    cases = [(2100, 1100, 0.37, 1), (2100, 1100, 0.37, 2), (2100, 1100, 0.37, 3),
             (2100, 1100, 0.37, 4), (2100, 1100, 0.37, 5), (1000, 900, 0.0, 6),
             (700, 1500, 0.02, 7)]
    Ys, refs, mats = [], [], []
    for d, m, rate, seed in cases:
        y = _slow_decay(d, m, seed, rate)
        mats.append(y)
        refs.append(interp.interpolative_decomposition(y, rtol))
        Ys.append(torch.from_numpy(np.ascontiguousarray(y.T)).cuda())
    print(f"id_batched large: {len(cases)} problems, path {path}", flush=True)
    capfd.readouterr()
    got = P.hss_id_batched(Ys, rtol)
    assert "persistent wait gave up" not in capfd.readouterr().err
    for (k, perm, E), ref, y, (d, m, rate, seed) in zip(got, refs, mats, cases):
        assert abs(k - ref.k) <= 1, (d, m, rate, k, ref.k)
        if rate >= 0.3:  # separated norms: the same pivots and interpolation matrix
            assert k == ref.k and list(perm[:k]) == list(ref.J)
            assert np.allclose(E, ref.E, rtol=1e-8, atol=1e-8 * max(1.0, np.abs(ref.E).max()))
        J, rest = perm[:k], perm[k:]
        X = np.zeros((k, m))
        X[:, J] = np.eye(k)
        if len(rest):
            X[:, rest] = E.T
        nu1 = np.linalg.norm(y, axis=0).max()
        err = np.linalg.norm(y - y[:, J] @ X, 2)
        assert err <= 10 * np.sqrt(max(1, m - k)) * rtol * nu1, (d, m, err)


def test_persistent_give_up_reruns_on_step_path(monkeypatch, capfd):
    """When a persistent launch's bounded wait gives up (forced here from the
    host: every workgroup leaves at its first wait, so every kernel exits
    normally), the problems are factored again on the per-step path from
    their untouched inputs: the IDs equal those of the step path itself,
    exactly, and match the oracle as above."""
    rtol = 1e-6
    cases = [(2100, 1100, 0.37, 11), (2100, 1100, 0.37, 12), (1000, 900, 0.0, 13)]
    mats = [_slow_decay(d, m, seed, rate) for d, m, rate, seed in cases]
    Ys = [torch.from_numpy(np.ascontiguousarray(y.T)).cuda() for y in mats]
    monkeypatch.setenv("HSS_QRCP_PATH", "step")
    print("id_batched give-up: step path reference", flush=True)
    ref_step = P.hss_id_batched(Ys, rtol)
    monkeypatch.setenv("HSS_QRCP_PATH", "persistent")
    monkeypatch.setenv("HSS_QRCP_GIVE_UP", "1")
    monkeypatch.setenv("HSS_VERBOSE", "1")
    capfd.readouterr()
    print("id_batched give-up: persistent launch that gives up", flush=True)
    got = P.hss_id_batched(Ys, rtol)
    err = capfd.readouterr().err
    assert "persistent wait gave up" in err, err
    for (k, perm, E), (k0, perm0, E0), y, (d, m, rate, seed) in zip(got, ref_step, mats, cases):
        assert k == k0 and np.array_equal(perm, perm0) and np.array_equal(E, E0)
        ref = interp.interpolative_decomposition(y, rtol)
        assert abs(k - ref.k) <= 1
        if rate >= 0.3:
            assert k == ref.k and list(perm[:k]) == list(ref.J)


@pytest.mark.parametrize("variant", list(range(-1, 7)))
def test_gemm_batched_tile_shapes(variant):
    """The batched FP64 GEMM of every per-node product (Alg. 1-4), in each
    of its tile shapes (variant -1: the tuning table's choice), against the
    FP64 product on the host: a dot product of length K differs from another
    correct one by at most 2 gamma_K |A||B| entrywise; problems cover empty
    K, single rows and columns, ragged edges of every tile and transposed A;
    every shape gives the same bits (the k order of each entry is the same)."""
    if variant >= P.hss_gemm_variants():
        pytest.skip("no such tile shape")
    g = np.random.default_rng(40)
    sizes = [(1, 1, 1, 0), (17, 5, 33, 1), (64, 64, 64, 0), (100, 130, 70, 1), (257, 3, 300, 0),
             (33, 200, 0, 0), (129, 17, 16, 1), (15, 65, 129, 0)]
    As, Bs, Cs, tr, ref, bnd = [], [], [], [], [], []
    alpha, beta = -1.5, 0.5
    for M, N, K, t in sizes:
        A = g.standard_normal((K, M) if t else (M, K))
        B = g.standard_normal((K, N))
        C = g.standard_normal((M, N))
        opA = A.T if t else A
        ref.append(alpha * (opA @ B) + beta * C)
        gam = 2 * K * U / (1 - K * U) if K else 0.0
        bnd.append(gam * abs(alpha) * (np.abs(opA) @ np.abs(B)) + 4 * U * (np.abs(alpha * (opA @ B)) + np.abs(beta * C)))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        Cs.append(torch.from_numpy(C).cuda())
        tr.append(bool(t))
    print(f"gemm_batched variant {variant}: {len(sizes)} problems", flush=True)
    out = P.hss_gemm_batched(As, Bs, [c.clone() for c in Cs], tr, alpha, beta, variant)
    base = P.hss_gemm_batched(As, Bs, [c.clone() for c in Cs], tr, alpha, beta, 0)
    torch.cuda.synchronize()
    for o, b0, r, bd in zip(out, base, ref, bnd):
        assert np.all(np.abs(o.cpu().numpy() - r) <= bd + 1e-300)
        assert torch.equal(o, b0)
