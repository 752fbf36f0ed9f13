"""Reduced-precision sampling on the GPU (FP32 MFMA, and A split into three
BF16 terms on BF16 MFMA), through the C ABI.

* R drawn with a reduced sample precision equals the oracle's Philox R
  rounded the same way (round_random), except where the two FP64 normals sit
  on either side of a rounding boundary (then one unit of the kept bits
  apart, and rare).
* The products equal the oracle's FP64 products of the same FP32 A and the
  same rounded R within the accumulation bound: FP32 over chunks of 256
  values of k (plus the 32 of the slice that ends a chunk), FP64 across
  chunks: |S - S_ref| <= (288 u32 + 2 gamma_n) |A||R|, u32 = 2^-24.
* Compressions sampled in FP32 and in BF16x3 meet the acceptance bounds at
  rtol 1e-4 and 1e-6 with the same adaptive schedule as FP64 sampling (the
  error of the products is far below the ID tolerance there).
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P
import workloads as W
from oracle import hss as ohss
from oracle import philox
from oracle.tree import bisection_tree

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _gauss(n, leaf):
    p = W.cube_points(n, 4)
    p = p[W.kd_order(p, leaf)]
    return W.device_kernel_matrix("gauss", p, torch.float32, torch.device("cuda:0"))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_random_matrix_rounding(prec):
    n, c0, c1 = 3000, 5, 69
    got = P.hss_random_normal(0, 1, n, c0, c1, sample_prec=prec).cpu().numpy()
    ref = ohss.round_random(philox.gaussian_columns(0, 1, n, c0, c1), prec)
    diff = got != ref
    assert diff.mean() < 1e-3
    bits = 24 if prec == "f32" else 8
    _, e = np.frexp(np.abs(ref[diff]))
    assert np.all(np.abs(got[diff] - ref[diff]) <= np.ldexp(1.0, e - bits))


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("n,ncols,masked", [(1000, 64, False), (2048, 128, True), (4133, 64, True),
                                            (65, 3, False)])
def test_products_within_accumulation_bound(prec, n, ncols, masked):
    A = _gauss(n, 64) if n >= 256 else torch.rand((n, n), dtype=torch.float32, device="cuda")
    Rr = P.hss_random_normal(0, 0, n, 0, ncols, sample_prec=prec)
    Rc = P.hss_random_normal(0, 1, n, 0, ncols, sample_prec=prec)
    leaf_of = None
    if masked:
        tree = bisection_tree(n, 64)
        lo = np.array([tree.lo[t] for t in range(tree.n_nodes) if tree.is_leaf(t)])
        leaf_of = torch.from_numpy(np.searchsorted(lo, np.arange(n), side="right").astype(np.int32) - 1).cuda()
    print(f"mixed sample prec={prec} n={n} ncols={ncols} masked={masked}", flush=True)
    Sr, Sc = P.hss_sample(A, Rr, Rc, leaf_of, sample_prec=prec)
    torch.cuda.synchronize()
    A64 = A.double().cpu().numpy()
    if masked:
        lf = leaf_of.cpu().numpy()
        A64 = np.where(lf[:, None] == lf[None, :], 0.0, A64)
    R1, R2 = Rr.cpu().numpy(), Rc.cpu().numpy()
    ref_r, ref_c = A64 @ R1, A64.T @ R2
    g = 2 * n * U64 / (1 - n * U64)
    bnd_r = (288 * U32 + g) * (np.abs(A64) @ np.abs(R1)) + 1e-300
    bnd_c = (288 * U32 + g) * (np.abs(A64).T @ np.abs(R2)) + 1e-300
    assert np.all(np.abs(Sr.cpu().numpy() - ref_r) <= bnd_r)
    assert np.all(np.abs(Sc.cpu().numpy() - ref_c) <= bnd_c)


def test_reduced_precision_needs_fp32_storage():
    A = torch.eye(64, dtype=torch.float64, device="cuda")
    R = P.hss_random_normal(0, 0, 64, 0, 8, sample_prec="bf16x3")
    with pytest.raises(P.HSSError) as e:
        P.hss_sample(A, R, None, None, sample_prec="bf16x3")
    assert e.value.status == P.HSS_ERR_ARG
    with pytest.raises(P.HSSError):
        P.hss_compress(A, sample_prec="f32")


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("rtol", [1e-4, 1e-6])
def test_compress_gauss4096_reduced_precision(prec, rtol):
    n, leaf = 4096, 256
    A = _gauss(n, leaf)
    kw = dict(rtol=rtol, d0=128, dd=64, leaf_size=leaf, p_margin=64)
    print(f"compress gauss4096 rtol={rtol} prec={prec}", flush=True)
    h64 = P.hss_compress(A, **kw)
    h = P.hss_compress(A, sample_prec=prec, **kw)
    s64, s = P.hss_stats(h64), P.hss_stats(h)
    assert s["converged"]
    assert abs(s["d_final"] - s64["d_final"]) <= 64
    x = torch.from_numpy(np.random.default_rng(2).uniform(-1, 1, (n, 2))).cuda()
    ref = A.double() @ x
    err = float(torch.linalg.norm(P.hss_matvec(h, x) - ref) / torch.linalg.norm(ref))
    assert err <= 10 * rtol
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    frob = float(torch.linalg.norm(P.hss_matvec(h, E) - A.double()) / torch.linalg.norm(A.double()))
    assert frob <= 10 * rtol
