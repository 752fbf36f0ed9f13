"""hss_sample_noalloc (the sampling products S^r = (A - M) R^r,
S^c = (A - M)^T R^c of Sec. 2.2 with the library's fixed scratch as
workspace) against hss_sample, through the C ABI.

Both run the same kernels with the same launch plans, so the outputs must be
equal bit for bit.  Two calls in a row, the second smaller, in every
precision; the largest size the scratch holds and one beyond it; and, with a
device allocator installed that refuses every request, the variant still
runs (it asks for nothing) while hss_sample fails to allocate.
"""
import numpy as np
import pytest
import torch

import paper_1503_05464_amd as P

pytestmark = pytest.mark.gpu

CASES = [("f64", torch.float64), ("f64", torch.float32), ("f32", torch.float32), ("bf16x3", torch.float32)]


def _leaf_of(n, leaf):
    return (torch.arange(n, device="cuda", dtype=torch.int32) // leaf).contiguous()


def _inputs(n, ncols, dtype, prec, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn((n, n), generator=g, device="cuda", dtype=torch.float64).to(dtype)
    Rr = P.hss_random_normal(seed, 0, n, 0, ncols, sample_prec=prec)
    Rc = P.hss_random_normal(seed, 1, n, 0, ncols, sample_prec=prec)
    return A, Rr, Rc


@pytest.mark.parametrize("prec,dtype", CASES, ids=[f"{p}-{str(d)[6:]}" for p, d in CASES])
def test_noalloc_equals_hss_sample(prec, dtype):
    for n, ncols, masked in [(9000, 100, True), (3001, 40, False)]:  # the second call smaller
        print(f"noalloc {prec} {dtype} n={n} ncols={ncols} masked={masked}", flush=True)
        A, Rr, Rc = _inputs(n, ncols, dtype, prec, n)
        leaf_of = _leaf_of(n, 128) if masked else None
        ref_r, ref_c = P.hss_sample(A, Rr, Rc, leaf_of, sample_prec=prec)
        Sr = torch.full((n, ncols), float("nan"), dtype=torch.float64, device="cuda")
        Sc = torch.full((n, ncols), float("nan"), dtype=torch.float64, device="cuda")
        P.hss_sample_noalloc(A, Rr, Rc, Sr, Sc, leaf_of, sample_prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Sr, ref_r) and torch.equal(Sc, ref_c)
        # one side only
        Sc.fill_(float("nan"))
        P.hss_sample_noalloc(A, None, Rc, None, Sc, leaf_of, sample_prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Sc, ref_c)


def test_noalloc_allocates_nothing():
    n, ncols = 4096, 64
    A, Rr, Rc = _inputs(n, ncols, torch.float32, "bf16x3", 3)
    ref_r, ref_c = P.hss_sample(A, Rr, Rc, sample_prec="bf16x3")
    Sr = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
    Sc = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    asked = []

    def refuse(nbytes, dev, stream):
        asked.append(nbytes)
        return 0

    P.hss_set_allocator(refuse, lambda p, nbytes, dev, stream: None)
    try:
        print("noalloc under an allocator that refuses every request", flush=True)
        P.hss_sample_noalloc(A, Rr, Rc, Sr, Sc, sample_prec="bf16x3")
        torch.cuda.synchronize()
        assert asked == []
        with pytest.raises(P.HSSError) as ei:
            P.hss_sample(A, Rr, Rc, sample_prec="bf16x3")
        assert ei.value.status == P.HSS_ERR_ALLOC and asked
    finally:
        P.hss_set_allocator(None, None)
    assert torch.equal(Sr, ref_r) and torch.equal(Sc, ref_c)


def test_noalloc_largest_size_and_limit():
    """n = 65536 with 64 columns fills the scratch exactly in BF16x3 (two R
    copies plus three split-K partials); 80 columns need more and are
    refused on the host before any device work."""
    n = 65536
    print("noalloc n=65536 ncols=64 bf16x3 (largest)", flush=True)
    A = torch.empty((n, n), dtype=torch.float32, device="cuda")
    A.normal_()
    leaf_of = _leaf_of(n, 256)
    for ncols in (64, 8):
        Rr = P.hss_random_normal(5, 0, n, 0, ncols, sample_prec="bf16x3")
        Rc = P.hss_random_normal(5, 1, n, 0, ncols, sample_prec="bf16x3")
        ref_r, ref_c = P.hss_sample(A, Rr, Rc, leaf_of, sample_prec="bf16x3")
        Sr = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
        Sc = torch.empty((n, ncols), dtype=torch.float64, device="cuda")
        P.hss_sample_noalloc(A, Rr, Rc, Sr, Sc, leaf_of, sample_prec="bf16x3")
        torch.cuda.synchronize()
        assert torch.equal(Sr, ref_r) and torch.equal(Sc, ref_c)
        del Rr, Rc, ref_r, ref_c, Sr, Sc
    Rr = P.hss_random_normal(5, 0, n, 0, 80, sample_prec="bf16x3")
    Sr = torch.empty((n, 80), dtype=torch.float64, device="cuda")
    with pytest.raises(P.HSSError) as ei:
        P.hss_sample_noalloc(A, Rr, Rr, Sr, Sr.clone(), leaf_of, sample_prec="bf16x3")
    assert ei.value.status == P.HSS_ERR_ARG and "scratch" in str(ei.value)
    del A
    torch.cuda.empty_cache()
