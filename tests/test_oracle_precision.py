"""Pins of the oracle's reduced-precision random matrices (round_random) and of
a compression that uses them.

* Hand-worked ties and carries for both precisions.
* Random values: the result has at most 8 (BF16) / 24 (FP32) significant
  bits, lies within half a unit of the last kept bit, and equals the nearer
  of the two neighbouring representable values computed independently from
  frexp/ldexp, ties to the even one.
* A compression whose random matrix was rounded to BF16 still meets the
  acceptance bound (the rounded R is just another random matrix).
"""
import numpy as np
import pytest

import workloads as W
from oracle import hss as ohss

pytestmark = pytest.mark.filterwarnings("ignore")


def test_hand_worked_bf16():
    x = np.array([1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-40, -(1 + 2**-8), 255.5, 255.75,
                  2**-8 * (1 + 2**-8), 3.0])
    want = np.array([1.0, 1 + 2**-6, 1 + 2**-7, -1.0, 256.0, 256.0, 2**-8, 3.0])
    assert np.array_equal(ohss.round_random(x, "bf16x3"), want)


def test_hand_worked_f32():
    x = np.array([1 + 2**-24, 1 + 3 * 2**-24, 1 + 2**-24 + 2**-50, -(1 + 2**-24), 0.1])
    want = np.array([1.0, 1 + 2**-22, 1 + 2**-23, -1.0, 0.100000001490116119384765625])
    assert np.array_equal(ohss.round_random(x, "f32"), want)


def _nearest(x, bits):
    """Nearest value with `bits` significant bits, ties to even, by
    frexp/ldexp arithmetic on each value separately."""
    out = np.empty_like(x)
    for q, v in enumerate(x):
        if v == 0.0:
            out[q] = 0.0
            continue
        m, e = np.frexp(abs(v))            # |v| = m 2^e, m in [0.5, 1)
        scaled = np.ldexp(m, bits)         # in [2^(bits-1), 2^bits)
        lo = np.floor(scaled)
        frac = scaled - lo
        if frac > 0.5 or (frac == 0.5 and int(lo) % 2 == 1):
            lo += 1.0
        out[q] = np.copysign(np.ldexp(lo, e - bits), v)
    return out


@pytest.mark.parametrize("prec,bits", [("bf16x3", 8), ("f32", 24)])
def test_random_values(prec, bits):
    g = np.random.default_rng(3)
    x = np.concatenate([g.standard_normal(4000), g.standard_normal(1000) * 1e-30,
                        g.standard_normal(1000) * 1e20])
    r = ohss.round_random(x, prec)
    assert np.array_equal(r, _nearest(x, bits))
    m, e = np.frexp(np.abs(r))
    assert np.all(np.ldexp(m, bits) == np.floor(np.ldexp(m, bits)))  # <= bits significant bits
    _, ex = np.frexp(np.abs(x))
    assert np.all(np.abs(x - r) <= np.ldexp(1.0, ex - bits - 1))     # half a unit of the last kept bit


def test_f64_is_identity():
    x = np.random.default_rng(1).standard_normal(100)
    assert np.array_equal(ohss.round_random(x, "f64"), x)


def test_compress_with_bf16_random_matrix_meets_bound():
    n, rtol = 1024, 1e-4
    p = W.cube_points(n, 4)
    p = p[W.kd_order(p, 64)]
    A = W.kernel_rows("gauss", p, np.arange(n), np.float32).astype(np.float32)
    opts = ohss.Options(rtol=rtol, d0=64, dd=32, leaf_size=64, p_margin=10, sample_prec="bf16x3")
    H = ohss.compress(A, opts, keep_samples=True)
    R = H.samples["Rr"]
    assert np.array_equal(R, ohss.round_random(R, "bf16x3"))
    assert ohss.relative_error(A.astype(np.float64), H) <= 10 * rtol
    with pytest.raises(ValueError):
        ohss.compress(A.astype(np.float64), opts)
