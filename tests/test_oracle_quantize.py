"""Pins of the 16-bit stored form of D (oracle/quantize.py) against references
that do not come from the oracle: torch's float32 -> bfloat16 conversion,
numpy's float64 -> binary16 conversion, exact rational rounding with
fractions.Fraction, hand-placed ties, and the defining properties of the
per-beamlet scale."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import quantize
from workloads import random_csr


def _fp32_values(n, lo_exp, hi_exp, seed):
    rng = np.random.default_rng(seed)
    m = rng.uniform(1.0, 2.0, n)
    e = rng.integers(lo_exp, hi_exp, n)
    return np.ldexp(m, e).astype(np.float32)


def test_bf16_matches_torch_conversion():
    import torch
    # normal and subnormal bfloat16 range, including exact ties
    v = np.concatenate([_fp32_values(200000, -135, 3, 1),
                        np.float32(1.0) + np.float32(2.0 ** -8) * np.arange(1, 64, dtype=np.float32)])
    ours = quantize.to_bits(quantize.round_to_format(v.astype(np.float64), "bf16"), "bf16")
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_f16_matches_numpy_conversion():
    rng = np.random.default_rng(2)
    # float64 values (not only float32 ones), normal and subnormal binary16 range
    v = np.ldexp(rng.uniform(1.0, 2.0, 200000), rng.integers(-26, 1, 200000))
    ours = quantize.to_bits(quantize.round_to_format(v, "f16"), "f16")
    ref = v.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)


def _exact_round(fr: Fraction, p: int, emin: int) -> Fraction:
    """Round a positive rational to p significand bits, ties to even (brute force)."""
    e = fr.numerator.bit_length() - fr.denominator.bit_length()
    while Fraction(2) ** e > fr:
        e -= 1
    while Fraction(2) ** (e + 1) <= fr:
        e += 1
    q = Fraction(2) ** (max(e, emin) - p + 1)
    n = fr / q
    f = n.numerator // n.denominator
    rem = n - f
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and f % 2 == 1):
        f += 1
    return f * q


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_quotients_round_like_exact_rationals(fmt):
    p, emin = quantize.FORMATS[fmt]
    rng = np.random.default_rng(3)
    a = rng.uniform(0.004, 1.0, 3000).astype(np.float32)
    b = np.maximum(a, rng.uniform(0.004, 1.0, 3000).astype(np.float32))
    got = quantize.round_to_format(a.astype(np.float64) / b.astype(np.float64), fmt)
    for ai, bi, gi in zip(a, b, got):
        assert Fraction(float(gi)) == _exact_round(Fraction(float(ai)) / Fraction(float(bi)), p, emin)


def test_ties_go_to_even():
    one = 1.0
    # bfloat16 spacing above 1 is 2^-7; f16's is 2^-10
    cases = {"bf16": 2.0 ** -7, "f16": 2.0 ** -10}
    for fmt, ulp in cases.items():
        v = np.array([one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + 2.0 ** -40])
        r = quantize.round_to_format(v, fmt)
        assert r[0] == one                 # tie, even neighbour is 1
        assert r[1] == one + 2 * ulp       # tie, even neighbour is 1 + 2 ulp
        assert r[2] == one + ulp           # just above the tie


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
def test_stored_form_properties(fmt):
    A = random_csr(3000, 90, 12.0, 4, empty_frac=0.3)
    D = sp.csr_matrix((A.val, A.col_idx, A.row_ptr), shape=(A.nv, A.nb))
    S = quantize.store(D, fmt)
    p, _ = quantize.FORMATS[fmt]
    C = D.tocsc()
    # scales are the exact column maxima; each column's largest entry codes 1.0
    for i in range(A.nb):
        col = C.data[C.indptr[i]:C.indptr[i + 1]]
        if col.size:
            assert S.scale[i] == col.max()
    q = quantize.from_bits(S.q_csr, fmt)
    hit = D.data == S.scale[D.indices]
    assert np.all(q[hit] == 1.0)
    # per-entry error of D~ within half a unit in the last place of the code
    rel = np.abs(S.Dq.data - D.data.astype(np.float64)) / D.data.astype(np.float64)
    assert rel.max() <= 2.0 ** -p
    # CSR and CSC codes describe the same matrix
    Qr = sp.csr_matrix((q, D.indices, D.indptr), shape=D.shape).toarray()
    Cq = sp.csc_matrix((quantize.from_bits(S.q_csc, fmt), C.indices, C.indptr), shape=D.shape).toarray()
    assert np.array_equal(Qr, Cq)
    # D~ = s q exactly
    assert np.array_equal(S.Dq.toarray(), Qr * S.scale.astype(np.float64)[None, :])


def test_empty_and_zero_columns_take_unit_scale():
    D = sp.csr_matrix((np.array([0.5, 0.25, 0.0], np.float32), np.array([0, 0, 2]), np.array([0, 1, 3])),
                      shape=(2, 3))
    S = quantize.store(D, "bf16")
    assert list(S.scale) == [0.5, 1.0, 1.0]
    assert list(quantize.from_bits(S.q_csr, "bf16")) == [1.0, 0.5, 0.0]
