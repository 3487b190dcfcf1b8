"""FP64 oracle: D stored in 16 bits with per-beamlet float32 scales.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the library never does.

The paper keeps D in float32 (its accuracy statement in Section 3 is for
single precision).  The stored form halves the bytes of both products by
keeping, for every beamlet i,

  s_i      = max_j D_ij                      (float32, an exact maximum; 1 for
                                              a column without a positive entry)
  q_ij     = RN_t(D_ij / s_i)                t = bfloat16 or IEEE binary16, round
                                             to nearest, ties to even, of the
                                             exact quotient (gradual underflow,
                                             no overflow since q <= 1)
  D~_ij    = s_i * q_ij                      exact in float64

and both products then use D~.  The exact quotient is rounded once: for
float32 D_ij and s_i the float64 quotient is never a tie of the 16-bit format
unless the exact quotient is one, and never lies across one, so rounding the
float64 quotient gives the same code (a non-tie quotient D/s sits at least
2^-36 relative away from every tie of a format with at most 11 significand
bits, while the float64 quotient is within 2^-53).

Rounding to a 16-bit format is written out: with p significand bits and
smallest normal exponent emin, the quantum of v > 0 is 2^(max(e, emin) - p + 1)
where 2^e <= v < 2^(e+1); v / quantum is exact in float64 and np.rint rounds it
half to even.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# (significand bits including the leading one, smallest normal exponent)
FORMATS = {"bf16": (8, -126), "f16": (11, -14)}


def round_to_format(v: np.ndarray, fmt: str) -> np.ndarray:
    """RN_t of nonnegative finite float64 values, returned as float64."""
    p, emin = FORMATS[fmt]
    v = np.asarray(v, dtype=np.float64)
    if np.any(v < 0) or not np.all(np.isfinite(v)):
        raise ValueError("values must be finite and >= 0")
    out = np.zeros_like(v)
    nz = v > 0
    _, E = np.frexp(v[nz])               # v = m 2^E, 0.5 <= m < 1
    e = np.maximum(E.astype(np.int64) - 1, emin)
    quantum_exp = e - (p - 1)
    n = np.ldexp(v[nz], -quantum_exp)    # exact
    out[nz] = np.ldexp(np.rint(n), quantum_exp)
    return out


def to_bits(v: np.ndarray, fmt: str) -> np.ndarray:
    """Bit patterns (uint16) of values that are representable in the format."""
    v = np.asarray(v, dtype=np.float64)
    if fmt == "f16":
        h = v.astype(np.float16)
        if not np.array_equal(h.astype(np.float64), v):
            raise ValueError("value not representable in binary16")
        return h.view(np.uint16)
    f = v.astype(np.float32)
    if not np.array_equal(f.astype(np.float64), v):
        raise ValueError("value not representable in bfloat16")
    b = f.view(np.uint32)
    if np.any(b & 0xFFFF):
        raise ValueError("value not representable in bfloat16")
    return (b >> 16).astype(np.uint16)


def from_bits(bits: np.ndarray, fmt: str) -> np.ndarray:
    """float64 values of 16-bit patterns."""
    bits = np.asarray(bits, dtype=np.uint16)
    if fmt == "f16":
        return bits.view(np.float16).astype(np.float64)
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@dataclass
class StoredD:
    """The stored form: scales, codes in CSR and CSC order, and D~."""
    fmt: str
    scale: np.ndarray        # float32 [nb]
    q_csr: np.ndarray        # uint16 [nnz], CSR order
    q_csc: np.ndarray        # uint16 [nnz], CSC order (rows ascending per column)
    Dq: sp.csr_matrix        # float64 D~ with D's sparsity


def column_scales(D: sp.spmatrix) -> np.ndarray:
    """s_i = max_j D_ij over the stored entries of column i (1 if none is > 0)."""
    C = sp.csc_matrix(D)
    s = np.ones(C.shape[1], dtype=np.float32)
    for i in range(C.shape[1]):
        col = C.data[C.indptr[i]:C.indptr[i + 1]]
        if col.size and col.max() > 0:
            s[i] = col.max()
    return s


def store(D: sp.spmatrix, fmt: str) -> StoredD:
    """Quantise a float32 D (scipy, sorted indices) to the stored form."""
    R = sp.csr_matrix(D)
    R.sort_indices()
    if R.dtype != np.float32:
        raise ValueError("D must hold float32 values")
    s = column_scales(R)
    quot = R.data.astype(np.float64) / s[R.indices].astype(np.float64)
    q = round_to_format(quot, fmt)
    q_csr = to_bits(q, fmt)
    Dq = sp.csr_matrix((s[R.indices].astype(np.float64) * q, R.indices.copy(), R.indptr.copy()), shape=R.shape)
    C = sp.csc_matrix(sp.csr_matrix((q_csr.astype(np.float64) + 1.0, R.indices, R.indptr), shape=R.shape))
    C.sort_indices()
    q_csc = (C.data - 1.0).astype(np.uint16)
    return StoredD(fmt, s, q_csr, q_csc, Dq)
