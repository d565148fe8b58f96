"""Reduced-precision candidate scoring followed by an exact rescore.

Test infrastructure only.

Encodings (written from their definitions, FP64 arithmetic on exact values):
* BF16: the FP32 value rounded to 8 significand bits, round-to-nearest-even,
  exponent range of FP32 (NaN stays NaN).
* FP8 E4M3 (OCP "FN" variant): 1 sign, 4 exponent bits (bias 7), 3 mantissa
  bits; largest finite 448; subnormal quantum 2^-9; no infinities, code 0x7F
  is NaN.  Encoding rounds to nearest even and saturates to +-448.
  A row is encoded with the per-row scale s = amax/448 (FP32 division) as
  code(x / s) with x / s an FP32 division, and decodes to value(code) * s.

Scoring (precision forms of the matched filter): scores of every voxel
against every atom are formed from the quantised operands and accumulated
exactly (FP64), multiplied by the atom's scale for FP8; the k best
(ties to the lower index) are re-scored from the FP32 operands in FP64 and
the best of those is the answer (ties to the lower index).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x: np.ndarray) -> np.ndarray:
    """FP32 -> nearest BF16 value (ties to even), returned as float32."""
    x = np.asarray(x, dtype=np.float32)
    xd = x.astype(np.float64)
    out = np.empty_like(xd)
    fin = np.isfinite(xd) & (xd != 0)
    a = np.abs(xd[fin])
    e = np.floor(np.log2(a))
    # guard against log2 rounding at exact powers of two
    e = np.where(2.0 ** e > a, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= a, e + 1, e)
    e = np.maximum(e, -126.0)                 # FP32 subnormals share the 2^-126 binade spacing
    q = 2.0 ** (e - 7)                        # 8 significand bits
    r = np.rint(a / q) * q                    # np.rint rounds half to even
    out[fin] = np.sign(xd[fin]) * r
    out[~fin] = xd[~fin]
    return out.astype(np.float32)


def e4m3_value(x: np.ndarray) -> np.ndarray:
    """FP32 -> nearest E4M3 value (ties to even, saturating), as float64."""
    xd = np.asarray(x, dtype=np.float32).astype(np.float64)
    out = np.full_like(xd, np.nan)
    fin = np.isfinite(xd)
    a = np.abs(xd[fin])
    nz = a > 0
    e = np.full(a.shape, -6.0)
    e[nz] = np.floor(np.log2(a[nz]))
    e[nz] = np.where(2.0 ** e[nz] > a[nz], e[nz] - 1, e[nz])
    e[nz] = np.where(2.0 ** (e[nz] + 1) <= a[nz], e[nz] + 1, e[nz])
    e = np.maximum(e, -6.0)                   # subnormals: quantum 2^-9
    q = 2.0 ** (e - 3)
    r = np.minimum(np.rint(a / q) * q, E4M3_MAX)
    out[fin] = np.where(xd[fin] < 0, -r, r)
    # keep the sign of a zero (the sign bit is part of the code)
    out[fin & (xd == 0)] = xd[fin & (xd == 0)]
    return out


def e4m3_code(v: np.ndarray) -> np.ndarray:
    """E4M3 value (from e4m3_value) -> 8-bit code."""
    v = np.asarray(v, dtype=np.float64)
    code = np.zeros(v.shape, dtype=np.uint8)
    nan = ~np.isfinite(v)
    sign = (np.signbit(v) & ~nan).astype(np.uint8) << 7
    a = np.abs(np.where(nan, 0.0, v))
    sub = a < 2.0 ** -6
    m_sub = np.rint(a / 2.0 ** -9).astype(np.int64)
    e = np.floor(np.log2(np.where(sub, 1.0, a)))
    m_norm = np.rint((np.where(sub, 1.0, a) / 2.0 ** e - 1.0) * 8).astype(np.int64)
    exp_bits = np.where(sub, 0, (e + 7).astype(np.int64))
    man = np.where(sub, m_sub, m_norm)
    code = (sign | ((exp_bits & 0xF) << 3).astype(np.uint8) | (man & 0x7).astype(np.uint8))
    code = np.where(nan, np.uint8(0x7F), code).astype(np.uint8)
    return code


def e4m3_decode(code: np.ndarray) -> np.ndarray:
    c = np.asarray(code, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * 2.0 ** (e - 7))
    val = np.where((e == 15) & (m == 7), np.nan, val)
    return s * val


def row_scales_e4m3(rows32: np.ndarray) -> np.ndarray:
    """Per-row FP32 scale amax/448 (1 for an all-zero row)."""
    r = np.asarray(rows32, dtype=np.float32)
    amax = np.max(np.abs(r), axis=1)
    s = amax / np.float32(E4M3_MAX)
    return np.where(amax > 0, s, np.float32(1.0)).astype(np.float32)


def quantise_rows_e4m3(rows32: np.ndarray):
    """Returns (codes uint8 [r][K], scales float32 [r], dequantised float64)."""
    r = np.asarray(rows32, dtype=np.float32)
    s = row_scales_e4m3(r)
    q = (r / s[:, None]).astype(np.float32)       # FP32 division, correctly rounded
    v = e4m3_value(q)
    return e4m3_code(v), s, v * s[:, None].astype(np.float64)


def as_real_rows(a: np.ndarray) -> np.ndarray:
    """Complex rows [r][L] -> interleaved real rows [r][2L] (re, im, re, ...)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        out = np.empty(a.shape[:-1] + (2 * a.shape[-1],), dtype=a.real.dtype)
        out[..., 0::2] = a.real
        out[..., 1::2] = a.imag
        return out
    return a


def quantised_match(Z32: np.ndarray, Dhat32: np.ndarray, precision: str, topk: int = 8):
    """Precision form of the matched filter.

    Z32: FP32 voxel rows [n][K] (real K-vectors: Re(Z) for real atoms, the
    interleaved complex vector otherwise); Dhat32: FP32 normalised atoms
    [d][K] in the same real form.  precision in {"bf16", "fp8"}.
    Returns dict(cand [n][k] in rank order, qscore [n][k], idx [n],
    score [n] = FP64 rescore of the chosen candidate).
    """
    Z32 = np.asarray(Z32, dtype=np.float32)
    D32 = np.asarray(Dhat32, dtype=np.float32)
    if precision == "bf16":
        zq = bf16_round(Z32).astype(np.float64)
        dq = bf16_round(D32).astype(np.float64)
    elif precision == "fp8":
        _, _, zq = quantise_rows_e4m3(Z32)
        _, _, dq = quantise_rows_e4m3(D32)
    else:
        raise ValueError(precision)
    qs = zq @ dq.T
    k = min(topk, D32.shape[0])
    cand = np.argsort(-qs, axis=1, kind="stable")[:, :k]      # stable: ties -> lower index
    qscore = np.take_along_axis(qs, cand, axis=1)
    exact = np.einsum("nk,njk->nj", Z32.astype(np.float64), D32.astype(np.float64)[cand])
    top = exact.max(axis=1, keepdims=True)
    idx = np.where(exact == top, cand, np.iinfo(np.int64).max).min(axis=1)
    return dict(cand=cand, qscore=qscore, idx=idx, score=top[:, 0])
