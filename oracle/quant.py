"""Reduced-precision factor formats written from their definitions -- tests only.

The fused GPU path computes the surplus from factors stored as BF16 or as
OCP FP8 e4m3 with one power-of-two scale per concatenated factor row. To
separate kernel error from quantisation error the oracle is fed the same
quantised values, produced here independently of the GPU's packing code.

* BF16: the upper 16 bits of an IEEE binary32 after round-to-nearest-even on
  the dropped 16 bits (1 sign, 8 exponent, 7 stored significand bits).
* FP8 e4m3 (OCP "e4m3fn"): 1 sign, 4 exponent bits (bias 7), 3 significand
  bits; normal values (1 + f/8) 2^(e-7) for e = 1..15 except the all-ones
  code, subnormals (f/8) 2^-6, largest finite 448, no infinities. Rounding is
  to nearest, ties to even, saturating at +-448.
* Row scale: s = 2^e with the smallest integer e such that amax <= 448 s
  (amax = largest magnitude in the row; s = 1 for an all-zero row). A
  power-of-two scale keeps x / s exact, so the quantised value of x is
  e4m3(x / s) * s with no further rounding. The paper gives no quantisation
  (its runs use the framework's default precision); this scale rule is a
  reading of this implementation.

* Prescale: the fused GPU path multiplies both sides' factors by
  p = sqrt(log2(e) / (2 sigma)) (rounded to FP32, applied in FP32) before
  rounding, so that the product of the two packed operands is the surplus in
  log2 units, T = Phi log2(e) / (2 sigma), and K = 2^T. ``packed_rows``
  reproduces those operand values; with them the oracle computes K = 2^T.

* FP32 operands (the fused path's FP32 mode) are the FP32 products p x; no
  further rounding.

Parity status: pinned in the test suite against brute-force nearest-value
search over every BF16 / e4m3 code; ``packed_rows`` against the GPU packing
bit for bit and, with p = 1, against the plain rounding functions; its FP32
values against the exact (FP64) product rounded once to FP32.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """BF16 round-to-nearest-even of float32 values; returns float32 holding
    exactly the BF16 values (NaN stays NaN)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint32)
    nan = np.isnan(f)
    r = np.where(nan, np.uint32(0x7FC0), r).astype(np.uint32)
    return (r << np.uint32(16)).view(np.float32).reshape(f.shape)


def bf16_bits(x) -> np.ndarray:
    """The 16-bit codes of ``bf16_round(x)``."""
    return (bf16_round(x).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def e4m3_round(x) -> np.ndarray:
    """Round float64 values to the nearest e4m3 value (ties to even,
    saturating at +-448); returns float64 e4m3 values."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.clip(e, -6, 8)                 # binade; -6 also covers subnormals
    q = np.exp2(e - 3)                    # spacing of 3-bit significands
    r = np.rint(ax / q) * q               # rint = round half to even
    r = np.minimum(r, E4M3_MAX)
    return np.copysign(r, x)


def e4m3_value_table() -> np.ndarray:
    """All 256 codes decoded (NaN codes 0x7F and 0xFF give NaN)."""
    vals = np.empty(256)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        f = code & 0x7
        if e == 0xF and f == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * (f / 8.0) * 2.0 ** -6
        else:
            vals[code] = s * (1.0 + f / 8.0) * 2.0 ** (e - 7)
    return vals


def e4m3_codes(x) -> np.ndarray:
    """Byte codes of ``e4m3_round(x)`` (positive zero for zero inputs)."""
    r = e4m3_round(x)
    table = e4m3_value_table()
    out = np.zeros(r.shape, dtype=np.uint8)
    flat = r.ravel()
    o = out.ravel()
    pos = {float(v): c for c, v in enumerate(table[:128]) if not np.isnan(v)}
    for i, v in enumerate(flat):
        if v == 0.0:
            o[i] = 0x80 if np.signbit(v) else 0
        elif v > 0:
            o[i] = pos[float(v)]
        else:
            o[i] = pos[float(-v)] | 0x80
    return out


def pow2_row_scale(rows) -> np.ndarray:
    """Per-row scale 2^e, smallest e with amax <= 448 * 2^e (1 for zero rows)."""
    rows = np.asarray(rows, dtype=np.float64)
    amax = np.max(np.abs(rows), axis=1)
    mant, ex = np.frexp(amax)             # amax = mant * 2^ex, mant in [0.5, 1)
    e = np.where(mant <= 0.875, ex - 9, ex - 8)   # 448 = 0.875 * 2^9
    return np.where(amax > 0, np.ldexp(1.0, e), 1.0)


def e4m3_quantize_rows(rows):
    """(values, scale): values = e4m3(row / s) * s per row, float64."""
    rows = np.asarray(rows, dtype=np.float64)
    s = pow2_row_scale(rows)
    return e4m3_round(rows / s[:, None]) * s[:, None], s


LOG2_E = 1.4426950408889634


def prescale(sigma: float) -> np.float32:
    """p = sqrt(log2(e) / (2 sigma)) rounded to FP32 (1 for sigma = 0)."""
    if sigma <= 0:
        return np.float32(1.0)
    return np.float32(np.sqrt(np.float64(LOG2_E) / (2.0 * float(sigma))))


def packed_rows(rows, sigma: float, compute: str) -> np.ndarray:
    """FP64 values of the fused path's operand rows p [A|B] ("bf16", "fp8" or
    "f32"): the input is rounded to FP32, multiplied by p in FP32, then
    rounded to the operand type ("f32": no further rounding)."""
    x = np.asarray(rows, dtype=np.float32) * prescale(sigma)
    if compute == "f32":
        return x.astype(np.float64)
    if compute == "bf16":
        return bf16_round(x).astype(np.float64)
    q, _ = e4m3_quantize_rows(x.astype(np.float64))
    return q
