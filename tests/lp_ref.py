"""Reference quantisers for the reduced-precision scoring tests (test
infrastructure, numpy only).

Each function returns the dequantised operand in float64 (the exact value the
matrix cores multiply, times its scale) and the per-row scale, following the
documented operand rules:

* BF16: round to nearest even, no scale;
* FP16: per-row power-of-two scale 2^(e - 15) with e the exponent of the row's
  largest magnitude (amax in [2^(e-1), 2^e)), so the row's largest value lands
  in [2^14, 2^15); the scaling is exact and the conversion rounds to nearest
  even;
* FP8 e4m3 (OCP: bias 7, largest finite 448, no infinities): per-row scale
  s = amax / 448 and factor r = 448 / amax (each an FP32 division), x r in
  FP32, rounded to nearest even on the e4m3 grid and saturated at 448.

The FP8 rounding is written as a search over the 127 non-negative e4m3 values
(decoded from the format's definition), not as bit arithmetic, and all three
are pinned against torch's own CPU conversions in tests/test_lp_ref.py.
"""
import numpy as np


def q_bf16(x):
    """Round-to-nearest-even FP32 -> BF16 on the bit pattern: add 0x7FFF plus
    the lowest kept bit, then truncate (finite inputs only)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64), np.ones(x.shape[0])


def f16_row_scales(x):
    amax = np.abs(x).max(axis=1)
    e = np.where(amax > 0, np.frexp(amax)[1], 1)
    sh = np.where(amax > 0, (e - 1) - 14, 0)
    return np.ldexp(1.0, sh)


def q_f16(x):
    scale = f16_row_scales(x)
    q = (x.astype(np.float64) / scale[:, None]).astype(np.float32).astype(np.float16)
    return q.astype(np.float64), scale


def _e4m3_values():
    v = []
    for code in range(0x7F):  # 0x00 .. 0x7E: the non-negative finite codes
        E, M = code >> 3, code & 7
        v.append(M * 2.0 ** -9 if E == 0 else (1 + M / 8) * 2.0 ** (E - 7))
    return np.array(v)


E4M3 = _e4m3_values()


def e4m3_round(y):
    """Nearest e4m3 value of float y (ties to the even code), saturating at
    448; returns float64."""
    a = np.minimum(np.abs(np.asarray(y, np.float64)), 448.0)
    hi = np.clip(np.searchsorted(E4M3, a), 0, len(E4M3) - 1)
    lo = np.clip(hi - 1, 0, len(E4M3) - 1)
    dl, dh = a - E4M3[lo], E4M3[hi] - a
    pick = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(lo % 2 == 0, lo, hi)))
    return np.sign(y) * E4M3[pick]


def e4m3_row_scales(x):
    amax = np.abs(x).max(axis=1).astype(np.float32)
    return np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)


def e4m3_row_factors(x):
    amax = np.abs(x).max(axis=1).astype(np.float32)
    safe = np.where(amax > 0, amax, np.float32(1.0)).astype(np.float32)
    return np.where(amax > 0, np.float32(448.0) / safe, np.float32(1.0)).astype(np.float32)


def q_e4m3(x):
    s = e4m3_row_scales(x)
    r = e4m3_row_factors(x)
    y = (x.astype(np.float32) * r[:, None]).astype(np.float32)
    return e4m3_round(y), s.astype(np.float64)


def f16_split(x):
    """Split FP32 rows as the library does for LBPF_F16X3: per-row
    power-of-two scale 2^sh as for FP16, y = x 2^-sh (exact in FP32),
    h = fp16(y), l = fp16(y - h) (the remainder is exact in FP32). Returns
    (h, l, scale) with h and l as float64."""
    scale = f16_row_scales(x)
    y = (np.asarray(x, np.float64) / scale[:, None]).astype(np.float32)
    h = y.astype(np.float16)
    r = (y - h.astype(np.float32)).astype(np.float32)
    l = r.astype(np.float16)
    return h.astype(np.float64), l.astype(np.float64), scale


def q_f16x3_features(x):
    """Feature rows as the GEMM reads them: [h | h | l]."""
    h, l, s = f16_split(x)
    return np.concatenate([h, h, l], axis=1), s


def q_f16x3_weights(w):
    """Weight rows: [h | l | h], so the product sums hh + hl + lh."""
    h, l, s = f16_split(w)
    return np.concatenate([h, l, h], axis=1), s


QUANT = {"bf16": q_bf16, "fp16": q_f16, "fp8": q_e4m3}
QUANT_X = dict(QUANT, f16x3=q_f16x3_features)
QUANT_W = dict(QUANT, f16x3=q_f16x3_weights)

# Products each MFMA instruction sums (32x32x16 for BF16/FP16, 32x32x64 for FP8).
K_PER_MFMA = {"bf16": 16, "fp16": 16, "fp8": 64, "f16x3": 16}
# Reduction length relative to D (split operands run three FP16 segments).
D_FACTOR = {"bf16": 1, "fp16": 1, "fp8": 1, "f16x3": 3}


def lp_tolerance(prec, D):
    """Relative bound (to sum |x_q w_q| s_x s_w + |b|) on FP32 accumulation of
    the exactly representable products: at most n = ceil(D / k) + k + 3
    roundings in sequence (the FP32 accumulator over the D / k instructions,
    the k products inside one, and the epilogue's scale product, scaling and
    bias add), each contributing at most 2^-24, so n * 2^-24."""
    k = K_PER_MFMA[prec]
    n = D * D_FACTOR[prec]
    return (-(-n // k) + k + 3) * 2.0 ** -24


def quantised_reference(X, W, b, prec):
    """(ref, scale): the exact FP64 scores of the quantised operands and the
    condition scale the tolerance is relative to."""
    qx, sx = QUANT_X[prec](X)
    qw, sw = QUANT_W[prec](W)
    ss = sx[:, None] * sw[None, :]
    ref = ss * (qx @ qw.T) + np.asarray(b, np.float64)[None, :]
    scale = ss * (np.abs(qx) @ np.abs(qw).T) + np.abs(np.asarray(b, np.float64))[None, :]
    return ref, scale
