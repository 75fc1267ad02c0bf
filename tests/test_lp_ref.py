"""Pins of the reduced-precision reference quantisers (tests/lp_ref.py)
against torch's own CPU conversions (an independent implementation of the
same IEEE / OCP roundings), on random values over a wide exponent range, on
exact midpoints (the ties-to-even cases), on subnormals and on the
saturation boundary of e4m3."""
import numpy as np
import pytest
import torch

from tests import lp_ref


def _wide_values(rng, n):
    """Random finite FP32 values whose magnitudes span 2^-30 .. 2^30."""
    mant = rng.uniform(1.0, 2.0, n)
    ex = rng.integers(-30, 31, n)
    sign = rng.choice([-1.0, 1.0], n)
    return (sign * np.ldexp(mant, ex)).astype(np.float32)


def _bf16_midpoints(rng, n):
    """FP32 values exactly halfway between two adjacent BF16 values (bit 15
    set, bits 0-14 clear), both parities of the kept bit."""
    u = rng.integers(0x00800000, 0x7F000000, n, dtype=np.uint64).astype(np.uint32)
    u = (u & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    return u.view(np.float32)


def test_bf16_matches_torch():
    rng = np.random.default_rng(11)
    x = np.concatenate([_wide_values(rng, 200_000), _bf16_midpoints(rng, 50_000),
                        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, -1e-42], np.float32)])
    got, s = lp_ref.q_bf16(x.reshape(1, -1))
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(got.ravel(), want)
    assert (s == 1.0).all()
    # The midpoints really are ties: half of them round up, half down.
    mids = x[200_000:250_000]
    up = np.abs(lp_ref.q_bf16(mids.reshape(1, -1))[0].ravel()) > np.abs(mids)
    assert 0.3 < up.mean() < 0.7


def test_f16_matches_torch_after_row_scaling():
    rng = np.random.default_rng(12)
    # Feature-like rows (non-negative, spread over several binades, zeros)
    # and weight-like rows (signed, some tiny values that land on FP16
    # subnormals after scaling).
    feat = rng.random((64, 7552)).astype(np.float32) ** 4 / 300.0
    feat[rng.random(feat.shape) < 0.3] = 0.0
    wts = rng.standard_normal((64, 7552)).astype(np.float32)
    wts[:, :50] *= np.float32(1e-7)
    for x in (feat, wts):
        got, scale = lp_ref.q_f16(x)
        assert np.all(np.log2(scale) == np.round(np.log2(scale)))  # powers of two
        amax = np.abs(x).max(axis=1) / scale
        assert ((amax >= 2.0 ** 14) & (amax < 2.0 ** 15)).all()
        y = torch.from_numpy(x / scale[:, None].astype(np.float32))  # exact: power of two
        want = y.to(torch.float16).to(torch.float64).numpy()
        assert np.array_equal(got, want)


def test_e4m3_matches_torch_in_range():
    rng = np.random.default_rng(13)
    # torch's e4m3fn conversion returns NaN above 464 (it does not saturate):
    # compare on |y| <= 464, which covers every finite rounding case.
    y = rng.uniform(-464.0, 464.0, 100_000)
    y = np.concatenate([y, np.ldexp(rng.uniform(1.0, 2.0, 50_000), rng.integers(-12, 9, 50_000))])
    mids = (lp_ref.E4M3[1:] + lp_ref.E4M3[:-1]) / 2.0  # exact ties, both parities
    y = np.concatenate([y, mids, -mids, lp_ref.E4M3, [0.0, 464.0, -464.0]]).astype(np.float32)
    y = y[np.abs(y) <= 464.0]
    got = lp_ref.e4m3_round(y)
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(got, want)


def test_e4m3_saturates_and_row_scales():
    big = np.array([464.5, 500.0, 1e6, -1e6, 448.0], np.float32)
    assert np.array_equal(lp_ref.e4m3_round(big), [448.0, 448.0, 448.0, -448.0, 448.0])
    assert len(lp_ref.E4M3) == 127 and lp_ref.E4M3[-1] == 448.0 and lp_ref.E4M3[1] == 2.0 ** -9
    rng = np.random.default_rng(14)
    x = rng.standard_normal((32, 7552)).astype(np.float32)
    q, s = lp_ref.q_e4m3(x)
    assert (np.abs(q).max(axis=1) <= 448.0).all()
    # the row maximum maps onto (or within rounding of) 448
    assert (np.abs(q).max(axis=1) >= 416.0).all()
    assert np.allclose(s, np.abs(x).max(axis=1) / 448.0, rtol=2 ** -23)
    # encoding: x times the row factor 448 / amax (both FP32), then torch's
    # saturating float8_e4m3fn rounding
    r = lp_ref.e4m3_row_factors(x)
    assert np.array_equal(r, np.float32(448.0) / np.abs(x).max(axis=1).astype(np.float32))
    y = np.clip(x * r[:, None], -448.0, 448.0).astype(np.float32)
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(q, want)


@pytest.mark.parametrize("prec,D,n", [("bf16", 7552, 472 + 16 + 3), ("fp8", 7552, 118 + 64 + 3)])
def test_lp_tolerance_counts_roundings(prec, D, n):
    assert lp_ref.lp_tolerance(prec, D) == n * 2.0 ** -24


def test_f16_split_matches_torch_and_bounds_the_remainder():
    """The split of LBPF_F16X3: h is torch's float16 of the row-scaled value,
    l torch's float16 of the (exact) FP32 remainder, and h + l reproduces the
    scaled value within 2^-22 of it plus half the smallest FP16 subnormal."""
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.random((64, 257), dtype=np.float32) / 300.0,
                        rng.standard_normal((64, 257)).astype(np.float32)])
    x[3, :] = 0.0
    x[5, 7] = 1e-30
    h, l, scale = lp_ref.f16_split(x)
    y = (x.astype(np.float64) / scale[:, None]).astype(np.float32)
    th = torch.from_numpy(y).to(torch.float16)
    assert np.array_equal(h, th.to(torch.float64).numpy())
    rem = torch.from_numpy(y) - th.to(torch.float32)
    assert np.array_equal(l, rem.to(torch.float16).to(torch.float64).numpy())
    err = np.abs(y.astype(np.float64) - h - l)
    assert (err <= 2.0 ** -22 * np.abs(y) + 2.0 ** -25).all()
    # The three products the GEMM sums approximate the FP64 dot product of the
    # scaled rows within 3 * 2^-22 of the condition scale (plus the floor).
    qx, sx = lp_ref.q_f16x3_features(x[:8])
    qw, sw = lp_ref.q_f16x3_weights(x[8:16])
    approx = (sx[:, None] * sw[None, :]) * (qx @ qw.T)
    exact = x[:8].astype(np.float64) @ x[8:16].astype(np.float64).T
    cond = np.abs(x[:8].astype(np.float64)) @ np.abs(x[8:16].astype(np.float64)).T
    floor = 257 * 2.0 ** -24 * (sx[:, None] * sw[None, :])
    assert (np.abs(approx - exact) <= 3 * 2.0 ** -22 * cond + floor).all()
