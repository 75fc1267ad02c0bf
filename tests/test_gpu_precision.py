"""Reduced-precision scoring (BF16, FP16 with power-of-two row scales, FP8
e4m3 with amax/448 row scales) on MFMA with FP32 accumulation.

Parity: the GPU scores equal, within the FP32 accumulation bound (n * 2^-24
of the condition scale, n the roundings in sequence), the exact FP64 dot
product of operands quantised here in numpy by the documented rules
(round to nearest even; FP8 saturating at 448). That pins the quantisation and
the MFMA operand handling. Against the FP64 oracle on the unquantised data the
error and the argmax agreement are reported (no pass bar beyond sanity)."""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, stacked_planes

pytestmark = pytest.mark.gpu


def q_bf16(x):
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64), np.ones(x.shape[0])


def q_f16(x):
    amax = np.abs(x).max(axis=1)
    e = np.where(amax > 0, np.frexp(amax)[1], 1)
    sh = np.where(amax > 0, (e - 1) - 14, 0)
    scale = np.ldexp(1.0, sh)
    q = (x.astype(np.float64) / scale[:, None]).astype(np.float32).astype(np.float16)
    return q.astype(np.float64), scale


def _e4m3_values():
    v = []
    for code in range(0x7F):  # 0x00 .. 0x7E, non-negative finite
        E, M = code >> 3, code & 7
        v.append(M * 2.0 ** -9 if E == 0 else (1 + M / 8) * 2.0 ** (E - 7))
    return np.array(v)


E4M3 = _e4m3_values()


def q_e4m3(x):
    amax = np.abs(x).max(axis=1).astype(np.float32)
    s = np.where(amax > 0, amax / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    y = (x.astype(np.float32) / s[:, None]).astype(np.float32)
    a = np.minimum(np.abs(y).astype(np.float64), 448.0)
    hi = np.clip(np.searchsorted(E4M3, a), 0, len(E4M3) - 1)
    lo = np.clip(hi - 1, 0, len(E4M3) - 1)
    dl, dh = a - E4M3[lo], E4M3[hi] - a
    pick = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(lo % 2 == 0, lo, hi)))
    return np.sign(y) * E4M3[pick], s.astype(np.float64)


QUANT = {"bf16": q_bf16, "fp16": q_f16, "fp8": q_e4m3}

# Products each MFMA instruction sums (32x32x16 for BF16/FP16, 32x32x64 for FP8).
K_PER_MFMA = {"bf16": 16, "fp16": 16, "fp8": 64}


def lp_tolerance(prec, D):
    """Relative bound (to sum |x_q w_q| s_x s_w + |b|) on FP32 accumulation of
    the exactly representable products: at most n = ceil(D / k) + k + 3
    roundings in sequence (the FP32 accumulator over the D / k instructions,
    the k products inside one, and the epilogue's scale product, scaling and
    bias add), each contributing at most 2^-24, so n * 2^-24."""
    k = K_PER_MFMA[prec]
    return (-(-D // k) + k + 3) * 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def data(ctx):
    g, z, labels = synth.make_crops(300, 128, 128, synth.W_PRECISION, 97)
    planes, boxes = stacked_planes(g, z)
    hist, _ = ctx.features(planes, boxes)
    torch.cuda.synchronize()
    W, b = synth.synthetic_weights(97, ctx.dim, synth.W_PRECISION)
    return hist, W, b


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_lp_scores_match_quantised_reference(ctx, data, prec):
    hist, W, b = data
    X = hist.cpu().numpy()
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    S, A = ctx.score(hist, wts)
    torch.cuda.synchronize()
    S = S.cpu().numpy().astype(np.float64)
    qx, sx = QUANT[prec](X)
    qw, sw = QUANT[prec](W)
    prod = qx @ qw.T
    ref = (sx[:, None] * sw[None, :]) * prod + b.astype(np.float64)[None, :]
    scale = (sx[:, None] * sw[None, :]) * (np.abs(qx) @ np.abs(qw).T) + np.abs(b)[None, :]
    err = np.abs(S - ref)
    tol = lp_tolerance(prec, ctx.dim)
    assert (err <= tol * scale + 1e-30).all(), f"max err/scale {(err / scale).max()} > {tol}"
    assert np.array_equal(A.cpu().numpy(), np.argmax(S.astype(np.float32), axis=1))


def test_lp_report_against_fp64_oracle(ctx, ref, data):
    hist, W, b = data
    X = hist.cpu().numpy()
    S64, A64 = ref.score_f64(X, W, b, n_threads=8)
    lines = []
    for prec in ("fp32", "bf16", "fp16", "fp8"):
        wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
        S, A = ctx.score(hist, wts)
        torch.cuda.synchronize()
        err = np.abs(S.cpu().numpy() - S64).max()
        agree = float((A.cpu().numpy() == A64).mean())
        lines.append(f"{prec}: max |S - S64| = {err:.3e}, argmax agreement {agree:.4f}")
        assert agree > 0.5
    print("\n".join(lines))


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_lp_ragged_shapes_and_argmax_only(ctx, prec):
    """N and K off the tile grid; argmax-only equals argmax of the scores."""
    rng = np.random.default_rng(5)
    X = torch.from_numpy(rng.random((301, ctx.dim), dtype=np.float32) / ctx.dim).cuda()
    W, b = synth.synthetic_weights(131, ctx.dim, synth.W_TINY)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    S, A = ctx.score(X, wts)
    _, A2 = ctx.score(X, wts, want_scores=False)
    torch.cuda.synchronize()
    assert torch.equal(A, A2)
    assert S.shape == (301, 131) and torch.isfinite(S).all()


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8"])
def test_lp_large_tiles_match_quantised_reference(ctx, data, prec):
    """Products with N >= 512 and K >= 256 run on the 256 x 256-tile kernel:
    N and K off its grid (1100 rows: the 300 feature rows tiled; 600
    identities), checked like the small-tile kernel against the exact product
    of the quantised operands."""
    hist, _, _ = data
    X = hist.repeat(4, 1)[:1100].contiguous()
    W, b = synth.synthetic_weights(600, ctx.dim, synth.W_PRECISION)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    S, A = ctx.score(X, wts)
    torch.cuda.synchronize()
    S = S.cpu().numpy().astype(np.float64)
    qx, sx = QUANT[prec](X.cpu().numpy())
    qw, sw = QUANT[prec](W)
    ref = (sx[:, None] * sw[None, :]) * (qx @ qw.T) + b.astype(np.float64)[None, :]
    scale = (sx[:, None] * sw[None, :]) * (np.abs(qx) @ np.abs(qw).T) + np.abs(b)[None, :]
    err = np.abs(S - ref)
    tol = lp_tolerance(prec, ctx.dim)
    assert (err <= tol * scale + 1e-30).all(), f"max err/scale {(err / scale).max()} > {tol}"
    assert np.array_equal(A.cpu().numpy(), np.argmax(S.astype(np.float32), axis=1))
