"""Reduced-precision scoring (BF16, FP16 with power-of-two row scales, FP8
e4m3 with amax/448 row scales) on MFMA with FP32 accumulation.

Parity: the GPU scores equal, within the FP32 accumulation bound (n * 2^-24
of the condition scale, n the roundings in sequence), the exact FP64 dot
product of operands quantised in numpy by the documented rules
(tests/lp_ref.py: round to nearest even; FP8 saturating at 448; pinned against
torch's own conversions). That pins the quantisation and
the MFMA operand handling. Against the FP64 oracle on the unquantised data the
error and the argmax agreement are reported (no pass bar beyond sanity)."""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, score_tolerance, stacked_planes
from tests.lp_ref import lp_tolerance, quantised_reference

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8", "f16x3"])
def test_lp_scores_match_quantised_reference(ctx, data, prec):
    hist, W, b = data
    X = hist.cpu().numpy()
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    S, A = ctx.score(hist, wts)
    torch.cuda.synchronize()
    S = S.cpu().numpy().astype(np.float64)
    ref, scale = quantised_reference(X, W, b, prec)
    err = np.abs(S - ref)
    tol = lp_tolerance(prec, ctx.dim)
    assert (err <= tol * scale + 1e-30).all(), f"max err/scale {(err / scale).max()} > {tol}"
    assert np.array_equal(A.cpu().numpy(), np.argmax(S.astype(np.float32), axis=1))


def test_lp_report_against_fp64_oracle(ctx, ref, data):
    hist, W, b = data
    X = hist.cpu().numpy()
    S64, A64 = ref.score_f64(X, W, b, n_threads=8)
    lines = []
    for prec in ("fp32", "bf16", "fp16", "fp8", "f16x3"):
        wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
        S, A = ctx.score(hist, wts)
        torch.cuda.synchronize()
        err = np.abs(S.cpu().numpy() - S64).max()
        agree = float((A.cpu().numpy() == A64).mean())
        lines.append(f"{prec}: max |S - S64| = {err:.3e}, argmax agreement {agree:.4f}")
        assert agree > 0.5
    print("\n".join(lines))


@pytest.mark.parametrize("prec", ["bf16", "fp8", "f16x3"])
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


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8", "f16x3"])
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
    ref, scale = quantised_reference(X.cpu().numpy(), W, b, prec)
    err = np.abs(S - ref)
    tol = lp_tolerance(prec, ctx.dim)
    assert (err <= tol * scale + 1e-30).all(), f"max err/scale {(err / scale).max()} > {tol}"
    assert np.array_equal(A.cpu().numpy(), np.argmax(S.astype(np.float32), axis=1))


@pytest.mark.parametrize("n,k", [(300, 97), (1100, 600)])
def test_f16x3_meets_the_fp32_bar(ctx, ref, data, n, k):
    """Split FP16 scoring against the FP64 oracle on the unquantised data: every
    score within 1e-5 of the dot product's condition scale (the FP32 bar), and
    the identities equal wherever the oracle's top-2 margin exceeds twice that
    tolerance; small tiles (300 x 97) and large tiles (1100 x 600)."""
    hist, _, _ = data
    X = hist.repeat(4, 1)[:n].contiguous()
    W, b = synth.synthetic_weights(k, ctx.dim, synth.W_PRECISION)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="f16x3")
    S, A = ctx.score(X, wts)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    S64, A64 = ref.score_f64(Xh, W, b, n_threads=8)
    tol = score_tolerance(Xh, W, b)
    err = np.abs(S.cpu().numpy().astype(np.float64) - S64)
    assert (err <= tol).all(), f"max err/tol {(err / tol).max():.3f}"
    top2 = np.sort(S64, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * tol.max(axis=1)
    assert np.array_equal(A.cpu().numpy()[clear], A64[clear])
    print(f"f16x3 {n}x{k}: max err / (1e-5 condition scale) {(err / tol).max():.4f}")
