"""GPU tests of the batching machinery: the persistent work-queue kernel, the
autotuner and HIP-graph capture. Every launch shape must give the same bits as
the oracle; graph replays must match the eager path on every replay."""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth, tune
from tests.gpu_util import require_gpu, score_tolerance

pytestmark = pytest.mark.gpu

SHAPES = [
    dict(persistent=0, wg_per_cu=4, row_prefetch=2, sorted=1),
    dict(persistent=0, wg_per_cu=4, row_prefetch=4, sorted=1),
    dict(persistent=1, wg_per_cu=1, row_prefetch=2, sorted=0),
    dict(persistent=1, wg_per_cu=2, row_prefetch=4, sorted=1),
    dict(persistent=1, wg_per_cu=4, row_prefetch=4, sorted=1),
]


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


@pytest.fixture(scope="module")
def ragged():
    """300 ragged crops (sides 48..256, aspect 0.8..1.25) packed in one pool,
    each addressed as its own image."""
    g, z, offs, sizes, labels = synth.make_ragged(300, 32)
    crops = [(g[o:o + w * h].reshape(h, w), z[o:o + w * h].reshape(h, w))
             for o, (w, h) in zip(offs, sizes)]
    return crops, labels


def _device_batch(ctx, crops):
    planes = [lbpf.to_device_planes(g, z) for g, z in crops]
    boxes = [[i, 0, 0, z.shape[1], z.shape[0]] for i, (g, z) in enumerate(crops)]
    return planes, boxes, ctx.batch(planes, boxes)


def test_every_launch_shape_bitexact(ctx, ref, ragged):
    crops, _ = ragged
    planes, boxes, b = _device_batch(ctx, crops)
    f, c, _ = ref.features(crops, boxes, n_threads=8)
    out = torch.empty((len(crops), ctx.dim), dtype=torch.float32, device="cuda")
    for shape in SHAPES:
        b.set_launch(**shape)
        assert b.get_launch() == shape
        out.fill_(-1.0)
        ctx.features_batch(b, out)
        # A second launch checks the self-resetting work queue.
        ctx.features_batch(b, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), f.view(np.uint32)), shape
    b.close()


def test_bad_launch_shape_rejected(ctx, ragged):
    crops, _ = ragged
    _, _, b = _device_batch(ctx, crops[:4])
    for bad in (dict(persistent=2), dict(wg_per_cu=0), dict(row_prefetch=3), dict(sorted=5)):
        with pytest.raises(lbpf.LbpfError):
            b.set_launch(**{**SHAPES[0], **bad})
    b.close()


def test_tuner_keeps_results(ctx, ref, ragged, tmp_path):
    crops, _ = ragged
    planes, boxes, b = _device_batch(ctx, crops)
    out = torch.empty((len(crops), ctx.dim), dtype=torch.float32, device="cuda")
    area = float(np.mean([z.size for _, z in crops]))
    r1 = tune.tuned(ctx, b, out, len(crops), area, reps=2, path=tmp_path / "t.json")
    assert not r1["cached"] and r1["us"] > 0 and b.get_launch() == r1["cfg"]
    r2 = tune.tuned(ctx, b, out, len(crops), area, reps=2, path=tmp_path / "t.json")
    assert r2["cached"] and r2["cfg"] == r1["cfg"]
    ctx.features_batch(b, out)
    torch.cuda.synchronize()
    f, _, _ = ref.features(crops, boxes, n_threads=8)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), f.view(np.uint32))
    b.close()


@pytest.mark.parametrize("persistent", [0, 1])
def test_graph_replays_match_eager(ctx, ref, ragged, persistent):
    """Capture features + scores + argmax; replay several times with eager work
    and synchronisations in between; every replay equals the eager result."""
    crops, labels = ragged
    planes, boxes, b = _device_batch(ctx, crops)
    b.set_launch(persistent=persistent, wg_per_cu=2, row_prefetch=4, sorted=1)
    K = 50
    W, bias = synth.synthetic_weights(K, ctx.dim, synth.W_RAGGED)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(bias).cuda())
    n = len(crops)
    hist = torch.empty((n, ctx.dim), dtype=torch.float32, device="cuda")
    S = torch.empty((n, K), dtype=torch.float32, device="cuda")
    A = torch.empty((n,), dtype=torch.int32, device="cuda")
    e_hist = torch.empty_like(hist)
    ctx.features_batch(b, e_hist)
    e_S, e_A = ctx.score(e_hist, wts)
    torch.cuda.synchronize()
    g = ctx.graph(b, hist, wts, S, A)
    for rep in range(4):
        hist.fill_(-1.0)
        S.fill_(0.0)
        A.fill_(-1)
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(hist, e_hist), rep
        assert torch.equal(S, e_S) and torch.equal(A, e_A), rep
        # eager work between replays
        ctx.features_batch(b, e_hist)
        torch.cuda.synchronize()
    f, _, _ = ref.features(crops, boxes, n_threads=8)
    assert np.array_equal(hist.cpu().numpy().view(np.uint32), f.view(np.uint32))
    S64, _ = ref.score_f64(f, W, bias, n_threads=8)
    assert (np.abs(S.cpu().numpy() - S64) <= score_tolerance(f, W, bias)).all()
    g.close()
    b.close()


def test_graph_features_only(ctx, ragged):
    crops, _ = ragged
    planes, boxes, b = _device_batch(ctx, crops[:50])
    hist = torch.empty((50, ctx.dim), dtype=torch.float32, device="cuda")
    ref_hist, _ = ctx.features(planes, boxes)
    g = ctx.graph(b, hist)
    for _ in range(3):
        hist.zero_()
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(hist, ref_hist)
    g.close()
    b.close()
