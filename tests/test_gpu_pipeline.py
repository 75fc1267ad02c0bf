"""The captured serving step (lbpf_pipeline_*): one HIP graph replay per batch
of face boxes over resident frames (Sec. 3's per-frame loop, many cameras
at once), batch sizes read from device memory.

Several batches in a row through one pipeline, sizes 0 .. max_boxes in
mixed order (rows of earlier, larger batches stay behind in the buffers):
  * every feature row equals the eager fused path's bit for bit, and one
    batch's rows equal the oracle's;
  * the identities copied to pinned host memory equal the device argmax,
    which is the first maximum of the pipeline's own scores;
  * FP32 scores are within 1e-5 of the FP64 oracle relative to the dot
    product's condition scale, BF16 scores within the FP32-accumulation
    bound of the exact product of the quantised operands.
"""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, score_tolerance
from tests.lp_ref import lp_tolerance, quantised_reference

pytestmark = pytest.mark.gpu

K = 300  # not a multiple of the 256-wide identity tiles
N_FRAMES = 24


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    ctx = lbpf.Context()
    frames = [synth.make_frame(s, i, K) for s in range(4) for i in range(N_FRAMES // 4)]
    planes = [lbpf.to_device_planes(g, z) for (g, z, _, _) in frames]
    table = lbpf.ImageTable(planes)
    rows = []
    for f, (_, _, bx, _) in enumerate(frames):
        for (x, y, w, h) in bx:
            rows.append([f, int(x), int(y), int(w), int(h)])
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_SERVING)
    yield ctx, frames, planes, table, np.array(rows, np.int32), W, b
    ctx.close()


def batches(all_rows, max_boxes):
    """Box subsets of mixed sizes, the largest first so later, smaller batches
    run over buffers holding stale rows."""
    rng = np.random.default_rng(5)
    sizes = [max_boxes, 1, 0, 37, max_boxes // 2, 3]
    out = []
    for n in sizes:
        idx = np.sort(rng.choice(len(all_rows), size=min(n, len(all_rows)), replace=False))
        out.append(all_rows[idx])
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_pipeline_batches_match_eager_and_oracle(setup, ref, prec):
    ctx, frames, planes, table, rows, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    max_boxes = min(64, len(rows))
    pipe = ctx.pipeline(wts, max_boxes)
    checked_oracle = False
    for bx in batches(rows, max_boxes):
        n = pipe.launch(table, bx)
        torch.cuda.synchronize()
        assert n == len(bx)
        if n == 0:
            continue
        hist = pipe.hist[:n].clone()
        S = pipe.scores[:n].cpu().numpy()
        A_dev = pipe.argmax[:n].cpu().numpy()
        A_host = pipe.argmax_host[:n].numpy().copy()
        eager, _ = ctx.features(planes, bx)
        torch.cuda.synchronize()
        assert torch.equal(hist.view(torch.int32), eager.view(torch.int32)), \
            f"{prec}: features differ from the eager path ({n} boxes)"
        assert np.array_equal(A_host, A_dev)
        assert np.array_equal(A_dev, np.argmax(S, axis=1))
        X = hist.cpu().numpy()
        if not checked_oracle:
            host = [(g, z) for (g, z, _, _) in frames]
            f, _, _ = ref.features(host, bx)
            assert np.array_equal(f.view(np.uint32), X.view(np.uint32)), "features differ from the oracle"
            checked_oracle = True
        if prec == "fp32":
            S64, _ = ref.score_f64(X, W, b)
            assert (np.abs(S.astype(np.float64) - S64) <= score_tolerance(X, W, b)).all()
        else:
            qref, scale = quantised_reference(X, W, b, prec)
            tol = lp_tolerance(prec, ctx.dim)
            assert (np.abs(S.astype(np.float64) - qref) <= tol * scale + 1e-30).all()
    pipe.close()
    wts.close()


def test_pipeline_argument_errors(setup):
    ctx, frames, planes, table, rows, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="bf16")
    pipe = ctx.pipeline(wts, 8)
    with pytest.raises(lbpf.LbpfError) as ei:
        pipe.launch(table, rows[:9])
    assert ei.value.status == lbpf.LBPF_E_BUDGET
    bad = rows[:2].copy()
    bad[1, 1] = 640 - int(bad[1, 3]) + 1  # one column past the frame's right edge
    with pytest.raises(lbpf.LbpfError) as ei:
        pipe.launch(table, bad)
    assert ei.value.status == lbpf.LBPF_E_INVALID
    # The pipeline still works after refused launches.
    pipe.launch(table, rows[:3])
    torch.cuda.synchronize()
    eager, _ = ctx.features(planes, rows[:3])
    torch.cuda.synchronize()
    assert torch.equal(pipe.hist[:3].view(torch.int32), eager.view(torch.int32))
    pipe.close()
    wts.close()
