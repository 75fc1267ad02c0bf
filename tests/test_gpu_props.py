"""Property tests of the fused feature path against the oracle (hypothesis).

Random crop sizes 3..300, random placement inside a larger frame (so the
over-read and right-edge paths are both taken), and adversarial contents:
uniform noise, constant planes, checkerboards, all-zero depth, a median within
the window of 0 (the generic counting path), saturated depth, sparse depth and
the seeded face generator. Counts and FP32 features must match the oracle bit
for bit, through the direct call and through a device-resident batch in each
launch shape (one workgroup per crop, persistent).
"""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

KINDS = ("noise", "constant", "checker", "zero_depth", "low_median", "saturated", "sparse",
         "face")


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


def _content(kind, w, h, seed):
    rng = np.random.default_rng([seed, w, h])
    if kind == "face":
        return synth.render_crop(w, h, synth.W_TINY, seed % 10, seed)
    if kind == "constant":
        return (np.full((h, w), seed % 256, np.uint8),
                np.full((h, w), 500 + seed % 3000, np.uint16))
    if kind == "checker":
        yy, xx = np.mgrid[0:h, 0:w]
        c = ((yy + xx) & 1).astype(np.int64)
        return (c * 255).astype(np.uint8), (1000 + 100 * c).astype(np.uint16)
    g = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
    if kind == "zero_depth":
        return g, np.zeros((h, w), np.uint16)
    if kind == "low_median":
        return g, rng.integers(0, 120, size=(h, w)).astype(np.uint16)
    if kind == "saturated":
        z = np.full((h, w), 65535, np.uint16)
        z[rng.random((h, w)) < 0.3] = 65400
        return g, z
    z = rng.integers(500, 1500, size=(h, w)).astype(np.uint16)
    if kind == "sparse":
        z[rng.random((h, w)) < 0.9] = 0
    else:
        z[rng.random((h, w)) < 0.05] = 0
    return g, z


crop_st = st.tuples(st.integers(3, 300), st.integers(3, 300), st.sampled_from(KINDS),
                    st.integers(0, 2**31 - 1), st.integers(0, 40), st.integers(0, 40))


@settings(max_examples=30, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture,
                                 HealthCheck.data_too_large])
@given(crops=st.lists(crop_st, min_size=1, max_size=6))
def test_random_crops_bitexact(ctx, ref, crops):
    host, planes, boxes = [], [], []
    for i, (w, h, kind, seed, px, py) in enumerate(crops):
        g, z = _content(kind, w, h, seed)
        # The crop sits at (px, py) in a frame with a random margin right and
        # below (0 margin: the crop ends at the frame's edge).
        fw, fh = w + px + (seed % 7), h + py + (seed % 5)
        G = np.zeros((fh, fw), np.uint8)
        Z = np.zeros((fh, fw), np.uint16)
        G[py:py + h, px:px + w] = g
        Z[py:py + h, px:px + w] = z
        host.append((G, Z))
        planes.append(lbpf.to_device_planes(G, Z))
        boxes.append([i, px, py, w, h])
    f, c, _ = ref.features(host, boxes, n_threads=8)

    hist, cnt = ctx.features(planes, boxes, with_counts=True)
    torch.cuda.synchronize()
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32), c), "direct call: counts differ"
    assert np.array_equal(hist.cpu().numpy().view(np.uint32), f.view(np.uint32)), \
        "direct call: features differ"

    batch = ctx.batch(planes, boxes)
    out = torch.empty((len(boxes), ctx.dim), dtype=torch.float32, device="cuda")
    counts = torch.empty((len(boxes), ctx.dim), dtype=torch.int32, device="cuda")
    for persistent in (0, 1):
        batch.set_launch(persistent=persistent, wg_per_cu=4, row_prefetch=4, sorted=1)
        ctx.features_batch(batch, out, counts_out=counts)
        torch.cuda.synchronize()
        assert np.array_equal(counts.cpu().numpy().view(np.uint32), c), \
            f"batch (persistent={persistent}): counts differ"
        assert np.array_equal(out.cpu().numpy().view(np.uint32), f.view(np.uint32)), \
            f"batch (persistent={persistent}): features differ"
    batch.close()
