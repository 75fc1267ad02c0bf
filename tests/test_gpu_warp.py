"""GPU parity of warped crops (Sec. 2.1, Eq. 1 affine frames; Sec. 3 resize
to 200 x 200) against the oracle: counts and FP32 features bit for bit."""
import math

import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

ONE = lbpf.ONE


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


def _frames(n, seed=0):
    return [synth.make_frame(s, seed + i, 16) for i in range(n) for s in (i % 3,)]


def _inside(fr, w, h, W, H):
    ux, uy, vx, vy, tx, ty = fr
    for x in (0, w - 1):
        for y in (0, h - 1):
            sx = (ux * x + vx * y + tx) >> 16
            sy = (uy * x + vy * y + ty) >> 16
            if not (0 <= sx < W and 0 <= sy < H):
                return False
    return True


def _random_affine(rng, W, H, n):
    """n (w, h, grey_frame, depth_frame): rotation within +-30 degrees, scale
    0.6-1.5, a little shear, output sides 3..300; the depth frame is the grey
    one moved by a few pixels (separate coordinate systems, Sec. 2.1)."""
    out = []
    while len(out) < n:
        w, h = (int(v) for v in rng.integers(3, 301, size=2))
        th = math.radians(rng.uniform(-30, 30))
        s = rng.uniform(0.6, 1.5)
        sh = rng.uniform(-0.15, 0.15)
        u = (s * math.cos(th), s * math.sin(th))
        v = (-s * math.sin(th) + sh * u[0], s * math.cos(th) + sh * u[1])
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        t = (cx - 0.5 * w * u[0] - 0.5 * h * v[0], cy - 0.5 * w * u[1] - 0.5 * h * v[1])
        gf = tuple(int(round(a * ONE)) for a in (u[0], u[1], v[0], v[1], t[0], t[1]))
        dx, dy = (int(d) for d in rng.integers(-6, 7, size=2))
        zf = gf[:4] + (gf[4] + dx * ONE + int(rng.integers(0, ONE)), gf[5] + dy * ONE)
        if _inside(gf, w, h, W, H) and _inside(zf, w, h, W, H):
            out.append((w, h, gf, zf))
    return out


def _run(ctx, ref, frames, boxes, workspace=None, **kw):
    planes = [lbpf.to_device_planes(g, z) for (g, z, _, _) in frames]
    hist, cnt = ctx.features_warped(planes, boxes, with_counts=True, workspace=workspace)
    torch.cuda.synchronize()
    f, c, _ = ref.features_warped([(g, z) for (g, z, _, _) in frames], boxes, **kw)
    return hist.cpu().numpy(), cnt.cpu().numpy().view(np.uint32), f, c


def _bitexact(gf, gc, f, c):
    assert np.array_equal(gc, c), f"counts differ in {np.count_nonzero(gc != c)} places"
    assert np.array_equal(gf.view(np.uint32), f.view(np.uint32)), "features differ"


def test_resize_faces_to_200(ctx, ref):
    """Every face box of six 640x480 frames resized to 200 x 200 (Sec. 3)."""
    frames = _frames(6)
    boxes = []
    for i, (_, _, bx, _) in enumerate(frames):
        for (x, y, w, h) in bx:
            fr = lbpf.resize_frame(int(x), int(y), int(w), int(h), 200, 200)
            boxes.append((i, 200, 200, fr, fr))
    assert len(boxes) >= 6
    _bitexact(*_run(ctx, ref, frames, boxes))


def test_random_affine_frames(ctx, ref):
    frames = _frames(2, seed=40)
    rng = np.random.default_rng([synth.SEED, 31, 1])
    boxes = [(i % 2, w, h, gf, zf)
             for i, (w, h, gf, zf) in enumerate(_random_affine(rng, 640, 480, 24))]
    _bitexact(*_run(ctx, ref, frames, boxes))


def test_identity_frames_equal_plain_boxes(ctx, ref):
    frames = _frames(3, seed=80)
    planes = [lbpf.to_device_planes(g, z) for (g, z, _, _) in frames]
    plain, wboxes = [], []
    for i, (_, _, bx, _) in enumerate(frames):
        for (x, y, w, h) in bx:
            plain.append((i, int(x), int(y), int(w), int(h)))
            fr = lbpf.box_frame(int(x), int(y))
            wboxes.append((i, int(w), int(h), fr, fr))
    a, ac = ctx.features(planes, plain, with_counts=True)
    b, bc = ctx.features_warped(planes, wboxes, with_counts=True)
    torch.cuda.synchronize()
    assert torch.equal(ac, bc)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_small_workspace_groups_equal_one_group(ctx, ref):
    frames = _frames(2, seed=120)
    rng = np.random.default_rng([synth.SEED, 31, 2])
    boxes = [(i % 2, w, h, gf, zf)
             for i, (w, h, gf, zf) in enumerate(_random_affine(rng, 640, 480, 30))]
    planes = [lbpf.to_device_planes(g, z) for (g, z, _, _) in frames]
    big, _ = ctx.features_warped(planes, boxes)
    largest = max(int(lbpf.load().lbpf_warp_crop_bytes(w, h)) for (_, w, h, _, _) in boxes)
    ws = torch.empty(largest, dtype=torch.uint8, device="cuda")
    small, _ = ctx.features_warped(planes, boxes, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(big.view(torch.int32), small.view(torch.int32))


@pytest.mark.parametrize("side", [300, 1024])
def test_large_sides(ctx, ref, side):
    """Upsampled crops wider than 256 columns (the per-pixel code path), up to
    the maximum side."""
    frames = _frames(1, seed=160)
    x, y, w, h = (int(v) for v in frames[0][2][0])
    fr = lbpf.resize_frame(x, y, w, h, side, side)
    _bitexact(*_run(ctx, ref, frames, [(0, side, side, fr, fr)]))


@pytest.mark.parametrize("kw", [dict(modality=lbpf.MOD_GREY), dict(modality=lbpf.MOD_DEPTH),
                                dict(mapping=lbpf.MAP_FULL256, grid=(1, 1))])
def test_paper_literal_configurations(ref, kw):
    """Single-modality (Table 1's rows) and the 256-bin single histogram
    (Sec. 3) on 200 x 200 resized faces."""
    require_gpu()
    grid = kw.pop("grid", (8, 8))
    c = lbpf.Context(grid=grid, **kw)
    try:
        frames = _frames(2, seed=200)
        boxes = []
        for i, (_, _, bx, _) in enumerate(frames):
            for (x, y, w, h) in bx:
                fr = lbpf.resize_frame(int(x), int(y), int(w), int(h), 200, 200)
                boxes.append((i, 200, 200, fr, fr))
        _bitexact(*_run(c, ref, frames, boxes, grid_x=grid[0], grid_y=grid[1], **kw))
    finally:
        c.close()


def test_errors(ctx):
    g, z, _, _ = _frames(1, seed=240)[0]
    planes = [lbpf.to_device_planes(g, z)]
    good = lbpf.box_frame(10, 10)
    with pytest.raises(lbpf.LbpfError):  # right edge outside the 640-wide image
        ctx.features_warped(planes, [(0, 100, 100, lbpf.box_frame(545, 0), good)])
    with pytest.raises(lbpf.LbpfError):  # floor(-0.5) = -1 on the left edge
        ctx.features_warped(planes, [(0, 50, 50, good, (ONE, 0, 0, ONE, -ONE // 2, 0))])
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbpf.LbpfError):  # workspace below one 100 x 100 crop
        ctx.features_warped(planes, [(0, 100, 100, good, good)], workspace=ws)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbpf.LbpfError):  # misaligned workspace
        ctx.features_warped(planes, [(0, 100, 100, good, good)], workspace=ws[1:])
    with pytest.raises(lbpf.LbpfError):
        ctx.features_warped(planes, [(0, 2, 100, good, good)])
