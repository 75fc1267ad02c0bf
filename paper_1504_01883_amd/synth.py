"""Seeded synthetic Kinect-shaped RGB-D face data.

This module only draws inputs: it holds none of the method's arithmetic (no
LBP, no median, no histogram, no scoring). Both the GPU path and the CPU
oracle are fed from it, so every test and benchmark input is reproducible from
(SEED, workload id, identity, sample) alone.

Shape of the data (the paper's recordings are not public; these stand in for
them): Kinect v1 style planes, grey u8 and depth u16 in millimetres with 0 for
invalid pixels, faces 0.5-1.5 m from the sensor (Sec. 2.1, Fig. 1 near/far),
crops of 48-256 px per side (Sec. 3 resizes to 200x200).

* grey: per identity a base level U[90,160] plus 12 Gaussian blobs (centre
  U[0.2,0.8] of the crop, sigma U[0.06,0.18] of the short side, amplitude
  U[-80,80]); per sample a jitter N(0,3 px) of the whole face and uniform
  integer noise in [-8, 8]; rounded and clipped to u8.
* depth: an ellipsoidal face (semi-axes 0.45 w x 0.47 h, centre jittered with
  the grey) whose surface is z0 + 200 (1 - sqrt(1 - r^2)) mm with z0 ~
  U[500,1500], plus 6 identity-specific relief bumps of U[-25,25] mm; the
  background is U[2500,4000] mm per crop plus integer noise in [-5,5]; 2% of
  pixels are set to 0 (invalid); rounded to u16.
"""
from __future__ import annotations

import numpy as np

SEED = 150401883

# Workload ids, used only as seed components.
W_TINY, W_UNIFORM, W_RAGGED, W_PRECISION, W_SERVING = 1, 2, 3, 4, 5


def _identity(workload: int, identity: int):
    rng = np.random.default_rng([SEED, workload, identity, 7_000_001])
    base = rng.uniform(90.0, 160.0)
    cen = rng.uniform(0.2, 0.8, size=(12, 2))
    sig = rng.uniform(0.06, 0.18, size=12)
    amp = rng.uniform(-80.0, 80.0, size=12)
    bump_c = rng.uniform(0.3, 0.7, size=(6, 2))
    bump_s = rng.uniform(0.05, 0.12, size=6)
    bump_a = rng.uniform(-25.0, 25.0, size=6)
    return base, cen, sig, amp, bump_c, bump_s, bump_a


def render_crop(w: int, h: int, workload: int, identity: int, sample: int):
    """One face crop: (grey u8 [h, w], depth u16 [h, w])."""
    base, cen, sig, amp, bump_c, bump_s, bump_a = _identity(workload, identity)
    rng = np.random.default_rng([SEED, workload, identity, sample])
    jy, jx = rng.normal(0.0, 3.0, size=2)
    ys = np.arange(h, dtype=np.float64)
    xs = np.arange(w, dtype=np.float64)
    short = float(min(w, h))

    s = sig * short
    cy = cen[:, 0] * h + jy
    cx = cen[:, 1] * w + jx
    gy = np.exp(-((ys[:, None] - cy[None, :]) ** 2) / (2.0 * s * s))
    gx = np.exp(-((xs[:, None] - cx[None, :]) ** 2) / (2.0 * s * s))
    img = base + (gy * amp) @ gx.T
    noise = rng.integers(-8, 9, size=(h, w))
    grey = np.clip(np.rint(img) + noise, 0, 255).astype(np.uint8)

    z0 = rng.uniform(500.0, 1500.0)
    ecy = (h - 1) / 2.0 + jy
    ecx = (w - 1) / 2.0 + jx
    r2 = ((ys[:, None] - ecy) / (0.47 * h)) ** 2 + ((xs[None, :] - ecx) / (0.45 * w)) ** 2
    face = r2 < 1.0
    zf = z0 + 200.0 * (1.0 - np.sqrt(np.clip(1.0 - r2, 0.0, 1.0)))
    bs = bump_s * short
    by = bump_c[:, 0] * h + jy
    bx = bump_c[:, 1] * w + jx
    hy = np.exp(-((ys[:, None] - by[None, :]) ** 2) / (2.0 * bs * bs))
    hx = np.exp(-((xs[:, None] - bx[None, :]) ** 2) / (2.0 * bs * bs))
    zf = zf + (hy * bump_a) @ hx.T
    bg = rng.uniform(2500.0, 4000.0) + rng.integers(-5, 6, size=(h, w))
    z = np.where(face, zf, bg)
    invalid = rng.random((h, w)) < 0.02
    depth = np.where(invalid, 0.0, np.clip(np.rint(z), 1, 65535)).astype(np.uint16)
    return grey, depth


def make_crops(n: int, w: int, h: int, workload: int, n_ident: int, first_sample: int = 1000):
    """n crops of one size, crop i of identity i mod n_ident and sample
    first_sample + i // n_ident. Returns grey [n, h, w] u8, depth [n, h, w] u16,
    labels [n] i32."""
    grey = np.empty((n, h, w), np.uint8)
    depth = np.empty((n, h, w), np.uint16)
    labels = np.empty((n,), np.int32)
    for i in range(n):
        ident = i % n_ident
        grey[i], depth[i] = render_crop(w, h, workload, ident, first_sample + i // n_ident)
        labels[i] = ident
    return grey, depth, labels


def make_training_set(n_ident: int, per_ident: int, w: int, h: int, workload: int):
    """Training crops: samples 0..per_ident-1 of every identity."""
    n = n_ident * per_ident
    grey = np.empty((n, h, w), np.uint8)
    depth = np.empty((n, h, w), np.uint16)
    labels = np.empty((n,), np.int32)
    i = 0
    for ident in range(n_ident):
        for s in range(per_ident):
            grey[i], depth[i] = render_crop(w, h, workload, ident, s)
            labels[i] = ident
            i += 1
    return grey, depth, labels


def stacked_boxes(n: int, w: int, h: int) -> np.ndarray:
    """Boxes of n equal crops stored one under another in a single image of
    width w and height n*h: rows of (image 0, x 0, y i*h, w, h)."""
    b = np.zeros((n, 5), np.int32)
    b[:, 2] = np.arange(n, dtype=np.int64) * h
    b[:, 3] = w
    b[:, 4] = h
    return b


def ragged_sizes(n: int, workload: int = W_RAGGED):
    """Side lengths for the ragged batch: w ~ U{48..256}, aspect a ~ U[0.8, 1.25],
    h = clamp(rint(w a), 48, 256)."""
    rng = np.random.default_rng([SEED, workload, 9_000_001])
    w = rng.integers(48, 257, size=n)
    a = rng.uniform(0.8, 1.25, size=n)
    h = np.clip(np.rint(w * a), 48, 256).astype(np.int64)
    return w.astype(np.int64), h


def _render_range(args):
    ws, hs, lo, hi, n_ident, workload, first_sample = args
    return [render_crop(int(ws[i]), int(hs[i]), workload, i % n_ident, first_sample + i // n_ident)
            for i in range(lo, hi)]


def make_ragged(n: int, n_ident: int, workload: int = W_RAGGED, first_sample: int = 1000,
                workers: int = 1):
    """n crops with ragged sizes packed into one grey and one depth pool.

    Returns (grey_pool u8 [P], depth_pool u16 [P], offsets i64 [n], sizes [n, 2]
    as (w, h), labels). Crop i occupies pool[offsets[i] : offsets[i] + w*h]
    row-major with pitch w. workers > 1 renders the crops in forked worker
    processes (call it before the process touches the GPU); the result does
    not depend on it."""
    ws, hs = ragged_sizes(n, workload)
    areas = ws * hs
    offsets = np.zeros(n, np.int64)
    offsets[1:] = np.cumsum(areas)[:-1]
    total = int(areas.sum())
    grey = np.empty(total, np.uint8)
    depth = np.empty(total, np.uint16)
    labels = (np.arange(n) % n_ident).astype(np.int32)
    step = max(1, -(-n // max(1, 4 * workers)))
    jobs = [(ws, hs, lo, min(n, lo + step), n_ident, workload, first_sample)
            for lo in range(0, n, step)]
    if workers > 1 and n > 256:
        import multiprocessing as mp
        # close + join, not the context manager's terminate(): the workers
        # then exit normally instead of being sent SIGTERM (which processes
        # running under a profiler may not survive cleanly).
        pool = mp.get_context("fork").Pool(workers)
        try:
            parts = pool.map(_render_range, jobs)
        finally:
            pool.close()
            pool.join()
    else:
        parts = [_render_range(j) for j in jobs]
    i = 0
    for part in parts:
        for g, z in part:
            grey[offsets[i]: offsets[i] + areas[i]] = g.ravel()
            depth[offsets[i]: offsets[i] + areas[i]] = z.ravel()
            i += 1
    return grey, depth, offsets, np.stack([ws, hs], axis=1), labels


def synthetic_weights(K: int, D: int, workload: int):
    """Seeded stand-in SVM weights (W [K, D] f32, b [K] f32) for timing runs
    that must not depend on a trainer: W ~ N(0, 1), b ~ N(0, 0.01)."""
    rng = np.random.default_rng([SEED, workload, 11_000_001])
    W = rng.standard_normal((K, D), dtype=np.float32)
    b = (0.01 * rng.standard_normal(K)).astype(np.float32)
    return W, b


FRAME_W, FRAME_H = 640, 480


def make_frame(stream: int, index: int, n_ident: int, workload: int = W_SERVING):
    """One Kinect-shaped 640x480 frame of stream `stream` with 1-8 faces.

    Returns (grey u8 [480, 640], depth u16 [480, 640], boxes i32 [n, 4] as
    (x, y, w, h), identities i32 [n]). Box sides are 48-256 px (aspect
    0.8-1.25), placed without overlap by rejection sampling; each face is a
    crop from render_crop pasted at its box. The grey background is a smooth
    gradient plus noise, the depth background a tilted plane in 2500-4000 mm
    plus noise, with 2% invalid (0) pixels."""
    rng = np.random.default_rng([SEED, workload, 13_000_001, stream, index])
    ys = np.arange(FRAME_H, dtype=np.float64)[:, None]
    xs = np.arange(FRAME_W, dtype=np.float64)[None, :]
    g0, gx, gy = rng.uniform(60, 180), rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1)
    grey = np.clip(np.rint(g0 + gx * xs + gy * ys) + rng.integers(-8, 9, size=(FRAME_H, FRAME_W)),
                   0, 255)
    z0, zx, zy = rng.uniform(2800, 3700), rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6)
    depth = np.clip(np.rint(z0 + zx * (xs - 320) + zy * (ys - 240)) +
                    rng.integers(-5, 6, size=(FRAME_H, FRAME_W)), 2500, 4000)
    grey = grey.astype(np.uint8)
    depth = depth.astype(np.uint16)
    want = int(rng.integers(1, 9))
    boxes, idents = [], []
    for _ in range(200):
        if len(boxes) == want:
            break
        w = int(rng.integers(48, 257))
        h = int(np.clip(np.rint(w * rng.uniform(0.8, 1.25)), 48, 256))
        h = min(h, FRAME_H)
        x = int(rng.integers(0, FRAME_W - w + 1))
        y = int(rng.integers(0, FRAME_H - h + 1))
        if any(x < bx + bw and bx < x + w and y < by + bh and by < y + h
               for bx, by, bw, bh in boxes):
            continue
        ident = int(rng.integers(0, n_ident))
        fg, fz = render_crop(w, h, workload, ident, 100_000 + stream * 10_000 + index)
        grey[y:y + h, x:x + w] = fg
        depth[y:y + h, x:x + w] = fz
        boxes.append((x, y, w, h))
        idents.append(ident)
    invalid = rng.random((FRAME_H, FRAME_W)) < 0.02
    depth[invalid] = 0
    return grey, depth, np.array(boxes, np.int32).reshape(-1, 4), np.array(idents, np.int32)
