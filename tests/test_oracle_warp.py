"""Pins for the oracle's warped crops (Sec. 2.1, Eq. 1 affine frame; Sec. 3
resize of the face to 200 x 200).

Each frame below is chosen so that the sampled crop equals a crop built by a
different route (NumPy slicing, np.repeat, transpose, np.rot90) whose features
come from the separately pinned plain path. A wrong sign, a swapped u/v, a
truncating instead of flooring division or an off-by-one in the offset fails
one of them.
"""
import numpy as np
import pytest

from paper_1504_01883_amd import synth

ONE = 1 << 16


def _scene(seed=0, H=300, W=260):
    rng = np.random.default_rng([synth.SEED, 77, seed])
    g, z = synth.render_crop(W, H, synth.W_TINY, seed % 5, 3000 + seed)
    # Independent noise so that a wrong sample position changes the codes.
    g = np.clip(g.astype(np.int64) + rng.integers(-20, 21, size=g.shape), 0, 255).astype(np.uint8)
    return g, z


def _plain(ref, g, z):
    h, w = z.shape
    f, c, n = ref.features([(g, z)], [[0, 0, 0, w, h]])
    return f[0], c[0], n[0]


def _warped(ref, g, z, w, h, frame, zframe=None):
    f, c, n = ref.features_warped([(g, z)], [(0, w, h, frame, zframe or frame)])
    return f[0], c[0], n[0]


def _same(a, b):
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[0].view(np.uint32), b[0].view(np.uint32))
    assert a[2] == b[2]


def test_identity_frame_is_the_box(ref):
    g, z = _scene(1)
    bx, by, w, h = 37, 21, 120, 140
    fr = (ONE, 0, 0, ONE, bx * ONE, by * ONE)
    _same(_warped(ref, g, z, w, h, fr), _plain(ref, g[by:by + h, bx:bx + w], z[by:by + h, bx:bx + w]))


def test_decimation_by_two_is_slicing(ref):
    g, z = _scene(2)
    bx, by, w, h = 10, 5, 100, 90
    fr = (2 * ONE, 0, 0, 2 * ONE, bx * ONE, by * ONE)
    sl = (slice(by, by + 2 * h, 2), slice(bx, bx + 2 * w, 2))
    _same(_warped(ref, g, z, w, h, fr), _plain(ref, g[sl], z[sl]))


def test_resize_to_200_from_100_is_pixel_doubling(ref):
    """The Sec. 3 resize with centre sampling (t offset by half a step): a
    100 x 100 face box to 200 x 200 repeats every pixel 2 x 2."""
    g, z = _scene(3)
    bx, by = 60, 70
    u = ONE // 2
    fr = (u, 0, 0, u, bx * ONE + u // 2, by * ONE + u // 2)
    crop = (slice(by, by + 100), slice(bx, bx + 100))
    rep = lambda a: np.repeat(np.repeat(a[crop], 2, axis=0), 2, axis=1)
    _same(_warped(ref, g, z, 200, 200, fr), _plain(ref, rep(g), rep(z)))


def test_transpose_frame(ref):
    g, z = _scene(4)
    bx, by, w, h = 30, 40, 80, 110  # source box w x h; output is h x w
    fr = (0, ONE, ONE, 0, bx * ONE, by * ONE)
    src = (slice(by, by + h), slice(bx, bx + w))
    _same(_warped(ref, g, z, h, w, fr), _plain(ref, np.ascontiguousarray(g[src].T),
                                              np.ascontiguousarray(z[src].T)))


def test_rotation_frame_with_negative_steps(ref):
    """np.rot90 (counter-clockwise): out(y, x) = src(x, w - 1 - y). As a frame:
    sx = bx + w - 1 - y, sy = by + x; a negative v and a floor across zero."""
    g, z = _scene(5)
    bx, by, w, h = 50, 20, 90, 70
    src = (slice(by, by + h), slice(bx, bx + w))
    # + ONE // 3 inside the pixel: exercises floor of the fractional part.
    fr = (0, ONE, -ONE, 0, (bx + w - 1) * ONE + ONE // 3, by * ONE + ONE // 3)
    _same(_warped(ref, g, z, h, w, fr), _plain(ref, np.ascontiguousarray(np.rot90(g[src])),
                                              np.ascontiguousarray(np.rot90(z[src]))))


def test_floor_not_truncation_near_zero(ref):
    """Samples at source x = 0 from a frame that starts half a pixel left of
    the image: floor(-0.5) = -1 must be rejected, truncation would give 0."""
    g, z = _scene(6)
    fr = (ONE, 0, 0, ONE, -ONE // 2, 0)
    with pytest.raises(ValueError):
        _warped(ref, g, z, 50, 50, fr)
    ok = (ONE, 0, 0, ONE, ONE // 2, 0)  # floor(0.5 + x) = x: the plain box at 0
    _same(_warped(ref, g, z, 50, 50, ok), _plain(ref, g[:50, :50], z[:50, :50]))


def test_separate_grey_and_depth_frames(ref):
    """Grey and depth have frames of their own (different coordinate systems
    in Sec. 2.1): shifting only the depth frame equals a depth plane shifted
    the other way."""
    g, z = _scene(7)
    w, h = 100, 100
    gf = (ONE, 0, 0, ONE, 20 * ONE, 30 * ONE)
    zf = (ONE, 0, 0, ONE, 25 * ONE, 33 * ONE)
    want = _plain(ref, g[30:130, 20:120], z[33:133, 25:125])
    _same(_warped(ref, g, z, w, h, gf, zf), want)


@pytest.mark.parametrize("corner", ["right", "bottom", "negative"])
def test_out_of_plane_rejected(ref, corner):
    g, z = _scene(8)
    H, W = z.shape
    fr = {"right": (ONE, 0, 0, ONE, (W - 49) * ONE, 0),
          "bottom": (ONE, 0, 0, ONE, 0, (H - 49) * ONE),
          "negative": (ONE, 0, 0, ONE, 0, -1)}[corner]
    with pytest.raises(ValueError):
        _warped(ref, g, z, 50, 50, fr)


def test_bad_sides_rejected(ref):
    g, z = _scene(9)
    fr = (ONE, 0, 0, ONE, 0, 0)
    for w, h in [(2, 10), (10, 2), (1025, 10)]:
        with pytest.raises(ValueError):
            ref.features_warped([(g, z)], [(0, w, h, fr, fr)])
