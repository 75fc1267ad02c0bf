"""Pins for the oracle's masked regional histograms and the L1-normalised feature.

The expected values are built from the (separately pinned) per-pixel codes with
a different histogram route (np.bincount over a flat index), from exact rational
arithmetic for the float rounding, and from invariants: shifting all valid
depth by a constant, masking thresholds, totals per cell and per channel.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1504_01883_amd import synth


def _uniform_table():
    codes = {0, 255}
    for L in range(1, 8):
        run = (1 << L) - 1
        for r in range(8):
            codes.add(((run << r) | (run >> (8 - r))) & 0xFF)
    built = sorted(codes)
    t = np.full(256, 58, np.int64)
    for rank, c in enumerate(built):
        t[c] = rank
    return t


U59 = _uniform_table()


def _cell_of(n, g=8):
    """Cell index of every coordinate 0..n-1 when a side of length n is cut in
    g bands at floor(i*n/g): written as the largest r with floor(r*n/g) <= y."""
    starts = [(r * n) // g for r in range(g)]
    out = np.zeros(n, np.int64)
    for y in range(n):
        out[y] = max(r for r in range(g) if starts[r] <= y)
    return out


def _expected_counts(ref, g, z, window=150):
    gc, zc, mk = ref.codes(g, z, window=window)
    h, w = z.shape
    cy, cx = _cell_of(h), _cell_of(w)
    cell = cy[:, None] * 8 + cx[None, :]
    sel = mk.astype(bool)
    counts = np.zeros(2 * 64 * 59, np.int64)
    for ch, codes in enumerate((gc, zc)):
        idx = (ch * 64 + cell[sel]) * 59 + U59[codes[sel]]
        counts += np.bincount(idx, minlength=2 * 64 * 59)
    return counts, int(sel.sum())


@pytest.mark.parametrize("size", [(3, 3), (5, 4), (9, 8), (17, 23), (40, 37), (64, 64)])
def test_counts_match_independent_histogram(ref, size):
    h, w = size
    g, z = synth.render_crop(w, h, synth.W_TINY, 3, 1000 + h)
    f, c, n_in = ref.crop_features(g, z)
    exp, n_sel = _expected_counts(ref, g, z)
    assert np.array_equal(c.astype(np.int64), exp)
    assert n_in == n_sel
    assert c[: 64 * 59].sum() == n_in and c[64 * 59:].sum() == n_in


def test_square_cells_closed_form(ref):
    """64x64 crop: cells are exact 8x8 blocks, so the per-cell totals are block
    sums of the mask (the border pixels never count)."""
    g, z = synth.render_crop(64, 64, synth.W_TINY, 1, 1001)
    _, c, n_in = ref.crop_features(g, z)
    _, _, mk = ref.codes(g, z)
    block = mk.reshape(8, 8, 8, 8).sum(axis=(1, 3)).ravel()
    per_cell = c.reshape(2, 64, 59).sum(axis=2)
    assert np.array_equal(per_cell[0], block) and np.array_equal(per_cell[1], block)
    assert mk[0].sum() == mk[-1].sum() == mk[:, 0].sum() == mk[:, -1].sum() == 0


def test_mask_thresholds(ref):
    """|d - m| < 150 is strict: centres at m +- 149 count, at m +- 150 do not,
    and zero depth never counts."""
    h, w = 9, 9
    z = np.full((h, w), 1000, np.uint16)
    g = np.zeros((h, w), np.uint8)
    # Keep the median at 1000 (most pixels are 1000).
    z[2, 2] = 1000 + 149
    z[2, 4] = 1000 - 149
    z[4, 2] = 1000 + 150
    z[4, 4] = 1000 - 150
    z[6, 6] = 0
    _, _, mk = ref.codes(g, z)
    assert ref.median(z) == 1000
    assert mk[2, 2] == 1 and mk[2, 4] == 1
    assert mk[4, 2] == 0 and mk[4, 4] == 0 and mk[6, 6] == 0
    _, c, n_in = ref.crop_features(g, z)
    assert n_in == 7 * 7 - 3


def test_depth_shift_invariance(ref):
    """Adding a constant to every valid depth moves the median with it and keeps
    every comparison, so the features do not change."""
    g, z = synth.render_crop(48, 52, synth.W_TINY, 2, 1003)
    f0, c0, n0 = ref.crop_features(g, z)
    z2 = np.where(z > 0, z.astype(np.int64) + 1234, 0).astype(np.uint16)
    f1, c1, n1 = ref.crop_features(g, z2)
    assert n0 == n1 and np.array_equal(c0, c1) and np.array_equal(f0, f1)


def test_all_zero_depth_gives_zero_feature(ref):
    g = np.random.default_rng(1).integers(0, 255, size=(20, 20)).astype(np.uint8)
    z = np.zeros((20, 20), np.uint16)
    f, c, n_in = ref.crop_features(g, z)
    assert n_in == 0 and not c.any() and not f.any()


def test_window_off_counts_every_interior_pixel(ref):
    g, z = synth.render_crop(30, 20, synth.W_TINY, 4, 1004)
    _, c, n_in = ref.crop_features(g, z, window=0)
    assert n_in == 28 * 18


def _is_nearest_float(x, num, den):
    """x is the round-to-nearest-even single-precision value of num/den."""
    q = Fraction(int(num), int(den))
    xf = Fraction(float(x))
    lo = Fraction(float(np.nextafter(np.float32(x), np.float32(-np.inf))))
    hi = Fraction(float(np.nextafter(np.float32(x), np.float32(np.inf))))
    d = abs(xf - q)
    if d < abs(lo - q) and d < abs(hi - q):
        return True
    if d == abs(lo - q) or d == abs(hi - q):  # a tie: the even mantissa wins
        return (int(np.float32(x).view(np.uint32)) & 1) == 0
    return False


def test_normalisation_is_exactly_rounded(ref):
    g, z = synth.render_crop(64, 64, synth.W_TINY, 5, 1005)
    f, c, n_in = ref.crop_features(g, z)
    T = 2 * n_in
    for v in np.unique(c):
        i = int(np.nonzero(c == v)[0][0])
        if v == 0:
            assert f[i] == 0.0
        else:
            assert _is_nearest_float(f[i], v, T)
    assert abs(float(f.astype(np.float64).sum()) - 1.0) <= f.size * 2.0 ** -24


def test_single_modality_and_full256(ref):
    g, z = synth.render_crop(33, 35, synth.W_TINY, 6, 1006)
    fb, cb, nb = ref.crop_features(g, z)
    fg, cg, ng = ref.crop_features(g, z, modality=1)
    fd, cd, nd = ref.crop_features(g, z, modality=2)
    assert nb == ng == nd
    assert np.array_equal(cg, cb[: 64 * 59]) and np.array_equal(cd, cb[64 * 59:])
    f256, c256, n256 = ref.crop_features(g, z, mapping=1)
    assert c256.size == 2 * 64 * 256 and n256 == nb
    folded = np.zeros(2 * 64 * 59, np.int64)
    src = c256.reshape(2 * 64, 256).astype(np.int64)
    for code in range(256):
        folded.reshape(2 * 64, 59)[:, U59[code]] += src[:, code]
    assert np.array_equal(folded, cb.astype(np.int64))


def test_crop_in_frame_equals_crop_alone(ref):
    """Boxes read in place: a crop cut from a larger image gives the same
    features as the same pixels passed alone (no halo from outside the box)."""
    rng = np.random.default_rng(7)
    G = rng.integers(0, 255, size=(60, 70)).astype(np.uint8)
    Z = rng.integers(900, 1100, size=(60, 70)).astype(np.uint16)
    boxes = [[0, 5, 7, 30, 25], [0, 0, 0, 70, 60], [0, 40, 30, 3, 3]]
    f, c, n = ref.features([(G, Z)], boxes)
    for i, (_, x, y, w, h) in enumerate(boxes):
        f1, c1, n1 = ref.crop_features(G[y:y + h, x:x + w], Z[y:y + h, x:x + w])
        assert np.array_equal(c[i], c1) and np.array_equal(f[i], f1) and n[i] == n1


def test_invalid_boxes_rejected(ref):
    G = np.zeros((10, 10), np.uint8)
    Z = np.ones((10, 10), np.uint16)
    for box in ([0, 8, 0, 3, 3], [0, 0, 0, 2, 5], [1, 0, 0, 3, 3], [0, -1, 0, 3, 3]):
        with pytest.raises(ValueError):
            ref.features([(G, Z)], [box])
