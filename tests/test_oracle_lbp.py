"""Pins for the oracle's LBP code, uniform mapping and median.

Each test fixes the oracle to something other than its own formula: the
paper's worked example (Fig. 7), exhaustive constructions whose expected code
comes from the construction itself, geometric invariants of the 3x3 operator,
the monotone-invariance property stated in Sec. 2.4, the closed-form count of
uniform patterns, and order statistics counted by brute force.
"""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Neighbour positions used by the construction tests: (dy, dx) of neighbour p,
# top-left first, clockwise. This is the convention under test, written as a
# picture of the 3x3 window rather than as offset tables.
WINDOW_PICTURE = [
    [0, 1, 2],
    [7, None, 3],
    [6, 5, 4],
]
POS = {}
for r, row in enumerate(WINDOW_PICTURE):
    for c, p in enumerate(row):
        if p is not None:
            POS[p] = (r, c)


def rotl8(c, k):
    c = np.asarray(c, np.int64)
    return ((c << k) | (c >> (8 - k))) & 0xFF


def _patch_from_bits(bits, centre, dtype):
    """3x3 patch whose neighbour p is >= centre iff bit p of `bits` is set."""
    a = np.zeros((3, 3), dtype)
    a[1, 1] = centre
    for p in range(8):
        r, c = POS[p]
        a[r, c] = centre if (bits >> p) & 1 else centre - 1
    return a


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = v
    return out


def test_fig7_worked_example(ref):
    g = _read_golden("fig7_lbp.txt")
    pattern, value = g["pattern"][0], int(g["value"][0])
    terms = [int(t) for t in g["terms"]]
    # The printed value is the sum of the printed terms, and the terms are the
    # powers of two of the set bits read most-significant first: weights are
    # 2^p (Eq. 2's printed "2^P" cannot give 241).
    assert sum(terms) == value
    assert sorted(1 << (7 - i) for i, ch in enumerate(pattern) if ch == "1") == sorted(terms)
    bits = int(pattern, 2)
    for centre in (17, 200):
        patch = _patch_from_bits(bits, centre, np.uint8)
        assert ref.lbp_code_u8(patch, 1, 1) == value
    patch16 = _patch_from_bits(bits, 40000, np.uint16)
    assert ref.lbp_code_u16(patch16, 1, 1) == value


@pytest.mark.parametrize("centre,dtype", [(100, np.uint8), (1, np.uint8), (254, np.uint8),
                                          (30000, np.uint16), (1, np.uint16),
                                          (65534, np.uint16)])
def test_exhaustive_tie_patterns(ref, centre, dtype):
    """All 3^8 neighbourhoods with neighbours in {c-1, c, c+1}: the code has
    bit p set exactly when neighbour p is not below the centre."""
    fn = ref.lbp_code_u8 if dtype == np.uint8 else ref.lbp_code_u16
    n_uniform = 0
    for deltas in itertools.product((-1, 0, 1), repeat=8):
        a = np.full((3, 3), centre, dtype)
        expect = 0
        for p, d in enumerate(deltas):
            r, c = POS[p]
            a[r, c] = centre + d
            if d >= 0:
                expect |= 1 << p
        got = fn(a, 1, 1)
        assert got == expect, (deltas, got, expect)
        n_uniform += ref.is_uniform(got)
    assert n_uniform > 0


def test_constant_crop_gives_255(ref):
    g = np.full((9, 11), 77, np.uint8)
    z = np.full((9, 11), 1234, np.uint16)
    gc, zc, mk = ref.codes(g, z)
    assert (gc[1:-1, 1:-1] == 255).all() and (zc[1:-1, 1:-1] == 255).all()
    assert mk[1:-1, 1:-1].all()
    assert ref.uniform_bin(255) == 57


def test_bright_and_dark_centre(ref):
    """A centre above all neighbours gives 0; below all gives 255 (sign of s)."""
    a = np.full((3, 3), 10, np.uint8)
    a[1, 1] = 11
    assert ref.lbp_code_u8(a, 1, 1) == 0
    a[1, 1] = 9
    assert ref.lbp_code_u8(a, 1, 1) == 255


def _random_crop(rng, h, w, levels):
    return rng.integers(0, levels, size=(h, w))


@pytest.mark.parametrize("seed", range(4))
def test_rotation_rotates_codes(ref, seed):
    """Rotating the crop 90 degrees clockwise moves neighbour p to p+2, so each
    code becomes rotl8(code, 2). Fails for any neighbour order that is not a
    clockwise cycle starting at a corner."""
    rng = np.random.default_rng(seed)
    h, w = 7 + seed, 9 + 2 * seed
    g = _random_crop(rng, h, w, 6).astype(np.uint8)
    z = (_random_crop(rng, h, w, 5) + 1000).astype(np.uint16)
    gc, zc, _ = ref.codes(g, z, window=0)
    gr, zr, _ = ref.codes(np.rot90(g, -1), np.rot90(z, -1), window=0)
    inner = (slice(1, -1), slice(1, -1))
    assert np.array_equal(gr[inner], rotl8(np.rot90(gc, -1), 2)[inner])
    assert np.array_equal(zr[inner], rotl8(np.rot90(zc, -1), 2)[inner])


def _permute_bits(codes, perm):
    codes = np.asarray(codes, np.int64)
    out = np.zeros_like(codes)
    for new_p, old_p in enumerate(perm):
        out |= ((codes >> old_p) & 1) << new_p
    return out


@pytest.mark.parametrize("seed", range(3))
def test_mirror_and_transpose_permute_bits(ref, seed):
    """A left-right mirror swaps neighbours 0<->2, 3<->7, 4<->6; a transpose
    swaps 1<->7, 2<->6, 3<->5. Catches swapped dy/dx tables."""
    rng = np.random.default_rng(100 + seed)
    g = _random_crop(rng, 8, 10, 5).astype(np.uint8)
    z = (_random_crop(rng, 8, 10, 4) + 500).astype(np.uint16)
    gc, zc, _ = ref.codes(g, z, window=0)
    mirror = [2, 1, 0, 7, 6, 5, 4, 3]
    gm, zm, _ = ref.codes(g[:, ::-1], z[:, ::-1], window=0)
    inner = (slice(1, -1), slice(1, -1))
    assert np.array_equal(gm[inner], _permute_bits(gc[:, ::-1], mirror)[inner])
    assert np.array_equal(zm[inner], _permute_bits(zc[:, ::-1], mirror)[inner])
    transpose = [0, 7, 6, 5, 4, 3, 2, 1]
    gt, zt, _ = ref.codes(g.T, z.T, window=0)
    assert np.array_equal(gt[1:-1, 1:-1], _permute_bits(gc.T, transpose)[1:-1, 1:-1])
    assert np.array_equal(zt[1:-1, 1:-1], _permute_bits(zc.T, transpose)[1:-1, 1:-1])


@pytest.mark.parametrize("seed", range(3))
def test_monotone_invariance(ref, seed):
    """Sec. 2.4: LBP is invariant to monotonic grey-level changes. A strictly
    increasing map of the values leaves every code unchanged."""
    rng = np.random.default_rng(200 + seed)
    g = rng.integers(0, 128, size=(12, 13)).astype(np.uint8)
    z = rng.integers(1, 20000, size=(12, 13)).astype(np.uint16)
    gc, zc, _ = ref.codes(g, z, window=0)
    g2 = (2 * g.astype(np.int64) + 1).astype(np.uint8)
    lut = np.cumsum(rng.integers(1, 3, size=20000)).astype(np.int64)  # strictly increasing
    z2 = lut[z.astype(np.int64)].astype(np.uint16)
    gc2, zc2, _ = ref.codes(g2, z2, window=0)
    assert np.array_equal(gc, gc2) and np.array_equal(zc, zc2)


def _uniform_codes_by_construction():
    """Uniform codes built directly: all zeros, all ones, and every rotation of
    a run of L ones (1 <= L <= 7)."""
    codes = {0, 255}
    for L in range(1, 8):
        run = (1 << L) - 1
        for r in range(8):
            codes.add(int(rotl8(run, r)))
    return sorted(codes)


def test_uniform_count_and_ranks(ref):
    built = _uniform_codes_by_construction()
    P = 8
    assert len(built) == P * (P - 1) + 2 == 58
    oracle_uniform = [c for c in range(256) if ref.is_uniform(c)]
    assert oracle_uniform == built
    for rank, c in enumerate(built):
        assert ref.uniform_bin(c) == rank
    for c in set(range(256)) - set(built):
        assert ref.uniform_bin(c) == 58
    assert ref.uniform_bin(0) == 0 and ref.uniform_bin(255) == 57
    assert ref.uniform_bin(241) == built.index(241) == 48


def _median_by_counting(vals):
    """Lower median by the order-statistic definition: the non-zero value v
    with #(< v) <= (n-1)//2 < #(<= v). No sorting."""
    nz = [int(v) for v in np.asarray(vals).ravel() if v != 0]
    if not nz:
        return -1
    k = (len(nz) - 1) // 2
    for v in set(nz):
        lt = sum(1 for u in nz if u < v)
        le = sum(1 for u in nz if u <= v)
        if lt <= k < le:
            return v
    raise AssertionError("no median")


@pytest.mark.parametrize("seed", range(20))
def test_median_by_counting(ref, seed):
    rng = np.random.default_rng(300 + seed)
    h, w = rng.integers(1, 9, size=2)
    levels = [3, 50, 65536][seed % 3]
    z = rng.integers(0, levels, size=(h, w)).astype(np.uint16)
    if seed % 5 == 0:
        z[rng.random((h, w)) < 0.7] = 0
    assert ref.median(z) == _median_by_counting(z)


def test_median_special_cases(ref):
    assert ref.median(np.zeros((4, 5), np.uint16)) == -1
    z = np.zeros((4, 5), np.uint16)
    z[2, 3] = 777
    assert ref.median(z) == 777
    z[0, 0] = 100  # two values: lower median is the smaller one
    assert ref.median(z) == 100
    assert ref.median(np.full((3, 3), 65535, np.uint16)) == 65535
