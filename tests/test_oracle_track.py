"""Pins for the oracle's nearest-centre tracking (Sec. 2.3, Fig. 4).

A worked scene in the shape of Fig. 4 (person A's box centre c1 in the previous
frame; the detections c2, c3, c4 of the next frame), an independent NumPy
brute force on half-integer centres in float64 (exact), and the edge cases:
streams, gate boundary, ties, conflicts, empty frames.
"""
import numpy as np
import pytest


def test_fig4_scene(ref):
    """c1 = centre of person A's box (100, 100, 50, 50) = (125, 125). In the next
    frame c2 (A moved: box (110, 105, 50, 50), centre (135, 130)), c3 (person B,
    centre (330, 130)), c4 (person C, centre (70, 320)). A follows c2; B and C
    are new faces, owned by no track."""
    prev = [[100, 100, 50, 50]]
    cur = [[110, 105, 50, 50], [300, 100, 60, 60], [50, 300, 40, 40]]
    match, owner = ref.track(prev, [0], cur, [0, 0, 0])
    assert match.tolist() == [0]
    assert owner.tolist() == [0, -1, -1]


def test_three_people_swap_order(ref):
    """Detections come in a different order in the next frame: each track
    still finds its own face."""
    prev = [[10, 10, 40, 40], [200, 50, 60, 60], [400, 300, 80, 80]]
    cur = [[405, 298, 80, 82], [12, 15, 40, 40], [190, 55, 62, 60]]
    match, owner = ref.track(prev, [0, 0, 0], cur, [0, 0, 0])
    assert match.tolist() == [1, 2, 0]
    assert owner.tolist() == [2, 0, 1]


def _brute(prev, ps, cur, cs, gate2):
    pc = np.array([[x + w / 2, y + h / 2] for x, y, w, h in prev], np.float64).reshape(-1, 2)
    cc = np.array([[x + w / 2, y + h / 2] for x, y, w, h in cur], np.float64).reshape(-1, 2)
    match = np.full(len(prev), -1)
    for p in range(len(prev)):
        d = ((cc - pc[p]) ** 2).sum(axis=1)
        ok = (np.asarray(cs) == ps[p]) & ((gate2 <= 0) | (d <= gate2))
        if ok.any():
            d = np.where(ok, d, np.inf)
            match[p] = int(np.argmin(d))  # first minimum: lowest index
    owner = np.full(len(cur), -1)
    for c in range(len(cur)):
        cand = [p for p in range(len(prev)) if match[p] == c]
        if cand:
            ds = [((cc[c] - pc[p]) ** 2).sum() for p in cand]
            owner[c] = cand[int(np.argmin(ds))]
    return match, owner


@pytest.mark.parametrize("seed", range(6))
def test_random_scenes_match_brute_force(ref, seed):
    rng = np.random.default_rng([150401883, 88, seed])
    P, C, S = int(rng.integers(0, 40)), int(rng.integers(0, 40)), int(rng.integers(1, 4))
    # Coarse positions make equal distances (ties) common.
    prev = [[int(rng.integers(0, 20)) * 8, int(rng.integers(0, 15)) * 8,
             int(rng.integers(3, 12)) * 4, int(rng.integers(3, 12)) * 4] for _ in range(P)]
    cur = [[int(rng.integers(0, 20)) * 8, int(rng.integers(0, 15)) * 8,
            int(rng.integers(3, 12)) * 4, int(rng.integers(3, 12)) * 4] for _ in range(C)]
    ps = rng.integers(0, S, size=P)
    cs = rng.integers(0, S, size=C)
    for gate2 in (0, 400, 2500):
        m, o = ref.track(np.array(prev, np.int32).reshape(-1, 4), ps,
                         np.array(cur, np.int32).reshape(-1, 4), cs, gate2)
        bm, bo = _brute(prev, ps, cur, cs, gate2)
        assert m.tolist() == bm.tolist()
        assert o.tolist() == bo.tolist()


def test_streams_are_separate(ref):
    prev = [[0, 0, 10, 10]]
    cur = [[0, 0, 10, 10], [500, 500, 10, 10]]
    m, o = ref.track(prev, [1], cur, [0, 1])
    assert m.tolist() == [1] and o.tolist() == [-1, 0]
    m, o = ref.track(prev, [2], cur, [0, 1])
    assert m.tolist() == [-1] and o.tolist() == [-1, -1]


def test_gate_boundary(ref):
    """Centres 30 px apart horizontally: gate2 = 900 keeps the box, 899 drops it."""
    prev = [[0, 0, 20, 20]]
    cur = [[30, 0, 20, 20]]
    assert ref.track(prev, [0], cur, [0], 900)[0].tolist() == [0]
    assert ref.track(prev, [0], cur, [0], 899)[0].tolist() == [-1]


def test_ties(ref):
    """Two detections equally far: the lower index wins. Two tracks equally far
    from one detection: the lower track owns it."""
    m, _ = ref.track([[50, 50, 10, 10]], [0], [[60, 50, 10, 10], [40, 50, 10, 10]], [0, 0])
    assert m.tolist() == [0]
    m, o = ref.track([[40, 50, 10, 10], [60, 50, 10, 10]], [0, 0], [[50, 50, 10, 10]], [0])
    assert m.tolist() == [0, 0] and o.tolist() == [0]


def test_empty(ref):
    m, o = ref.track(np.zeros((0, 4), np.int32), np.zeros(0), [[1, 1, 5, 5]], [0])
    assert m.tolist() == [] and o.tolist() == [-1]
    m, o = ref.track([[1, 1, 5, 5]], [0], np.zeros((0, 4), np.int32), np.zeros(0))
    assert m.tolist() == [-1] and o.tolist() == []
