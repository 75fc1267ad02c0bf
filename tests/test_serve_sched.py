"""CPU tests of the serving scheduler and loop with a stand-in backend: FIFO
admission under an HBM byte budget, slot reuse, no request lost or reordered,
continuous batching (arrivals join the next batch while one is in flight)."""
import numpy as np
import pytest

from paper_1504_01883_amd import serve


class FakeBackend:
    """Completes a batch after `latency_polls` polls; records what it saw."""

    def __init__(self, inflight=2, latency_polls=3):
        self.inflight = inflight
        self.latency_polls = latency_polls
        self.running = []
        self.launched = []
        self.uploaded = []

    def upload_many(self, reqs):
        self.uploaded.extend(r.rid for r in reqs)

    def can_launch(self):
        return len(self.running) < self.inflight

    def launch(self, batch):
        self.launched.append([r.rid for r in batch])
        self.running.append([batch, self.latency_polls])

    def poll(self):
        done = []
        for item in self.running:
            item[1] -= 1
        for item in list(self.running):
            if item[1] <= 0:
                for r in item[0]:
                    r.argmax = np.zeros(len(r.boxes), np.int32)
                done.append(item[0])
                self.running.remove(item)
        return done

    def busy(self):
        return bool(self.running)


def _req(i, nboxes=2):
    return serve.Request(rid=i, stream=i % 3, t_arrival=0.0, boxes=np.zeros((nboxes, 4), np.int32))


def test_budget_defers_in_order_and_loses_nothing():
    s = serve.Scheduler(n_slots=8, budget_bytes=3 * serve.FRAME_BYTES, max_batch_frames=2)
    for i in range(7):
        s.submit(_req(i))
    first = s.admit()
    assert [r.rid for r in first] == [0, 1, 2] and s.deferrals == 1
    assert s.admit() == []  # still full
    b = s.next_batch()
    assert [r.rid for r in b] == [0, 1]
    s.complete(b)
    assert [r.rid for r in s.admit()] == [3, 4]
    order = [r.rid for r in first[:3]] + [3, 4]
    while not s.idle():
        batch = s.next_batch()
        s.complete(batch)
        order += [r.rid for r in s.admit()]
    assert order == list(range(7))
    assert s.bytes_in_use == 0 and len(s.free_slots) == 8


def test_slots_are_unique_while_admitted():
    s = serve.Scheduler(n_slots=4, budget_bytes=100 * serve.FRAME_BYTES)
    for i in range(10):
        s.submit(_req(i))
    got = s.admit()
    assert len(got) == 4 and len({r.slot for r in got}) == 4


def test_budget_smaller_than_a_frame_rejected():
    with pytest.raises(ValueError):
        serve.Scheduler(n_slots=4, budget_bytes=serve.FRAME_BYTES - 1)


def test_run_loop_continuous_batching():
    """All arrive at once; with 2 batches in flight of at most 3 frames, the
    later frames are batched while earlier batches run, every request finishes
    exactly once, and batches preserve arrival order."""
    arrivals = [(0.0, i % 4, i) for i in range(20)]
    frames = {(s, i): (None, np.zeros((1 + i % 3, 4), np.int32), None) for (_, s, i) in arrivals}
    be = FakeBackend(inflight=2, latency_polls=2)
    sch = serve.Scheduler(n_slots=6, budget_bytes=6 * serve.FRAME_BYTES, max_batch_frames=3)
    measured, wall, reqs = serve.run(be, sch, arrivals, frames)
    assert sorted(r.rid for r in measured) == list(range(20))
    flat = [rid for b in be.launched for rid in b]
    assert flat == list(range(20))
    assert max(len(b) for b in be.launched) <= 3
    assert all(r.argmax is not None and len(r.argmax) == len(r.boxes) for r in measured)
    summ = serve.summarize(measured, max(wall, 1e-9))
    assert summ["frames"] == 20 and summ["crops"] == sum(1 + i % 3 for i in range(20))


def test_poisson_arrivals_rate_and_order():
    arr = serve.poisson_arrivals(16, 30.0, 10.0, seed=1)
    ts = [a[0] for a in arr]
    assert ts == sorted(ts)
    assert 0.85 * 4800 < len(arr) < 1.15 * 4800
    per = np.bincount([a[1] for a in arr], minlength=16)
    assert (per > 200).all()


def _treq(rid, stream, prev, owner):
    r = serve.Request(rid=rid, stream=stream, t_arrival=0.0,
                      boxes=np.zeros((len(owner), 4), np.int32))
    r.prev = prev
    r._owner = np.asarray(owner, np.int64)
    return r


def test_trackbook_resolves_in_stream_order():
    """Results arrive out of order; ids still follow each stream's frames: a
    box continuing box o of the previous frame inherits o's id, new faces get
    fresh ids in resolution order."""
    book = serve.TrackBook()
    a0 = _treq(0, 0, None, [-1, -1])          # stream 0: two new faces
    b0 = _treq(1, 1, None, [-1])              # stream 1: one new face
    a1 = _treq(2, 0, a0, [1, -1, 0])          # continues a0's 1 and 0, one new
    a2 = _treq(3, 0, a1, [2])                 # continues a1's box 2
    for r in (a0, b0, a1, a2):
        book.add(r)
    for r in (a2, a1):                        # later frames finish first
        r.owner = r._owner
    assert book.resolve() == 0 and a2.track_ids is None
    b0.owner = b0._owner
    assert book.resolve() == 1 and b0.track_ids.tolist() == [0]
    a0.owner = a0._owner
    assert book.resolve() == 3
    assert a0.track_ids.tolist() == [1, 2]
    assert a1.track_ids.tolist() == [2, 3, 1]
    assert a2.track_ids.tolist() == [1]
