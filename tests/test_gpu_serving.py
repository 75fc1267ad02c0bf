"""GPU tests of the serving loop: every frame's result is the same alone and in
the mix (features and scores row-independent: bitwise), results match the
oracle, and a tight HBM budget defers admission without losing frames."""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, serve, synth
from tests.gpu_util import require_gpu
from tests.lp_ref import lp_tolerance, quantised_reference

pytestmark = pytest.mark.gpu

K = 64


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    ctx = lbpf.Context()
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_SERVING)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="bf16")
    frames = [synth.make_frame(s, i, K) for s in range(4) for i in range(6)]
    yield ctx, wts, W, b, frames
    ctx.close()


def _serve(ctx, wts, frames, arrivals, n_slots=32, budget_frames=32, batch=16, inflight=2,
           track=False, keep_features=False):
    be = serve.GpuBackend(ctx, wts, n_slots, batch, inflight=inflight, keep_scores=True,
                          track=track, keep_features=keep_features)
    handles = {}
    for (t, s, i) in arrivals:
        g, z, bx, ids = frames[i]
        handles[(s, i)] = (be.host_frame(g, z), bx, ids)
    sch = serve.Scheduler(n_slots, budget_frames * serve.FRAME_BYTES, max_batch_frames=batch)
    measured, wall, reqs = serve.run(be, sch, arrivals, handles)
    return {r.rid: r for r in measured}, sch


def test_tracking_in_the_serving_loop(setup, ref):
    """Sec. 2.3 inside the loop: every frame's association with the previous
    frame of its stream equals the oracle's, and track ids follow it (a
    continued box keeps its predecessor's id, new faces get unused ids)."""
    ctx, wts, W, b, frames = setup
    # frames[i] is stream i // 6, frame i % 6; interleave the four streams.
    arrivals = [(0.0003 * k, i // 6, i) for k, i in
                enumerate(sorted(range(len(frames)), key=lambda i: (i % 6, i // 6)))]
    res, _ = _serve(ctx, wts, frames, arrivals, batch=5, track=True)
    by_stream = {}
    for k, (_, st, i) in enumerate(arrivals):
        by_stream.setdefault(st, []).append((k, i))
    seen = set()
    for st, seq in by_stream.items():
        prev_ids, prev_boxes = None, None
        for k, i in seq:
            r = res[k]
            boxes = frames[i][2]
            if prev_boxes is None:
                want = np.full(len(boxes), -1)
            else:
                _, want = ref.track(prev_boxes, np.zeros(len(prev_boxes)), boxes,
                                    np.zeros(len(boxes)))
            assert r.owner.tolist() == want.tolist()
            for c, o in enumerate(r.owner):
                if o >= 0:
                    assert r.track_ids[c] == prev_ids[o]
                else:
                    assert r.track_ids[c] not in seen
                    seen.add(int(r.track_ids[c]))
            prev_ids, prev_boxes = r.track_ids, boxes


def test_alone_equals_mix(setup):
    ctx, wts, W, b, frames = setup
    mix_arrivals = [(0.0005 * i, i % 4, i) for i in range(len(frames))]
    mix, _ = _serve(ctx, wts, frames, mix_arrivals)
    assert len(mix) == len(frames)
    for i in range(len(frames)):
        alone, _ = _serve(ctx, wts, frames, [(0.0, 0, i)], batch=1, inflight=1)
        a = alone[0]
        m = mix[i]
        assert np.array_equal(a.argmax, m.argmax)
        assert np.array_equal(a.scores.view(np.uint32), m.scores.view(np.uint32))


def test_serving_matches_oracle(setup, ref):
    """Frames served in one batch: every crop's FP32 features equal the
    oracle's bit for bit, the BF16 scores equal the exact product of the
    BF16-rounded operands within the FP32 accumulation tolerance, and the
    argmax agrees with the FP64 oracle wherever its top-2 margin is clear of
    the row's BF16 error."""
    ctx, wts, W, b, frames = setup
    arrivals = [(0.0, 0, i) for i in range(6)]
    res, _ = _serve(ctx, wts, frames, arrivals, keep_features=True)
    tol = lp_tolerance("bf16", ctx.dim)
    for i in range(6):
        g, z, bx, _ = frames[i]
        boxes = [[0, int(x), int(y), int(w), int(h)] for (x, y, w, h) in bx]
        f, _, _ = ref.features([(g, z)], boxes, n_threads=8)
        got = res[i]
        assert np.array_equal(got.features.view(np.uint32), f.view(np.uint32))
        qref, scale = quantised_reference(f, W, b, "bf16")
        assert (np.abs(got.scores.astype(np.float64) - qref) <= tol * scale + 1e-30).all()
        S64, A64 = ref.score_f64(f, W, b)
        e_row = np.abs(got.scores - S64).max(axis=1)
        top2 = np.sort(S64, axis=1)[:, -2:]
        clear = (top2[:, 1] - top2[:, 0]) > 2 * e_row
        assert np.array_equal(got.argmax[clear], A64[clear])


def test_tight_budget_defers_but_completes(setup):
    ctx, wts, W, b, frames = setup
    arrivals = [(0.0, i % 4, i) for i in range(len(frames))]
    res, sch = _serve(ctx, wts, frames, arrivals, n_slots=8, budget_frames=2, batch=4)
    assert sorted(res) == list(range(len(frames)))
    assert sch.deferrals > 0
    assert sch.bytes_in_use == 0
