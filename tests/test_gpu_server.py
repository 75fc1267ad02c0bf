"""The native serving loop (lbpf_server_*): a library thread releases
requests at their arrival times, admits them into frame slots under an HBM
byte budget (first come, first served), uploads them and runs each batch as
one captured-pipeline replay (Sec. 3's per-frame loop, many cameras at once).

  * every frame's identities equal those of the eager path on the same boxes
    (features bit-exact; the argmax compared wherever the top-2 margin of the
    eager scores is clear of the scores' tolerance), in FP32 and BF16;
  * a frame's identities are the same alone and in a mix of other frames;
  * requests are not served before their arrival time, a budget of fewer
    frames than requests defers admission without losing any, and bad
    requests are refused whole.
"""
import time

import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, score_tolerance
from tests.lp_ref import lp_tolerance, quantised_reference

pytestmark = pytest.mark.gpu

K = 300
FW, FH = synth.FRAME_W, synth.FRAME_H
FRAME_BYTES = 3 * FW * FH


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    ctx = lbpf.Context()
    frames = [synth.make_frame(s, i, K) for s in range(4) for i in range(6)]
    pinned = [(torch.from_numpy(g).pin_memory(), torch.from_numpy(z.view(np.int16)).pin_memory())
              for (g, z, _, _) in frames]
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_SERVING)
    yield ctx, frames, pinned, W, b
    ctx.close()


def collect(srv, n, timeout=60.0):
    """Poll until n results have arrived; returns {id: (result, argmax)}."""
    out = {}
    t_end = time.monotonic() + timeout
    while len(out) < n:
        res, amax = srv.poll()
        for r in res:
            o, k = int(r["argmax_offset"]), int(r["n_boxes"])
            out[int(r["id"])] = (r, amax[o:o + k].copy())
        if time.monotonic() > t_end:
            raise AssertionError(f"only {len(out)} of {n} results after {timeout} s")
        time.sleep(0.001)
    return out


def eager_reference(ctx, wts, W, b, frames, prec):
    """Per frame: (eager argmax, mask of boxes whose top-2 score margin is
    clear of twice the scores' tolerance)."""
    out = []
    for (g, z, bx, _) in frames:
        planes = [lbpf.to_device_planes(g, z)]
        rows = [[0, int(x), int(y), int(w), int(h)] for (x, y, w, h) in bx]
        hist, _ = ctx.features(planes, rows)
        S, A = ctx.score(hist, wts)
        torch.cuda.synchronize()
        X = hist.cpu().numpy()
        S = S.cpu().numpy().astype(np.float64)
        if prec == "fp32":
            tol = score_tolerance(X, W, b).max(axis=1)
        else:
            _, scale = quantised_reference(X, W, b, prec)
            tol = lp_tolerance(prec, ctx.dim) * scale.max(axis=1)
        top2 = np.sort(S, axis=1)[:, -2:]
        out.append((A.cpu().numpy(), (top2[:, 1] - top2[:, 0]) > 2 * tol))
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_server_matches_eager_path(setup, prec):
    """24 frames submitted at once into 4 slots (a 4-frame budget), uploads
    spread over 4 copy streams, batches of up to 3 frames on 2 sets: every
    identity equals the eager path's."""
    ctx, frames, pinned, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    ref = eager_reference(ctx, wts, W, b, frames, prec)
    srv = ctx.server(wts, FW, FH, n_slots=4, budget_bytes=4 * FRAME_BYTES, max_batch_frames=3,
                     max_boxes_per_frame=8, inflight=2, copy_streams=4)
    n = len(frames)
    t = srv.clock()
    srv.submit(np.arange(n), np.full(n, t), pinned, [f[2] for f in frames])
    got = collect(srv, n)
    for i in range(n):
        r, amax = got[i]
        A, clear = ref[i]
        assert r["n_boxes"] == len(frames[i][2])
        assert r["t_done"] >= r["t_arrival"]
        assert np.array_equal(amax[clear], A[clear]), f"{prec}: frame {i} identities differ"
    st = srv.stats()
    assert st["frames"] == n and st["boxes"] == sum(len(f[2]) for f in frames)
    assert st["batches"] >= n // 3
    assert st["deferrals"] > 0  # 24 frames through 4 slots
    srv.close()
    wts.close()


def test_server_alone_equals_mix(setup):
    """A frame served alone and served among 23 others gets the same
    identities bit for bit (one captured step for every batch size, rows
    independent)."""
    ctx, frames, pinned, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="bf16")
    srv = ctx.server(wts, FW, FH, n_slots=8, budget_bytes=8 * FRAME_BYTES, max_batch_frames=8,
                     copy_streams=1)
    n = len(frames)
    alone = {}
    for i in (0, 7, 23):
        srv.submit([1000 + i], [srv.clock()], [pinned[i]], [frames[i][2]])
        alone[i] = collect(srv, 1)[1000 + i][1]
    srv.submit(np.arange(n), np.full(n, srv.clock()), pinned, [f[2] for f in frames])
    mix = collect(srv, n)
    for i, a in alone.items():
        assert np.array_equal(a, mix[i][1])
    srv.close()
    wts.close()


def test_server_releases_at_arrival_time(setup):
    """Requests with future arrival times are served after them, in order."""
    ctx, frames, pinned, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="bf16")
    srv = ctx.server(wts, FW, FH, n_slots=4, budget_bytes=4 * FRAME_BYTES, max_batch_frames=4)
    t0 = srv.clock() + 0.05
    arr = t0 + 0.01 * np.arange(6)
    srv.submit(np.arange(6), arr, pinned[:6], [f[2] for f in frames[:6]])
    got = collect(srv, 6)
    for i in range(6):
        r = got[i][0]
        assert abs(r["t_arrival"] - arr[i]) < 1e-12
        assert r["t_done"] >= arr[i]
    srv.close()
    wts.close()


def test_server_rejects_bad_requests(setup):
    ctx, frames, pinned, W, b = setup
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision="bf16")
    srv = ctx.server(wts, FW, FH, n_slots=2, budget_bytes=2 * FRAME_BYTES, max_batch_frames=2)
    t = srv.clock() + 10.0  # never released during the test
    bad = frames[0][2].copy()
    bad[0, 0] = FW - bad[0, 2] + 1  # one column past the right edge
    with pytest.raises(lbpf.LbpfError) as ei:
        srv.submit([0, 1], [t, t], pinned[:2], [frames[1][2], bad])
    assert ei.value.status == lbpf.LBPF_E_INVALID
    with pytest.raises(lbpf.LbpfError) as ei:
        srv.submit([0, 1], [t, t - 1.0], pinned[:2], [frames[0][2], frames[1][2]])
    assert ei.value.status == lbpf.LBPF_E_INVALID
    with pytest.raises(ValueError):
        g, z = frames[0][0], frames[0][1]
        srv.submit([0], [t], [(torch.from_numpy(g), torch.from_numpy(z.view(np.int16)))],
                   [frames[0][2]])
    with pytest.raises(lbpf.LbpfError) as ei:
        ctx.server(wts, FW, FH, n_slots=2, budget_bytes=FRAME_BYTES - 1, max_batch_frames=2)
    assert ei.value.status == lbpf.LBPF_E_INVALID
    for bad_cfg in ({"copy_streams": 0}, {"copy_streams": 9}, {"inflight": 0}):
        with pytest.raises(lbpf.LbpfError) as ei:
            ctx.server(wts, FW, FH, n_slots=2, budget_bytes=2 * FRAME_BYTES, max_batch_frames=2,
                       **bad_cfg)
        assert ei.value.status == lbpf.LBPF_E_INVALID
    # Accepted requests far in the future: destroying the server drops them.
    srv.submit([5], [t], pinned[:1], [frames[0][2]])
    assert srv.stats()["frames"] == 0
    srv.close()
    wts.close()
