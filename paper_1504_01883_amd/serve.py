"""Continuous-batching server for synthetic RGB-D face streams.

Requests are frames (640x480 grey u8 + depth u16) with 1-8 face boxes each,
arriving from many streams (the paper's per-frame detect -> map -> features ->
classify loop, Sec. 3, Fig. 10, run for many cameras at once). The server

* admits a request into a free device frame slot only while the bytes of all
  admitted frames stay within an HBM budget (first come, first served: a
  request that does not fit waits, and nothing behind it overtakes it);
* copies admitted frames host -> device on a copy stream;
* launches a batch (features of every box of every admitted frame, then
  scores + argmax against the enrolled identities) whenever a batch buffer is
  free, so frames that arrive while earlier batches run on the GPU join the
  next batch (continuous batching), with up to `inflight` batches on
  different compute streams at once; each in-flight set owns a captured
  pipeline (lbpf_pipeline: box table upload, features, scores, argmax and
  the identities' copy to pinned memory as one HIP graph replay, the batch
  size read from device memory), so a batch costs the host one call;
* retires batches when their completion event fires, frees their slots and
  records each frame's latency (completion seen by the host minus arrival);
* optionally tracks faces across each stream's frames (Sec. 2.3: nearest box
  centre): the association runs on the device inside the batch, and track
  ids are handed out on the host in each stream's arrival order (TrackBook).

The Scheduler is pure host logic (tested on the CPU with a stand-in backend);
GpuBackend drives liblbpf through the binding. The "plain" backend processes
each frame alone with the plain unbatched FP32 kernels, as the comparator.
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import sys
import time

import numpy as np

FRAME_BYTES = 640 * 480 * 3  # grey u8 + depth u16


@dataclasses.dataclass
class Request:
    rid: int
    stream: int
    t_arrival: float
    boxes: np.ndarray          # [n, 4] (x, y, w, h)
    frame: object = None       # backend-specific host frame handle
    idents: np.ndarray | None = None
    slot: int = -1
    t_done: float = 0.0
    argmax: np.ndarray | None = None
    scores: np.ndarray | None = None
    features: np.ndarray | None = None  # [n, D] FP32 (backends asked to keep them)
    prev: "Request | None" = None     # previous frame of the same stream (tracking)
    owner: np.ndarray | None = None   # per box: index of the previous box it continues, or -1
    track_ids: np.ndarray | None = None
    prev_off: int = 0                 # where the previous frame's boxes sit in the device call


class TrackBook:
    """Track ids from the device's association. Each frame's `owner` array
    (per current box: the index of the previous frame's box whose track it
    continues, or -1) may arrive in any order across batches; a frame gets its
    ids once its own owner and its predecessor's ids are known, so every
    stream resolves in arrival order. New faces get fresh ids."""

    def __init__(self):
        self.next_id = 0
        self.pending: dict[int, collections.deque] = {}

    def add(self, req: Request):
        self.pending.setdefault(req.stream, collections.deque()).append(req)

    def resolve(self) -> int:
        n = 0
        for q in self.pending.values():
            while q and q[0].owner is not None and (q[0].prev is None or
                                                    q[0].prev.track_ids is not None):
                req = q.popleft()
                ids = np.empty(len(req.owner), np.int64)
                for c, o in enumerate(req.owner):
                    if o >= 0:
                        ids[c] = req.prev.track_ids[o]
                    else:
                        ids[c] = self.next_id
                        self.next_id += 1
                req.track_ids = ids
                req.prev = None  # only the latest frame of a stream is needed
                n += 1
        return n


class Scheduler:
    """FIFO admission into frame slots under a byte budget; batch formation."""

    def __init__(self, n_slots: int, budget_bytes: int, frame_bytes: int = FRAME_BYTES,
                 max_batch_frames: int = 64):
        if frame_bytes > budget_bytes:
            raise ValueError("the budget cannot hold a single frame")
        self.free_slots = collections.deque(range(n_slots))
        self.budget = budget_bytes
        self.frame_bytes = frame_bytes
        self.max_batch_frames = max_batch_frames
        self.bytes_in_use = 0
        self.waiting: collections.deque[Request] = collections.deque()
        self.admitted: collections.deque[Request] = collections.deque()
        self.deferrals = 0

    def submit(self, req: Request):
        self.waiting.append(req)

    def admit(self) -> list[Request]:
        """Admit waiting requests in arrival order while a slot and budget allow."""
        out = []
        while self.waiting:
            if not self.free_slots or self.bytes_in_use + self.frame_bytes > self.budget:
                self.deferrals += 1
                break
            req = self.waiting.popleft()
            req.slot = self.free_slots.popleft()
            self.bytes_in_use += self.frame_bytes
            self.admitted.append(req)
            out.append(req)
        return out

    def next_batch(self) -> list[Request]:
        batch = []
        while self.admitted and len(batch) < self.max_batch_frames:
            batch.append(self.admitted.popleft())
        return batch

    def complete(self, batch: list[Request]):
        for req in batch:
            self.free_slots.append(req.slot)
            self.bytes_in_use -= self.frame_bytes
            req.slot = -1

    def idle(self) -> bool:
        return not self.waiting and not self.admitted


class GpuBackend:
    """Batched features + scores through liblbpf (fused path)."""

    def __init__(self, ctx, weights, n_slots: int, max_batch_frames: int, inflight: int = 2,
                 keep_scores: bool = False, plain: bool = False, track: bool = False,
                 keep_features: bool = False, keep_batches: int | None = None,
                 graph: bool = True):
        import torch
        self.torch = torch
        self.ctx, self.weights, self.plain = ctx, weights, plain
        self.track = track
        self.book = TrackBook()
        self.last_req: dict[int, Request] = {}
        self.K = weights.K
        self.keep_scores = keep_scores
        self.keep_features = keep_features
        # Scores / features are copied back for the first keep_batches
        # launches only (None: every launch).
        self.keep_left = keep_batches
        dev = torch.device("cuda")
        self.grey = torch.empty((n_slots, 480, 640), dtype=torch.uint8, device=dev)
        self.depth = torch.empty((n_slots, 480, 640), dtype=torch.int16, device=dev)
        self.copy_stream = torch.cuda.Stream()
        # Per slot: (sequence number, event) of the copy group that filled it.
        # Groups run in order on the one copy stream, so a batch waits on its
        # newest group's event only.
        self.copy_seq = 0
        self.copied = [(0, None)] * n_slots
        max_boxes = 8 * max_batch_frames
        # The fused path replays one captured step per batch (lbpf_pipeline):
        # the frame slots are described once, a batch is its box rows.
        self.graph = graph and not plain
        if self.graph:
            from . import lbpf
            self.table = lbpf.ImageTable([(self.grey[i], self.depth[i]) for i in range(n_slots)])
        self.sets = []
        for _ in range(inflight):
            pipe = ctx.pipeline(weights, max_boxes) if self.graph else None
            self.sets.append({
                "pipe": pipe,
                "stream": torch.cuda.Stream(),
                # With a pipeline its own buffers hold the batch's results.
                "hist": (pipe.hist if pipe else
                         torch.empty((max_boxes, ctx.dim), dtype=torch.float32, device=dev)),
                "S": (pipe.scores if pipe else
                      torch.empty((max_boxes, self.K), dtype=torch.float32, device=dev)),
                "A": pipe.argmax if pipe else torch.empty((max_boxes,), dtype=torch.int32, device=dev),
                "A_host": (pipe.argmax_host if pipe else
                           torch.empty((max_boxes,), dtype=torch.int32).pin_memory()),
                "O_host": torch.empty((max_boxes,), dtype=torch.int32).pin_memory(),
                "S_host": (torch.empty((max_boxes, self.K), dtype=torch.float32).pin_memory()
                           if keep_scores else None),
                "F_host": (torch.empty((max_boxes, ctx.dim), dtype=torch.float32).pin_memory()
                           if keep_features else None),
                "done": torch.cuda.Event(), "batch": None, "nb": 0, "kept": False})
        self.free_sets = collections.deque(range(inflight))

    def host_frame(self, grey: np.ndarray, depth: np.ndarray):
        t = self.torch
        g = t.from_numpy(grey).pin_memory()
        z = t.from_numpy(depth.view(np.int16)).pin_memory()
        return (g, z)

    def upload(self, req: Request):
        self.upload_many([req])

    def upload_many(self, reqs: list[Request]):
        """Copy the admitted frames to their slots on the copy stream: one
        call for all of them, and one event that every slot of the group
        waits on."""
        if not reqs:
            return
        t = self.torch
        dst = [self.grey[r.slot] for r in reqs] + [self.depth[r.slot] for r in reqs]
        src = [r.frame[0] for r in reqs] + [r.frame[1] for r in reqs]
        with t.cuda.stream(self.copy_stream):
            t._foreach_copy_(dst, src, non_blocking=True)
            ev = t.cuda.Event()
            ev.record(self.copy_stream)
        self.copy_seq += 1
        for r in reqs:
            self.copied[r.slot] = (self.copy_seq, ev)

    def can_launch(self) -> bool:
        return bool(self.free_sets)

    def launch(self, batch: list[Request]):
        si = self.free_sets.popleft()
        st = self.sets[si]
        s = st["stream"]
        seq, ev = max((self.copied[req.slot] for req in batch), key=lambda c: c[0])
        if ev is not None:
            s.wait_event(ev)
        counts = [len(req.boxes) for req in batch]
        nb = sum(counts)
        if not self.graph:
            planes, boxes = [], []
            for i, req in enumerate(batch):
                planes.append((self.grey[req.slot], self.depth[req.slot]))
                for (x, y, w, h) in req.boxes:
                    boxes.append([i, int(x), int(y), int(w), int(h)])
        with self.torch.cuda.stream(s):
            if self.graph:
                # Box table rows [slot, x, y, w, h], built with a few array calls.
                rows = np.empty((nb, 5), np.int32)
                if nb:
                    rows[:, 0] = np.repeat([req.slot for req in batch], counts)
                    rows[:, 1:] = np.concatenate([np.asarray(req.boxes).reshape(-1, 4)
                                                  for req in batch])
                st["pipe"].launch(self.table, rows)
            elif self.plain:
                for i, req in enumerate(batch):
                    lo = sum(len(r.boxes) for r in batch[:i])
                    n = len(req.boxes)
                    fb = [[0, int(x), int(y), int(w), int(h)] for (x, y, w, h) in req.boxes]
                    self.ctx.features_plain([planes[i]], fb, out=st["hist"][lo:lo + n])
                    self.ctx.score_plain(st["hist"][lo:lo + n], self.weights,
                                         scores_out=st["S"][lo:lo + n],
                                         argmax_out=st["A"][lo:lo + n])
            else:
                self.ctx.features(planes, boxes, out=st["hist"][:nb])
                self.ctx.score(st["hist"][:nb], self.weights, scores_out=st["S"][:nb],
                               argmax_out=st["A"][:nb])
            if self.track:
                self._associate(batch, st, nb)
            if not self.graph:  # the pipeline's replay copies the identities itself
                st["A_host"][:nb].copy_(st["A"][:nb], non_blocking=True)
            kept = self.keep_left is None or self.keep_left > 0
            if self.keep_left is not None and self.keep_left > 0:
                self.keep_left -= 1
            if self.keep_scores and kept:
                st["S_host"][:nb].copy_(st["S"][:nb], non_blocking=True)
            if self.keep_features and kept:
                st["F_host"][:nb].copy_(st["hist"][:nb], non_blocking=True)
            st["done"].record(s)
        st["batch"], st["nb"], st["kept"] = batch, nb, kept

    def _associate(self, batch: list[Request], st, nb: int):
        """Nearest-centre association of every frame in the batch with the
        previous frame of its stream (launched earlier, possibly in this
        batch), as one device call; pair i is frame i of the batch."""
        prev_boxes, prev_pair, cur_pair = [], [], []
        off = 0
        for i, req in enumerate(batch):
            req.prev = self.last_req.get(req.stream)
            self.last_req[req.stream] = req
            self.book.add(req)
            req.prev_off = off
            if req.prev is not None:
                prev_boxes.append(np.asarray(req.prev.boxes, np.int32).reshape(-1, 4))
                prev_pair.append(np.full(len(req.prev.boxes), i, np.int32))
                off += len(req.prev.boxes)
            cur_pair.append(np.full(len(req.boxes), i, np.int32))
        pb = np.concatenate(prev_boxes) if prev_boxes else np.zeros((0, 4), np.int32)
        pp = np.concatenate(prev_pair) if prev_pair else np.zeros(0, np.int32)
        cb = np.concatenate([np.asarray(r.boxes, np.int32).reshape(-1, 4) for r in batch])
        _, owner = self.ctx.track(pb, pp, cb, np.concatenate(cur_pair))
        st["O_host"][:nb].copy_(owner, non_blocking=True)

    def poll(self) -> list[list[Request]]:
        done = []
        for si, st in enumerate(self.sets):
            if st["batch"] is not None and st["done"].query():
                t = time.perf_counter()
                A = st["A_host"][:st["nb"]].numpy().copy()
                kept = st["kept"]
                S = st["S_host"][:st["nb"]].numpy().copy() if self.keep_scores and kept else None
                F = (st["F_host"][:st["nb"]].numpy().copy()
                     if self.keep_features and kept else None)
                O = st["O_host"][:st["nb"]].numpy().copy() if self.track else None
                pos = 0
                for req in st["batch"]:
                    n = len(req.boxes)
                    req.argmax = A[pos:pos + n]
                    req.scores = S[pos:pos + n] if S is not None else None
                    req.features = F[pos:pos + n] if F is not None else None
                    if O is not None:  # owners index the call's track list
                        o = O[pos:pos + n]
                        req.owner = np.where(o >= 0, o - req.prev_off, -1)
                    req.t_done = t
                    pos += n
                done.append(st["batch"])
                st["batch"] = None
                self.free_sets.append(si)
        if self.track and done:
            self.book.resolve()
        return done

    def busy(self) -> bool:
        return any(st["batch"] is not None for st in self.sets)


def poisson_arrivals(n_streams: int, fps: float, duration: float, seed: int):
    """(t, stream, frame index) sorted by time: each stream a Poisson process."""
    rng = np.random.default_rng([seed, 17_000_001])
    out = []
    for s in range(n_streams):
        t, i = float(rng.exponential(1.0 / fps)), 0
        while t < duration:
            out.append((t, s, i))
            i += 1
            t += float(rng.exponential(1.0 / fps))
    out.sort()
    return out


def run(backend, sched: Scheduler, arrivals, frames, warmup: float = 0.0, stats=None,
        freeze_gc: bool = False):
    """Serve `arrivals` in real time. frames[(stream, index)] -> (frame handle,
    boxes, idents). Returns the completed requests (arrival >= warmup) and the
    wall time of the measured window. With a `stats` dict the loop records
    its own cost there: iterations, the longest iteration, the share of the
    wall time spent outside sleeps, and Python's garbage-collection pauses.
    freeze_gc moves the objects alive at the start out of the collector's
    reach and turns automatic collection off for the run (the loop's own
    garbage is then freed by reference counting alone)."""
    reqs, done = [], []
    gcs = {"n": 0, "total": 0.0, "max": 0.0, "t": 0.0}

    def on_gc(phase, info):
        if phase == "start":
            gcs["t"] = time.perf_counter()
        else:
            d = time.perf_counter() - gcs["t"]
            gcs["n"] += 1
            gcs["total"] += d
            gcs["max"] = max(gcs["max"], d)

    if freeze_gc:
        gc.collect()
        gc.freeze()
        gc.disable()
    if stats is not None:
        gc.callbacks.append(on_gc)
    iters, slept, longest = 0, 0.0, 0.0
    t0 = time.perf_counter()
    ai = 0
    try:
        while ai < len(arrivals) or not sched.idle() or backend.busy():
            t_it = time.perf_counter()
            now = t_it - t0
            while ai < len(arrivals) and arrivals[ai][0] <= now:
                t, s, i = arrivals[ai]
                fr, boxes, idents = frames[(s, i)]
                req = Request(rid=ai, stream=s, t_arrival=t0 + t, boxes=boxes, frame=fr,
                              idents=idents)
                reqs.append(req)
                sched.submit(req)
                ai += 1
            admitted = sched.admit()
            if admitted:
                backend.upload_many(admitted)
            while backend.can_launch():
                batch = sched.next_batch()
                if not batch:
                    break
                backend.launch(batch)
            for batch in backend.poll():
                sched.complete(batch)
                done.extend(batch)
            t_work = time.perf_counter()
            longest = max(longest, t_work - t_it)
            iters += 1
            if ai < len(arrivals) and not backend.busy() and sched.idle():
                nxt = arrivals[ai][0] - (time.perf_counter() - t0)
                if nxt > 0.0005:
                    time.sleep(min(nxt, 0.002))
            else:
                time.sleep(0.0001)
            slept += time.perf_counter() - t_work
    finally:
        if freeze_gc:
            gc.enable()
            gc.unfreeze()
        if stats is not None:
            gc.callbacks.remove(on_gc)
    end = time.perf_counter()
    if stats is not None:
        stats.update({"loop_iterations": iters, "longest_iteration_ms": longest * 1e3,
                      "host_busy_fraction": 1.0 - slept / max(end - t0, 1e-9),
                      "gc_pauses": gcs["n"], "gc_total_ms": gcs["total"] * 1e3,
                      "gc_longest_ms": gcs["max"] * 1e3})
    measured = [r for r in done if r.t_arrival - t0 >= warmup]
    return measured, end - (t0 + warmup), reqs


def summarize(measured, wall: float) -> dict:
    lat = np.array([r.t_done - r.t_arrival for r in measured]) * 1e3
    crops = int(sum(len(r.boxes) for r in measured))
    if len(lat) == 0:
        return {"frames": 0}
    return {"frames": len(measured), "crops": crops, "crops_per_s": crops / wall,
            "frames_per_s": len(measured) / wall,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max())}


def quick_latency(ctx, seconds: float = 30.0, warmup: float = 2.0, plain_seconds: float = 10.0,
                  pool: int = 24, keep_results: bool = False) -> dict:
    """The serving workload for the headline line: 16 streams x 30 fps Poisson
    arrivals, BF16 scores against 1024 identities, `warmup` + `seconds`
    measured, through the Python loop with pipeline replays; then the plain
    unbatched FP32 path on the first `plain_seconds` of the same arrivals;
    then the same arrivals through the native loop. p50/p99 frame latency
    and crops/s of each. With
    keep_results the fused run's features and scores are returned under
    "_fused_results" (and the FP32 weights under "_weights") for an accuracy
    statement against the FP64 oracle."""
    import torch

    from . import synth
    n_streams, fps, K = 16, 30.0, 1024
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_SERVING)
    Wd, bd = torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()
    w_bf16 = ctx.weights(Wd, bd, precision="bf16")
    w_fp32 = ctx.weights(Wd, bd, precision="fp32")
    arr = poisson_arrivals(n_streams, fps, warmup + seconds, synth.SEED)
    raw = {}
    for (_, s, i) in arr:
        if (s, i % pool) not in raw:
            raw[(s, i % pool)] = synth.make_frame(s, i % pool, K)
    out = {"workload": f"serving: {n_streams} streams x {fps:.0f} fps Poisson, 640x480 frames, "
                       f"1-8 faces (48-256 px, {pool} distinct frames per stream), {K} "
                       f"identities; fused BF16: {warmup:.0f} s warm-up + {seconds:.0f} s; "
                       f"plain FP32: the first {plain_seconds:.0f} s of the same arrivals"}
    plain_arr = [a for a in arr if a[0] < warmup + plain_seconds]
    for name, wts, plain, arrivals in (("fused_bf16", w_bf16, False, arr),
                                       ("plain_unbatched_fp32", w_fp32, True, plain_arr)):
        keep = keep_results and not plain
        # Results are copied back only for the first 256 batches, which fall
        # in the warm-up: the measured window carries no extra copies.
        be = GpuBackend(ctx, wts, 128, 64, inflight=2, plain=plain, keep_scores=keep,
                        keep_features=keep, keep_batches=256 if keep else None)
        frames = {}
        for (_, s, i) in arrivals:
            g, z, bx, ids = raw[(s, i % pool)]
            frames[(s, i)] = (be.host_frame(g, z), bx, ids)
        sch = Scheduler(128, 128 * FRAME_BYTES, max_batch_frames=64)
        measured, wall, reqs = run(be, sch, arrivals, frames, warmup, freeze_gc=True)
        summ = summarize(measured, wall)
        out[name] = {k: summ[k] for k in ("frames", "crops", "crops_per_s", "p50_ms", "p99_ms")
                     if k in summ}
        if keep:
            out["_fused_results"] = [r for r in reqs if r.features is not None]
            out["_weights"] = (W, b)
        if not plain:
            fused_ids = {r.rid: r.argmax for r in reqs if r.argmax is not None}
    # The same arrivals through the native loop (lbpf_server): every host step
    # in the library's thread. Its identities are compared with the Python
    # loop's, frame by frame (the same kernels: they must be equal).
    pinned, boxes_of = {}, {}
    for key, (g, z, bx, _) in raw.items():
        pinned[key] = (torch.from_numpy(g).pin_memory(),
                       torch.from_numpy(z.view(np.int16)).pin_memory())
        boxes_of[key] = np.asarray(bx, np.int32)
    nat = native_run(ctx, w_bf16, [(t, s, (s, i % pool)) for (t, s, i) in arr], pinned,
                     boxes_of, warmup, keep_identities=True)
    ids = nat.pop("_identities")
    same = [np.array_equal(a, fused_ids[rid]) for rid, a in ids.items() if rid in fused_ids]
    nat["identities_equal_to_python_loop"] = float(np.mean(same)) if same else None
    out["fused_bf16_native"] = nat
    w_bf16.close()
    w_fp32.close()
    return out


def native_run(ctx, weights, arrivals, frames, boxes_of, warmup: float, n_slots: int = 128,
               budget: int = 128 * FRAME_BYTES, max_batch_frames: int = 64, inflight: int = 2,
               copy_streams: int = 2, timeout: float = 120.0,
               keep_identities: bool = False) -> dict:
    """Serve `arrivals` [(t, stream, key)] with the native loop (lbpf_server):
    every request is submitted up front with its arrival time, and the
    library thread releases, admits, uploads and batches them. frames[key]:
    pinned (grey, depth) tensors, boxes_of[key]: [n, 4]. Latency = the
    server's completion time minus the arrival time, over arrivals at or
    after `warmup`."""
    srv = ctx.server(weights, 640, 480, n_slots, budget, max_batch_frames, 8, inflight,
                     copy_streams)
    n = len(arrivals)
    t0 = srv.clock() + 0.05
    t_arr = t0 + np.array([a[0] for a in arrivals], np.float64)
    keys = [a[2] for a in arrivals]
    n_box = np.array([len(boxes_of[k]) for k in keys], np.int64)
    srv.submit(np.arange(n), t_arr, [frames[k] for k in keys], [boxes_of[k] for k in keys])
    t_done = np.full(n, np.nan)
    identities = {}
    got = 0
    deadline = time.monotonic() + (t_arr[-1] - srv.clock() if n else 0.0) + timeout
    while got < n:
        res, amax = srv.poll(65536)
        if len(res):
            t_done[res["id"]] = res["t_done"]
            got += len(res)
            if keep_identities:
                for r in res:
                    o = int(r["argmax_offset"])
                    identities[int(r["id"])] = amax[o:o + int(r["n_boxes"])].copy()
        elif time.monotonic() > deadline:
            break
        else:
            time.sleep(0.005)
    st = srv.stats()
    srv.close()
    m = (t_arr - t0 >= warmup) & np.isfinite(t_done)
    lat = (t_done[m] - t_arr[m]) * 1e3
    wall = (t_done[m].max() - (t0 + warmup)) if m.any() else float("nan")
    crops = int(n_box[m].sum())
    out = {"frames": int(m.sum()), "crops": crops, "crops_per_s": crops / wall,
           "frames_per_s": float(m.sum()) / wall,
           "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
           "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
           "max_ms": float(lat.max()) if len(lat) else None,
           "unfinished": int(n - got),
           "server": {"batches": st["batches"], "frames_per_batch": st["frames"] / max(st["batches"], 1),
                      "deferring_iterations": st["deferrals"],
                      "thread_busy_fraction": st["busy_seconds"] / max(st["seconds"], 1e-9)}}
    if keep_identities:
        out["_identities"] = identities
    return out


def bench(args) -> dict:
    """Serving workload: 16 streams x 30 fps Poisson arrivals, 640x480 frames with
    1-8 faces, BF16 scoring against 1024 identities; 2 s warm-up + 30 s
    measured. The same arrivals are replayed through the plain unbatched FP32
    path for comparison, and the offered rate is raised until p99 exceeds one
    frame interval (33 ms) to find the saturation throughput. The serving loop
    runs with Python's garbage collection frozen unless a sweep says
    otherwise."""
    import torch

    from . import lbpf, synth
    n_streams, fps, K = 16, 30.0, 1024
    warm = float(getattr(args, "serve_warmup", 2.0))
    secs = float(getattr(args, "serve_seconds", 30.0))
    torch.cuda.set_device(0)
    ctx = lbpf.Context()
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_SERVING)
    Wd, bd = torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()
    w_bf16 = ctx.weights(Wd, bd, precision="bf16")
    w_fp32 = ctx.weights(Wd, bd, precision="fp32")
    pool = 24  # distinct frames per stream, cycled
    n_slots, budget = 128, 128 * FRAME_BYTES

    def frames_for(backend, arrivals):
        cache = {}
        handles = {}
        for (_, s, i) in arrivals:
            key = (s, i % pool)
            if key not in cache:
                g, z, bx, ids = synth.make_frame(s, i % pool, K)
                cache[key] = (backend.host_frame(g, z), bx, ids)
            handles[(s, i)] = cache[key]
        return handles

    def one(rate_mult, plain=False, duration=secs, warmup=warm, track=False, graph=True,
            freeze_gc=True):
        arr = poisson_arrivals(n_streams, fps * rate_mult, warmup + duration, synth.SEED)
        be = GpuBackend(ctx, w_fp32 if plain else w_bf16, n_slots, 64, inflight=2, plain=plain,
                        track=track, graph=graph)
        frames = frames_for(be, arr)
        sch = Scheduler(n_slots, budget, max_batch_frames=64)
        st = {}
        measured, wall, _ = run(be, sch, arr, frames, warmup, stats=st, freeze_gc=freeze_gc)
        out = summarize(measured, wall)
        out["deferrals"] = sch.deferrals
        out["host_loop"] = st
        print(f"[serve] x{rate_mult:g} {'plain' if plain else ('graph' if graph else 'eager')}"
              f"{' +track' if track else ''}{'' if freeze_gc else ' gc on'}: "
              f"{out.get('crops_per_s', 0):.0f} crops/s, p50 {out.get('p50_ms', 0):.2f} ms, "
              f"p99 {out.get('p99_ms', 0):.2f} ms; loop busy {st['host_busy_fraction']:.2f}, "
              f"longest iteration {st['longest_iteration_ms']:.1f} ms, gc {st['gc_pauses']} "
              f"pauses, longest {st['gc_longest_ms']:.1f} ms", file=sys.stderr, flush=True)
        return out

    fused = one(1.0)
    tracked = one(1.0, duration=min(secs, 10.0), track=True)
    plain = one(1.0, plain=True, duration=min(secs, 10.0))
    # Saturation: raise the offered rate until p99 passes one frame interval,
    # with the captured pipeline and with eager per-batch calls (garbage
    # collection frozen in both), and with the pipeline under Python's
    # automatic collection.
    sweeps = {}
    for name, graph, frz in (("graph", True, True), ("eager", False, True),
                             ("graph_gc_on", True, False)):
        sweep = []
        for mult in (4.0, 16.0, 32.0, 48.0, 64.0, 128.0):
            r = one(mult, duration=4.0, warmup=0.5, graph=graph, freeze_gc=frz)
            r["rate_mult"] = mult
            sweep.append(r)
            if r.get("p99_ms", 1e9) > 1000.0 / fps:
                break
        sweeps[name] = sweep
    # The native loop: the same arrivals, every host step in the library's
    # thread. Frames are the same pinned pool; boxes as generated.
    pinned, boxes_of = {}, {}
    for s_ in range(n_streams):
        for i in range(pool):
            g, z, bx, _ = synth.make_frame(s_, i, K)
            pinned[(s_, i)] = (torch.from_numpy(g).pin_memory(),
                               torch.from_numpy(z.view(np.int16)).pin_memory())
            boxes_of[(s_, i)] = np.asarray(bx, np.int32)

    def native(rate_mult, duration, warmup):
        arr = [(t, s_, (s_, i % pool)) for (t, s_, i) in
               poisson_arrivals(n_streams, fps * rate_mult, warmup + duration, synth.SEED)]
        r = native_run(ctx, w_bf16, arr, pinned, boxes_of, warmup, n_slots=n_slots,
                       budget=budget)
        r["rate_mult"] = rate_mult
        print(f"[serve] x{rate_mult:g} native: {r['crops_per_s']:.0f} crops/s, p50 "
              f"{r['p50_ms']:.2f} ms, p99 {r['p99_ms']:.2f} ms; server thread busy "
              f"{r['server']['thread_busy_fraction']:.2f}, {r['server']['frames_per_batch']:.1f} "
              f"frames per batch, unfinished {r['unfinished']}", file=sys.stderr, flush=True)
        return r

    fused_native = native(1.0, secs, warm)
    sweeps["native"] = []
    for mult in (4.0, 16.0, 32.0, 48.0, 64.0, 80.0, 96.0, 128.0, 192.0, 256.0):
        r = native(mult, 4.0, 0.5)
        sweeps["native"].append(r)
        if r.get("p99_ms") is None or r["p99_ms"] > 1000.0 / fps or r["unfinished"]:
            break
    sat_n = max((r for r in sweeps["native"] if r.get("p99_ms") is not None and
                 r["p99_ms"] <= 1000.0 / fps and not r["unfinished"]),
                key=lambda r: r["crops_per_s"], default=None)
    sweep = sweeps["graph"]
    sat = max((r for r in sweep if r.get("p99_ms", 1e9) <= 1000.0 / fps),
              key=lambda r: r["crops_per_s"], default=None)
    sat_e = max((r for r in sweeps["eager"] if r.get("p99_ms", 1e9) <= 1000.0 / fps),
                key=lambda r: r["crops_per_s"], default=None)
    ctx.close()
    return {"metric": "face crops/s and p50/p99 frame latency, serving",
            "value": fused.get("crops_per_s"), "unit": "crops/s", "n_gpus": 1,
            "higher_is_better": True, "data": "synthetic", "dtype": "bf16 scoring",
            "config": {"workload": f"serving: {n_streams} streams x {fps:.0f} fps Poisson, "
                                   "640x480 grey+depth frames, 1-8 faces (48-256 px), "
                                   f"BF16 scoring vs {K} identities, {warm:.0f} s warm-up + "
                                   f"{secs:.0f} s measured, {n_slots} frame slots, budget "
                                   f"{budget} B", "streams": n_streams, "fps": fps,
                       "identities": K},
            "fused": fused, "fused_native": fused_native, "fused_with_tracking": tracked,
            "plain_unbatched_fp32": plain, "saturation_sweep": sweep,
            "saturation_sweep_graph_gc_on": sweeps["graph_gc_on"],
            "saturation_sweep_eager": sweeps["eager"],
            "saturation_sweep_native": sweeps["native"],
            "max_crops_per_s_with_p99_under_frame_interval_native":
                sat_n["crops_per_s"] if sat_n else None,
            "max_crops_per_s_with_p99_under_frame_interval":
                sat["crops_per_s"] if sat else None,
            "max_crops_per_s_with_p99_under_frame_interval_eager":
                sat_e["crops_per_s"] if sat_e else None}
