"""Thin ctypes binding of liblbpf.so (C ABI in include/lbpf.h).

Argument marshalling only: torch CUDA tensors are passed as raw device
pointers together with ``torch.cuda.current_stream()``; every step of the
computation runs in the library's HIP kernels. There is no fallback: if the
library is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Sequence

import numpy as np
import torch

_LIB_PATH = Path(__file__).resolve().parent / "liblbpf.so"

LBPF_OK, LBPF_E_INVALID, LBPF_E_BUDGET, LBPF_E_HIP, LBPF_E_UNSUPPORTED = 0, -1, -2, -3, -4
FP32, BF16, FP16, FP8_E4M3, F16X3 = 0, 1, 2, 3, 4
MAP_U59, MAP_FULL256 = 0, 1
MOD_BOTH, MOD_GREY, MOD_DEPTH = 0, 1, 2
MAX_SIDE = 1024
MAX_BOXES_PER_CALL = 65536

_PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3,
               "f16x3": F16X3}

EXPORTS = [
    "lbpf_version", "lbpf_create", "lbpf_destroy", "lbpf_feature_dim", "lbpf_features",
    "lbpf_batch_create", "lbpf_batch_destroy", "lbpf_batch_size", "lbpf_features_batch",
    "lbpf_weights_create", "lbpf_weights_destroy", "lbpf_weights_count", "lbpf_score",
    "lbpf_debug_codes", "lbpf_status_string", "lbpf_last_error", "lbpf_features_plain",
    "lbpf_score_plain", "lbpf_batch_set_launch", "lbpf_batch_get_launch", "lbpf_tune_batch",
    "lbpf_graph_create", "lbpf_graph_launch", "lbpf_graph_destroy", "lbpf_warp_crop_bytes",
    "lbpf_features_warped", "lbpf_train_workspace_bytes", "lbpf_train_ovr",
    "lbpf_train_gram_workspace_bytes", "lbpf_train_ovr_gram", "lbpf_track",
    "lbpf_score_noalloc", "lbpf_pipeline_create", "lbpf_pipeline_launch",
    "lbpf_pipeline_max_boxes", "lbpf_pipeline_destroy", "lbpf_server_create",
    "lbpf_server_clock", "lbpf_server_submit", "lbpf_server_poll", "lbpf_server_get_stats",
    "lbpf_server_destroy",
]


class LbpfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)}: {detail}")
        self.status = status


class Image(ctypes.Structure):
    _fields_ = [("grey", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("grey_pitch", ctypes.c_int32), ("depth_pitch", ctypes.c_int32)]


class Box(ctypes.Structure):
    _fields_ = [("image", ctypes.c_int32), ("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("ux", "uy", "vx", "vy", "tx", "ty")]


class WarpBox(ctypes.Structure):
    _fields_ = [("image", ctypes.c_int32), ("w", ctypes.c_int32), ("h", ctypes.c_int32),
                ("grey", Frame), ("depth", Frame)]


ONE = 1 << 16  # 1.0 in the frames' 16.16 fixed point


def box_frame(x: int, y: int) -> tuple:
    """The identity frame of a box whose top-left pixel is (x, y)."""
    return (ONE, 0, 0, ONE, x * ONE, y * ONE)


def resize_frame(x: int, y: int, w: int, h: int, out_w: int, out_h: int) -> tuple:
    """Nearest-sample resize of box (x, y, w, h) to out_w x out_h, sampling at
    the centre of each output pixel: step w/out_w (16.16, rounded down) and
    half a step of offset."""
    ux = (w * ONE) // out_w
    vy = (h * ONE) // out_h
    return (ux, 0, 0, vy, x * ONE + ux // 2, y * ONE + vy // 2)


class LaunchCfg(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("row_prefetch", ctypes.c_int32), ("sorted", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServerCfg(ctypes.Structure):
    _fields_ = [("frame_w", ctypes.c_int32), ("frame_h", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("budget_bytes", ctypes.c_int64),
                ("max_batch_frames", ctypes.c_int32), ("max_boxes_per_frame", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("copy_streams", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("frames", ctypes.c_int64),
                ("boxes", ctypes.c_int64), ("deferrals", ctypes.c_int64),
                ("loop_iterations", ctypes.c_int64), ("busy_seconds", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# lbpf_request and lbpf_result as numpy record types (C layout, natural
# alignment), so that thousands of requests are marshalled as one array.
REQUEST_DTYPE = np.dtype([("id", np.int64), ("t_arrival", np.float64), ("grey", np.uint64),
                          ("depth", np.uint64), ("boxes", np.uint64), ("n_boxes", np.int32),
                          ("pad", np.int32)])
RESULT_DTYPE = np.dtype([("id", np.int64), ("t_arrival", np.float64), ("t_done", np.float64),
                         ("n_boxes", np.int32), ("argmax_offset", np.int32)])


class FeatureCfg(ctypes.Structure):
    _fields_ = [("grid_x", ctypes.c_int32), ("grid_y", ctypes.c_int32),
                ("mapping", ctypes.c_int32), ("depth_window_mm", ctypes.c_int32),
                ("modality", ctypes.c_int32)]


_lib = None


def load():
    """Load liblbpf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1504_01883_amd.build`")
    lib = ctypes.CDLL(str(_LIB_PATH))
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "lbpf_version": (ctypes.c_char_p, []),
        "lbpf_create": (st, [vp, vp, sz]),
        "lbpf_destroy": (None, [vp]),
        "lbpf_feature_dim": (i32, [vp]),
        "lbpf_features": (st, [vp, vp, i32, vp, i32, vp, vp, vp]),
        "lbpf_batch_create": (st, [vp, vp, i32, vp, i32, vp]),
        "lbpf_batch_destroy": (None, [vp]),
        "lbpf_batch_size": (i32, [vp]),
        "lbpf_features_batch": (st, [vp, vp, vp, vp, vp]),
        "lbpf_weights_create": (st, [vp, vp, vp, i32, st, vp, vp]),
        "lbpf_weights_destroy": (None, [vp]),
        "lbpf_weights_count": (i32, [vp]),
        "lbpf_score": (st, [vp, vp, i32, vp, vp, vp, vp]),
        "lbpf_debug_codes": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "lbpf_features_plain": (st, [vp, vp, i32, vp, i32, vp, vp, vp]),
        "lbpf_score_plain": (st, [vp, vp, i32, vp, vp, vp, vp]),
        "lbpf_batch_set_launch": (st, [vp, vp]),
        "lbpf_batch_get_launch": (st, [vp, vp]),
        "lbpf_tune_batch": (st, [vp, vp, vp, i32, vp, vp, vp]),
        "lbpf_graph_create": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "lbpf_graph_launch": (st, [vp, vp]),
        "lbpf_graph_destroy": (None, [vp]),
        "lbpf_warp_crop_bytes": (sz, [i32, i32]),
        "lbpf_features_warped": (st, [vp, vp, i32, vp, i32, vp, sz, vp, vp, vp]),
        "lbpf_train_workspace_bytes": (sz, [i32]),
        "lbpf_train_ovr": (st, [vp, vp, vp, i32, i32, ctypes.c_double, ctypes.c_double, i32,
                                ctypes.c_uint64, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp]),
        "lbpf_train_gram_workspace_bytes": (sz, [i32, i32]),
        "lbpf_train_ovr_gram": (st, [vp, vp, vp, i32, i32, ctypes.c_double, ctypes.c_double, i32,
                                     ctypes.c_uint64, vp, i32, vp, vp, vp, vp, sz, vp]),
        "lbpf_track": (st, [vp, vp, vp, i32, vp, vp, i32, ctypes.c_int64, vp, vp, vp]),
        "lbpf_score_noalloc": (st, [vp, i32, vp, vp, i32, i32, vp, vp, vp]),
        "lbpf_pipeline_create": (st, [vp, vp, i32, vp, vp, vp, vp, vp]),
        "lbpf_pipeline_launch": (st, [vp, vp, i32, vp, i32, vp]),
        "lbpf_pipeline_max_boxes": (i32, [vp]),
        "lbpf_pipeline_destroy": (None, [vp]),
        "lbpf_server_create": (st, [vp, vp, vp, vp]),
        "lbpf_server_clock": (ctypes.c_double, [vp]),
        "lbpf_server_submit": (st, [vp, vp, i32]),
        "lbpf_server_poll": (st, [vp, vp, i32, vp, i32, vp]),
        "lbpf_server_get_stats": (st, [vp, vp]),
        "lbpf_server_destroy": (None, [vp]),
        "lbpf_status_string": (ctypes.c_char_p, [st]),
        "lbpf_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return load().lbpf_status_string(status).decode()


def version() -> str:
    return load().lbpf_version().decode()


def _check(status: int):
    if status != LBPF_OK:
        raise LbpfError(status, load().lbpf_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA (HIP) tensor")
    return t.data_ptr()


def _plane(t: torch.Tensor, elem_size: int):
    if t.dim() != 2 or t.element_size() != elem_size or t.stride(1) != 1:
        raise ValueError(f"expected a row-major 2-D plane of {elem_size}-byte elements")
    return t.stride(0)


def make_images(planes: Sequence[tuple]):
    """ctypes array of lbpf_image from [(grey u8 [H,W] | None, depth u16 [H,W])] CUDA tensors."""
    arr = (Image * max(1, len(planes)))()
    for i, (g, z) in enumerate(planes):
        zp = _plane(z, 2)
        gp = _plane(g, 1) if g is not None else 0
        arr[i] = Image(_dptr(g) if g is not None else None, _dptr(z), z.shape[1], z.shape[0],
                       gp, zp)
    return arr


def make_boxes(boxes) -> ctypes.Array:
    b = np.ascontiguousarray(np.asarray(boxes, np.int32).reshape(-1, 5))
    arr = (Box * max(1, len(b)))()
    ctypes.memmove(arr, b.ctypes.data, b.nbytes)
    return arr, len(b)


class Batch:
    """A validated, device-resident box table (lbpf_batch)."""

    def __init__(self, ctx: "Context", planes, boxes):
        self._ctx = ctx
        self._planes = list(planes)  # keep the tensors alive
        imgs = make_images(self._planes)
        bx, n = make_boxes(boxes)
        h = ctypes.c_void_p()
        _check(load().lbpf_batch_create(ctx._h, imgs, len(self._planes), bx, n, ctypes.byref(h)))
        self._h = h
        self.n = n

    def set_launch(self, persistent=0, wg_per_cu=4, row_prefetch=4, sorted=1):
        cfg = LaunchCfg(persistent, wg_per_cu, row_prefetch, sorted)
        _check(load().lbpf_batch_set_launch(self._h, ctypes.byref(cfg)))

    def get_launch(self) -> dict:
        cfg = LaunchCfg()
        _check(load().lbpf_batch_get_launch(self._h, ctypes.byref(cfg)))
        return cfg.as_dict()

    def close(self):
        if self._h:
            load().lbpf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Weights:
    """Enrolled identities (lbpf_weights)."""

    def __init__(self, ctx: "Context", W: torch.Tensor, b: torch.Tensor, precision="fp32"):
        W = W.to(torch.float32).contiguous()
        b = b.to(torch.float32).contiguous()
        if W.dim() != 2 or W.shape[1] != ctx.dim or b.shape != (W.shape[0],):
            raise ValueError(f"W must be [K, {ctx.dim}] and b [K]")
        self._ctx = ctx
        self.K = W.shape[0]
        self.precision = precision
        h = ctypes.c_void_p()
        _check(load().lbpf_weights_create(ctx._h, _dptr(W), _dptr(b), self.K,
                                          _PRECISIONS[precision], ctypes.byref(h), _stream()))
        self._h = h

    def close(self):
        if self._h:
            load().lbpf_weights_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured, instantiated HIP graph of features (+ scores/argmax)."""

    def __init__(self, ctx: "Context", batch: Batch, weights, hist, scores=None, argmax=None):
        self._keep = (ctx, batch, weights, hist, scores, argmax)
        h = ctypes.c_void_p()
        _check(load().lbpf_graph_create(ctx._h, batch._h, weights._h if weights else None,
                                        _dptr(hist), _dptr(scores), _dptr(argmax),
                                        ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(load().lbpf_graph_launch(self._h, _stream()))

    def close(self):
        if self._h:
            load().lbpf_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """A captured serving step (lbpf_pipeline): features + scores + argmax of
    batches of up to max_boxes boxes, one graph replay per batch. Outputs live
    in tensors the pipeline holds: hist [max, D], scores [max, K], argmax
    [max] on the device and argmax_host [max] in pinned host memory."""

    def __init__(self, ctx: "Context", weights: Weights, max_boxes: int, device="cuda"):
        self._keep = (ctx, weights)
        self.max_boxes = max_boxes
        self.hist = torch.empty((max_boxes, ctx.dim), dtype=torch.float32, device=device)
        self.scores = torch.empty((max_boxes, weights.K), dtype=torch.float32, device=device)
        self.argmax = torch.empty((max_boxes,), dtype=torch.int32, device=device)
        self.argmax_host = torch.empty((max_boxes,), dtype=torch.int32).pin_memory()
        h = ctypes.c_void_p()
        _check(load().lbpf_pipeline_create(ctx._h, weights._h, max_boxes, _dptr(self.hist),
                                           _dptr(self.scores), _dptr(self.argmax),
                                           self.argmax_host.data_ptr(), ctypes.byref(h)))
        self._h = h

    def launch(self, images: "ImageTable", boxes):
        """Queue one batch on the current stream. boxes: [n, 5] (image, x, y,
        w, h) host rows indexing `images`."""
        bx, n = make_boxes(boxes)
        _check(load().lbpf_pipeline_launch(self._h, images.arr, images.n, bx, n, _stream()))
        return n

    def close(self):
        if self._h:
            load().lbpf_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The native serving loop (lbpf_server_*): a library thread admits,
    uploads and batches frames; submit() queues requests, poll() collects
    the finished ones. Host frame planes must be pinned CPU tensors and stay
    alive until their results have been polled (the server keeps references
    to the tensors of submitted requests until then)."""

    def __init__(self, ctx: "Context", weights: "Weights", frame_w: int, frame_h: int,
                 n_slots: int, budget_bytes: int, max_batch_frames: int,
                 max_boxes_per_frame: int = 8, inflight: int = 2, copy_streams: int = 2):
        self._ctx, self._weights = ctx, weights  # must outlive the server
        cfg = ServerCfg(frame_w, frame_h, n_slots, budget_bytes, max_batch_frames,
                        max_boxes_per_frame, inflight, copy_streams)
        h = ctypes.c_void_p()
        _check(load().lbpf_server_create(ctx._h, weights._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.frame_w, self.frame_h = frame_w, frame_h
        self.max_boxes_per_frame = max_boxes_per_frame
        self._keep: dict[int, tuple] = {}  # id -> (grey, depth) of requests in flight

    def clock(self) -> float:
        return float(load().lbpf_server_clock(self._h))

    def submit(self, ids, t_arrival, frames, boxes):
        """Queue requests: ids [n] int64, t_arrival [n] seconds on the server
        clock (non-decreasing), frames: n (grey u8 [H, W], depth int16/u16
        [H, W]) pinned CPU tensors, boxes: n arrays [k, 4] (x, y, w, h)."""
        n = len(ids)
        req = np.zeros(n, REQUEST_DTYPE)
        counts = np.array([len(b) for b in boxes], np.int64)
        flat = (np.ascontiguousarray(np.concatenate([np.asarray(b, np.int32).reshape(-1, 4)
                                                     for b in boxes]))
                if n else np.zeros((0, 4), np.int32))
        offs = np.concatenate([[0], np.cumsum(counts)[:-1]]) if n else counts
        gp, zp = req["grey"], req["depth"]
        seen: dict[int, tuple] = {}  # frames repeat: check each tensor pair once
        for i, f in enumerate(frames):
            ptrs = seen.get(id(f))
            if ptrs is None:
                g, z = f
                if g.is_cuda or z.is_cuda or not (g.is_pinned() and z.is_pinned()):
                    raise ValueError("server frames must be pinned CPU tensors")
                if (tuple(g.shape) != (self.frame_h, self.frame_w) or g.shape != z.shape or
                        g.element_size() != 1 or z.element_size() != 2 or
                        not (g.is_contiguous() and z.is_contiguous())):
                    raise ValueError("frame planes must be contiguous u8 / 16-bit "
                                     "[frame_h, frame_w]")
                ptrs = seen[id(f)] = (g.data_ptr(), z.data_ptr())
            gp[i], zp[i] = ptrs
        req["id"] = np.asarray(ids, np.int64)
        req["t_arrival"] = np.asarray(t_arrival, np.float64)
        req["n_boxes"] = counts
        req["boxes"] = flat.ctypes.data + 16 * offs
        _check(load().lbpf_server_submit(self._h, req.ctypes.data, n))
        for i, f in zip(req["id"].tolist(), frames):
            self._keep[i] = f

    def poll(self, max_results: int = 4096):
        """Finished requests (oldest first) as a RESULT_DTYPE array and the
        identities: result i's boxes are argmax[argmax_offset : + n_boxes]."""
        res = np.zeros(max_results, RESULT_DTYPE)
        amax = np.zeros(max_results * self.max_boxes_per_frame, np.int32)
        n = ctypes.c_int32()
        st = load().lbpf_server_poll(self._h, res.ctypes.data, max_results, amax.ctypes.data,
                                     len(amax), ctypes.byref(n))
        res = res[:n.value]
        for i in res["id"].tolist():
            self._keep.pop(i, None)
        _check(st)
        return res, amax

    def stats(self) -> dict:
        out = ServerStats()
        _check(load().lbpf_server_get_stats(self._h, ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if self._h:
            load().lbpf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ImageTable:
    """A reusable lbpf_image array for a list of (grey, depth) device planes
    (keeps the tensors alive)."""

    def __init__(self, planes):
        self.planes = list(planes)
        self.arr = make_images(self.planes)
        self.n = len(self.planes)
        self.device = self.planes[0][1].device if self.planes else torch.device("cuda")


class WarpBoxTable:
    """A reusable lbpf_warp_box array: [(image, w, h, grey_frame, depth_frame)],
    marshalled once for calls that repeat the same boxes."""

    def __init__(self, boxes):
        self.n = len(boxes)
        rows = np.zeros((max(1, self.n), 15), np.int32)
        for i, (im, w, h, gf, zf) in enumerate(boxes):
            rows[i, 0:3] = (im, w, h)
            rows[i, 3:9] = gf
            rows[i, 9:15] = zf
        self.arr = (WarpBox * max(1, self.n))()
        ctypes.memmove(self.arr, rows.ctypes.data, rows.nbytes)
        self.workspace_bytes = sum(int(load().lbpf_warp_crop_bytes(int(w), int(h)))
                                   for (_, w, h, _, _) in boxes)


class Context:
    """An lbpf_ctx on the current device."""

    def __init__(self, grid=(8, 8), mapping=MAP_U59, window=150, modality=MOD_BOTH,
                 budget_bytes=0):
        cfg = FeatureCfg(grid[0], grid[1], mapping, window, modality)
        h = ctypes.c_void_p()
        _check(load().lbpf_create(ctypes.byref(h), ctypes.byref(cfg), budget_bytes))
        self._h = h
        self.dim = int(load().lbpf_feature_dim(h))

    def close(self):
        if getattr(self, "_h", None):
            load().lbpf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def features(self, planes, boxes, with_counts=False, out=None, counts_out=None):
        """Features of host-described boxes over device planes -> (hist, counts|None)."""
        imgs = make_images(planes)
        bx, n = make_boxes(boxes)
        dev = planes[0][1].device if planes else torch.device("cuda")
        hist = out if out is not None else torch.empty((n, self.dim), dtype=torch.float32,
                                                       device=dev)
        cnt = counts_out
        if with_counts and cnt is None:
            cnt = torch.empty((n, self.dim), dtype=torch.int32, device=dev)
        _check(load().lbpf_features(self._h, imgs, len(planes), bx, n, _dptr(hist),
                                    _dptr(cnt), _stream()))
        return hist, cnt

    def features_warped(self, planes, boxes, with_counts=False, out=None, workspace=None):
        """Features of warped crops. planes: [(grey, depth)] device tensors or a
        prepared ImageTable; boxes: [(image, w, h, grey_frame, depth_frame)] with
        frames as 6-tuples (see box_frame / resize_frame), or a prepared
        WarpBoxTable. workspace: a uint8 CUDA tensor (256-byte aligned);
        default: one sized for every crop."""
        imgs = planes if isinstance(planes, ImageTable) else ImageTable(planes)
        tab = boxes if isinstance(boxes, WarpBoxTable) else WarpBoxTable(boxes)
        n = tab.n
        dev = imgs.device
        if workspace is None:
            workspace = torch.empty(max(tab.workspace_bytes, 256), dtype=torch.uint8, device=dev)
        hist = out if out is not None else torch.empty((n, self.dim), dtype=torch.float32,
                                                       device=dev)
        cnt = torch.empty((n, self.dim), dtype=torch.int32, device=dev) if with_counts else None
        _check(load().lbpf_features_warped(self._h, imgs.arr, imgs.n, tab.arr, n,
                                           _dptr(workspace), workspace.numel(), _dptr(hist),
                                           _dptr(cnt), _stream()))
        return hist, cnt

    def train(self, X: torch.Tensor, labels: torch.Tensor, K: int, C=1.0, eps=1e-6,
              max_epochs=200, seed=150401883, alpha=None, warm=False, want_f64=False,
              solver="gram"):
        """One-vs-rest SVM training on the device -> dict with W, b (FP32) and
        epochs [K]. solver="gram" (default): the FP32 Gram-matrix solver
        (lbpf_train_ovr_gram), alpha FP32 [K, N]; solver="f64": the FP64
        solver (lbpf_train_ovr), alpha FP64 [K, N], W64 / b64 with want_f64.
        alpha is updated in place when given (warm=True starts from it)."""
        if X.dim() != 2 or X.dtype != torch.float32 or not X.is_contiguous():
            raise ValueError("X must be a contiguous FP32 [N, D] tensor")
        if X.shape[1] != self.dim:
            raise ValueError(f"X has {X.shape[1]} columns, the context's feature dim is {self.dim}")
        if solver not in ("gram", "f64"):
            raise ValueError("solver must be 'gram' or 'f64'")
        N = X.shape[0]
        lab = labels.to(device=X.device, dtype=torch.int32).contiguous()
        dev = X.device
        W = torch.empty((K, self.dim), dtype=torch.float32, device=dev)
        b = torch.empty((K,), dtype=torch.float32, device=dev)
        if solver == "gram":
            if want_f64:
                raise ValueError("want_f64 needs solver='f64'")
            if alpha is not None and (alpha.dtype != torch.float32 or tuple(alpha.shape) != (K, N)
                                      or not alpha.is_contiguous()):
                raise ValueError("alpha must be a contiguous FP32 [K, N] tensor")
            ep = torch.empty((K,), dtype=torch.int32, device=dev)
            nbytes = int(load().lbpf_train_gram_workspace_bytes(N, K))
            ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device=dev)
            _check(load().lbpf_train_ovr_gram(self._h, _dptr(X), _dptr(lab), N, K, float(C),
                                              float(eps), int(max_epochs), int(seed),
                                              _dptr(alpha), int(bool(warm)), _dptr(W), _dptr(b),
                                              _dptr(ep), _dptr(ws), ws.numel(), _stream()))
            return {"W": W, "b": b, "epochs": ep, "workspace": ws}
        W64 = torch.empty((K, self.dim), dtype=torch.float64, device=dev) if want_f64 else None
        b64 = torch.empty((K,), dtype=torch.float64, device=dev) if want_f64 else None
        ep = torch.empty((K,), dtype=torch.int32, device=dev)
        if alpha is not None and (alpha.dtype != torch.float64 or tuple(alpha.shape) != (K, N)
                                  or not alpha.is_contiguous()):
            raise ValueError("alpha must be a contiguous FP64 [K, N] tensor")
        nbytes = int(load().lbpf_train_workspace_bytes(N))
        ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=dev)
        _check(load().lbpf_train_ovr(self._h, _dptr(X), _dptr(lab), N, K, float(C), float(eps),
                                     int(max_epochs), int(seed), _dptr(alpha), int(bool(warm)),
                                     _dptr(W), _dptr(b), _dptr(W64), _dptr(b64), _dptr(ep),
                                     _dptr(ws), ws.numel(), _stream()))
        out = {"W": W, "b": b, "epochs": ep, "workspace": ws}
        if want_f64:
            out["W64"], out["b64"] = W64, b64
        return out

    def track(self, prev_boxes, prev_stream, cur_boxes, cur_stream, gate2=0, device="cuda"):
        """Nearest-centre tracking: host box arrays ([n, 4] (x, y, w, h), streams
        [n]) -> (match [P], owner [C]) int32 device tensors."""
        pb = np.ascontiguousarray(np.asarray(prev_boxes, np.int32).reshape(-1, 4))
        cb = np.ascontiguousarray(np.asarray(cur_boxes, np.int32).reshape(-1, 4))
        ps = np.ascontiguousarray(np.asarray(prev_stream, np.int32).reshape(-1))
        cs = np.ascontiguousarray(np.asarray(cur_stream, np.int32).reshape(-1))
        if ps.shape[0] != pb.shape[0] or cs.shape[0] != cb.shape[0]:
            raise ValueError("one stream id per box")
        match = torch.empty(pb.shape[0], dtype=torch.int32, device=device)
        owner = torch.empty(cb.shape[0], dtype=torch.int32, device=device)
        _check(load().lbpf_track(self._h, pb.ctypes.data, ps.ctypes.data, pb.shape[0],
                                 cb.ctypes.data, cs.ctypes.data, cb.shape[0], int(gate2),
                                 _dptr(match) if match.numel() else None,
                                 _dptr(owner) if owner.numel() else None, _stream()))
        return match, owner

    def features_plain(self, planes, boxes, with_counts=False, out=None):
        """The plain unbatched comparator path (same results, per-crop launches)."""
        imgs = make_images(planes)
        bx, n = make_boxes(boxes)
        dev = planes[0][1].device if planes else torch.device("cuda")
        hist = out if out is not None else torch.empty((n, self.dim), dtype=torch.float32,
                                                       device=dev)
        cnt = torch.empty((n, self.dim), dtype=torch.int32, device=dev) if with_counts else None
        _check(load().lbpf_features_plain(self._h, imgs, len(planes), bx, n, _dptr(hist),
                                          _dptr(cnt), _stream()))
        return hist, cnt

    def score_plain(self, hist: torch.Tensor, weights: "Weights", want_scores=True,
                    want_argmax=True, scores_out=None, argmax_out=None):
        hist = hist.contiguous()
        N = hist.shape[0]
        S = scores_out if scores_out is not None else (
            torch.empty((N, weights.K), dtype=torch.float32, device=hist.device)
            if want_scores else None)
        A = argmax_out if argmax_out is not None else (
            torch.empty((N,), dtype=torch.int32, device=hist.device) if want_argmax else None)
        _check(load().lbpf_score_plain(self._h, _dptr(hist), N, weights._h, _dptr(S), _dptr(A),
                                       _stream()))
        return S, A

    def batch(self, planes, boxes) -> Batch:
        return Batch(self, planes, boxes)

    def features_batch(self, batch: Batch, out: torch.Tensor, counts_out: torch.Tensor | None = None):
        if out.shape != (batch.n, self.dim) or out.dtype != torch.float32:
            raise ValueError("out must be float32 [n, D]")
        _check(load().lbpf_features_batch(self._h, batch._h, _dptr(out), _dptr(counts_out),
                                          _stream()))
        return out

    def tune(self, batch: Batch, hist: torch.Tensor, reps: int = 5):
        """Time every launch shape on `batch`, keep the fastest; -> (cfg dict, us)."""
        best = LaunchCfg()
        us = ctypes.c_float()
        _check(load().lbpf_tune_batch(self._h, batch._h, _dptr(hist), reps, ctypes.byref(best),
                                      ctypes.byref(us), _stream()))
        return best.as_dict(), float(us.value)

    def graph(self, batch: Batch, hist, weights=None, scores=None, argmax=None) -> Graph:
        return Graph(self, batch, weights, hist, scores, argmax)

    def pipeline(self, weights: Weights, max_boxes: int) -> Pipeline:
        return Pipeline(self, weights, max_boxes)

    def server(self, weights: Weights, frame_w: int, frame_h: int, n_slots: int,
               budget_bytes: int, max_batch_frames: int, max_boxes_per_frame: int = 8,
               inflight: int = 2, copy_streams: int = 2) -> Server:
        return Server(self, weights, frame_w, frame_h, n_slots, budget_bytes, max_batch_frames,
                      max_boxes_per_frame, inflight, copy_streams)

    def weights(self, W: torch.Tensor, b: torch.Tensor, precision="fp32") -> Weights:
        return Weights(self, W, b, precision)

    def score(self, hist: torch.Tensor, weights: Weights, want_scores=True, want_argmax=True,
              scores_out=None, argmax_out=None):
        if hist.dim() != 2 or hist.shape[1] != self.dim or hist.dtype != torch.float32:
            raise ValueError("hist must be float32 [N, D]")
        hist = hist.contiguous()
        N = hist.shape[0]
        S = scores_out
        if want_scores and S is None:
            S = torch.empty((N, weights.K), dtype=torch.float32, device=hist.device)
        A = argmax_out
        if want_argmax and A is None:
            A = torch.empty((N,), dtype=torch.int32, device=hist.device)
        _check(load().lbpf_score(self._h, _dptr(hist), N, weights._h, _dptr(S), _dptr(A),
                                 _stream()))
        return S, A

    def debug_codes(self, grey: torch.Tensor, depth: torch.Tensor, box):
        """Per-pixel (grey codes, depth codes, mask) of one box, as u8 [h, w] tensors."""
        imgs = make_images([(grey, depth)])
        x, y, w, h = (int(v) for v in box)
        bx = Box(0, x, y, w, h)
        outs = [torch.zeros((h, w), dtype=torch.uint8, device=depth.device) for _ in range(3)]
        _check(load().lbpf_debug_codes(self._h, imgs, ctypes.byref(bx), *(_dptr(o) for o in outs),
                                       _stream()))
        return tuple(outs)


NOALLOC_SCRATCH_BYTES = 16 << 20


def score_noalloc(hist: torch.Tensor, W: torch.Tensor, b: torch.Tensor, want_scores=True,
                  want_argmax=True, scores_out=None, argmax_out=None):
    """FP32 scoring through lbpf_score_noalloc (no context, no allocation in
    the library): hist [N, D], W [K, D], b [K] FP32 CUDA tensors ->
    (scores [N, K] | None, argmax [N] | None)."""
    for t in (hist, W, b):
        if t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("hist, W and b must be contiguous float32 CUDA tensors")
    N, D = hist.shape
    K = W.shape[0]
    if W.shape[1] != D or b.shape != (K,):
        raise ValueError("W must be [K, D] and b [K]")
    S = scores_out
    if want_scores and S is None:
        S = torch.empty((N, K), dtype=torch.float32, device=hist.device)
    A = argmax_out
    if want_argmax and A is None:
        A = torch.empty((N,), dtype=torch.int32, device=hist.device)
    _check(load().lbpf_score_noalloc(_dptr(hist), N, _dptr(W), _dptr(b), K, D, _dptr(S),
                                     _dptr(A), _stream()))
    return S, A


def to_device_planes(grey: np.ndarray | None, depth: np.ndarray, device="cuda"):
    """Copy host planes to the device as (grey u8, depth u16) tensors."""
    z = torch.from_numpy(np.ascontiguousarray(depth, np.uint16)).to(device)
    g = None
    if grey is not None:
        g = torch.from_numpy(np.ascontiguousarray(grey, np.uint8)).to(device)
    return g, z
