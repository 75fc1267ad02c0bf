// Native serving loop (lbpf_server_*): continuous batching of RGB-D frames
// from many cameras on one library thread. Sec. 3 runs detection, mapping,
// feature extraction and classification once per frame; here every frame's
// face boxes go through the captured serving step (lbpf_pipeline_*), batched
// with whatever other frames are admitted when a batch set is free.
//
// Threads: the caller's thread(s) submit and poll; the server thread owns
// the schedule (release at arrival time, admission by slots and byte
// budget, uploads spread over several copy streams, batch formation,
// completion) and is the only thread that
// issues HIP work on the server's streams. The two sides meet in `pending`
// (submitted requests) and `done` (finished ones), both under `mu`.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <limits>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctx_internal.h"
#include "lbpf_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kMaxBoxesPerFrame = 64;
constexpr int32_t kMaxSlots = 4096;
constexpr int32_t kMaxSide = 4096;
constexpr int32_t kMaxInflight = 8;
constexpr int32_t kMaxCopyStreams = 8;

struct Req {
    int64_t id = 0;
    double t_arrival = 0.0;
    const uint8_t *grey = nullptr;
    const uint16_t *depth = nullptr;
    std::vector<int32_t> boxes;  // [n][4] x, y, w, h
    int32_t y0 = 0, y1 = 0;      // rows the boxes span (only these are uploaded)
    int32_t slot = -1;
    int32_t cs = 0;    // copy stream of its upload
    uint64_t seq = 0;  // upload order
};

struct Done {
    int64_t id;
    double t_arrival, t_done;
    std::vector<int32_t> argmax;
};

// One batch set: a stream, a captured pipeline and its buffers.
struct Set {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    lbpf_pipeline *pipe = nullptr;
    float *hist = nullptr;
    int32_t *argmax = nullptr;
    int32_t *argmax_host = nullptr;  // pinned
    std::vector<Req> batch;
    bool busy = false;
};

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

}  // namespace

struct lbpf_server {
    lbpf_ctx *ctx = nullptr;
    const lbpf_weights *w = nullptr;
    lbpf_server_cfg cfg{};
    int device = 0;
    size_t plane_px = 0, frame_bytes = 0, charged = 0;
    int32_t max_boxes = 0;
    uint8_t *d_grey = nullptr;
    uint16_t *d_depth = nullptr;
    std::vector<lbpf_image> images;  // one per slot
    std::vector<hipStream_t> copy_streams;
    std::vector<hipEvent_t> slot_ev;  // end of the copies into each slot
    std::vector<Set> sets;
    Clock::time_point t0;

    // Shared with the caller's threads, under mu. wake: a submission or the
    // stop request arrived while the server thread may be sleeping on cv.
    std::mutex mu;
    std::condition_variable cv;
    bool wake = false;
    std::deque<Req> pending;
    double last_arrival = -std::numeric_limits<double>::infinity();
    std::deque<Done> done;
    lbpf_status error = LBPF_OK;
    std::string error_msg;

    // Server thread only.
    std::deque<Req> waiting, admitted;
    std::deque<int32_t> free_slots;
    std::deque<int32_t> free_sets;
    int64_t bytes_in_use = 0;
    uint64_t seq = 0;

    std::atomic<int64_t> n_batches{0}, n_frames{0}, n_boxes{0}, n_deferrals{0}, n_iter{0};
    std::atomic<double> busy_s{0.0};
    std::atomic<bool> stop{false};
    std::thread thread;
};

namespace {

// Record the server thread's first error; the thread then stops.
void thread_fail(lbpf_server *S, hipError_t e, const char *what) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error == LBPF_OK) {
        S->error = LBPF_E_HIP;
        S->error_msg = std::string("server thread: ") + what + ": " + hipGetErrorString(e);
    }
}

void thread_fail_status(lbpf_server *S, const char *what) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->error == LBPF_OK) {
        S->error = LBPF_E_HIP;
        S->error_msg = std::string("server thread: ") + what + ": " + lbpf_last_error();
    }
}

// Admit waiting requests in arrival order while a slot and the budget allow,
// and queue their uploads. Returns false on a HIP error.
bool admit(lbpf_server *S, bool &worked) {
    const lbpf_server_cfg &c = S->cfg;
    bool held = false;
    while (!S->waiting.empty()) {
        if (S->free_slots.empty() ||
            S->bytes_in_use + (int64_t)S->frame_bytes > c.budget_bytes) {
            held = true;
            break;
        }
        Req r = std::move(S->waiting.front());
        S->waiting.pop_front();
        r.slot = S->free_slots.front();
        S->free_slots.pop_front();
        S->bytes_in_use += (int64_t)S->frame_bytes;
        r.cs = (int32_t)(S->seq % S->copy_streams.size());
        hipStream_t cs = S->copy_streams[(size_t)r.cs];
        // Only the rows the frame's boxes span: the kernels read nothing
        // else of the slot (their reads past a crop's right edge stay inside
        // the slot's plane and are never used).
        const size_t o = (size_t)r.slot * S->plane_px + (size_t)r.y0 * (size_t)c.frame_w;
        const size_t px = (size_t)(r.y1 - r.y0) * (size_t)c.frame_w;
        const size_t src = (size_t)r.y0 * (size_t)c.frame_w;
        hipError_t e = hipSuccess;
        if (px) {
            e = hipMemcpyAsync(S->d_grey + o, r.grey + src, px, hipMemcpyHostToDevice, cs);
            if (e == hipSuccess)
                e = hipMemcpyAsync(S->d_depth + o, r.depth + src, 2 * px, hipMemcpyHostToDevice,
                                   cs);
        }
        if (e == hipSuccess) e = hipEventRecord(S->slot_ev[(size_t)r.slot], cs);
        if (e != hipSuccess) {
            thread_fail(S, e, "frame upload");
            return false;
        }
        r.seq = ++S->seq;
        S->admitted.push_back(std::move(r));
        worked = true;
    }
    if (held) S->n_deferrals.fetch_add(1, std::memory_order_relaxed);
    return true;
}

// Form batches from the admitted frames while a set is free.
bool launch(lbpf_server *S, std::vector<lbpf_box> &boxes, bool &worked) {
    while (!S->free_sets.empty() && !S->admitted.empty()) {
        const int32_t si = S->free_sets.front();
        S->free_sets.pop_front();
        Set &st = S->sets[(size_t)si];
        st.batch.clear();
        boxes.clear();
        // Per copy stream, the slot of the batch's newest frame uploaded there.
        int32_t last[kMaxCopyStreams];
        uint64_t last_seq[kMaxCopyStreams] = {};
        while (!S->admitted.empty() && (int32_t)st.batch.size() < S->cfg.max_batch_frames) {
            Req r = std::move(S->admitted.front());
            S->admitted.pop_front();
            const size_t nb = r.boxes.size() / 4;
            for (size_t k = 0; k < nb; ++k)
                boxes.push_back(lbpf_box{r.slot, r.boxes[4 * k], r.boxes[4 * k + 1],
                                         r.boxes[4 * k + 2], r.boxes[4 * k + 3]});
            if (r.seq > last_seq[r.cs]) {
                last_seq[r.cs] = r.seq;
                last[r.cs] = r.slot;
            }
            st.batch.push_back(std::move(r));
        }
        // Copies run in order on each copy stream: per stream, the newest
        // frame's event covers the batch's other frames uploaded there.
        for (size_t c = 0; c < S->copy_streams.size(); ++c) {
            if (!last_seq[c]) continue;
            const hipError_t e = hipStreamWaitEvent(st.stream, S->slot_ev[(size_t)last[c]], 0);
            if (e != hipSuccess) {
                thread_fail(S, e, "hipStreamWaitEvent");
                return false;
            }
        }
        hipError_t e;
        if (lbpf_pipeline_launch(st.pipe, S->images.data(), (int32_t)S->images.size(),
                                 boxes.data(), (int32_t)boxes.size(), st.stream) != LBPF_OK) {
            thread_fail_status(S, "pipeline launch");
            return false;
        }
        e = hipEventRecord(st.done, st.stream);
        if (e != hipSuccess) {
            thread_fail(S, e, "hipEventRecord");
            return false;
        }
        st.busy = true;
        worked = true;
    }
    return true;
}

// Retire finished batches: results to `done`, slots back to the free list.
bool retire(lbpf_server *S, bool &worked) {
    for (size_t si = 0; si < S->sets.size(); ++si) {
        Set &st = S->sets[si];
        if (!st.busy) continue;
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            thread_fail(S, q, "hipEventQuery");
            return false;
        }
        const double t = seconds_since(S->t0);
        int64_t nbox = 0;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            size_t pos = 0;
            for (Req &r : st.batch) {
                const size_t n = r.boxes.size() / 4;
                S->done.push_back(Done{r.id, r.t_arrival, t,
                                       std::vector<int32_t>(st.argmax_host + pos,
                                                            st.argmax_host + pos + n)});
                pos += n;
            }
            nbox = (int64_t)pos;
        }
        for (Req &r : st.batch) {
            S->free_slots.push_back(r.slot);
            S->bytes_in_use -= (int64_t)S->frame_bytes;
        }
        S->n_batches.fetch_add(1, std::memory_order_relaxed);
        S->n_frames.fetch_add((int64_t)st.batch.size(), std::memory_order_relaxed);
        S->n_boxes.fetch_add(nbox, std::memory_order_relaxed);
        st.batch.clear();
        st.busy = false;
        S->free_sets.push_back((int32_t)si);
        worked = true;
    }
    return true;
}

void run(lbpf_server *S) {
    hipError_t e = hipSetDevice(S->device);
    if (e != hipSuccess) {
        thread_fail(S, e, "hipSetDevice");
        return;
    }
    std::vector<lbpf_box> boxes;
    boxes.reserve((size_t)S->max_boxes);
    for (;;) {
        const auto it0 = Clock::now();
        const bool stopping = S->stop.load(std::memory_order_acquire);
        double next_arrival = std::numeric_limits<double>::infinity();
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (stopping) {
                S->pending.clear();
            } else {
                const double now = seconds_since(S->t0);
                while (!S->pending.empty() && S->pending.front().t_arrival <= now) {
                    S->waiting.push_back(std::move(S->pending.front()));
                    S->pending.pop_front();
                }
                if (!S->pending.empty()) next_arrival = S->pending.front().t_arrival;
            }
        }
        if (stopping) {  // drop what has not reached a batch
            while (!S->admitted.empty()) {
                S->free_slots.push_back(S->admitted.front().slot);
                S->bytes_in_use -= (int64_t)S->frame_bytes;
                S->admitted.pop_front();
            }
            S->waiting.clear();
        }
        bool worked = false;
        if (!admit(S, worked) || !launch(S, boxes, worked) || !retire(S, worked)) return;
        S->n_iter.fetch_add(1, std::memory_order_relaxed);
        const bool busy = std::any_of(S->sets.begin(), S->sets.end(),
                                      [](const Set &s) { return s.busy; });
        if (stopping && !busy) return;
        if (worked) {
            const double d = std::chrono::duration<double>(Clock::now() - it0).count();
            S->busy_s.store(S->busy_s.load(std::memory_order_relaxed) + d,
                            std::memory_order_relaxed);
        }
        // Batches in flight or a frame about to arrive: poll again at once.
        // Otherwise sleep until shortly before the next arrival (at most
        // 10 ms); a submission or the stop request wakes the thread early.
        const double wait = next_arrival - seconds_since(S->t0);
        if (busy || !S->waiting.empty() || !S->admitted.empty() || wait < 200e-6) {
            std::this_thread::yield();
        } else {
            const double sl = std::min(wait - 100e-6, 10e-3);
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait_for(lk, std::chrono::duration<double>(sl), [S] {
                return S->wake || S->stop.load(std::memory_order_acquire);
            });
            S->wake = false;
        }
    }
}

void release(lbpf_server *S) {
    (void)hipSetDevice(S->device);
    for (Set &st : S->sets) {
        if (st.stream) (void)hipStreamSynchronize(st.stream);
        if (st.pipe) lbpf_pipeline_destroy(st.pipe);
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.stream) (void)hipStreamDestroy(st.stream);
        if (st.hist) (void)hipFree(st.hist);
        if (st.argmax) (void)hipFree(st.argmax);
        if (st.argmax_host) (void)hipHostFree(st.argmax_host);
    }
    for (hipStream_t cs : S->copy_streams) {
        if (!cs) continue;
        (void)hipStreamSynchronize(cs);
        (void)hipStreamDestroy(cs);
    }
    for (hipEvent_t ev : S->slot_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (S->d_grey) (void)hipFree(S->d_grey);
    if (S->d_depth) (void)hipFree(S->d_depth);
    if (S->charged) lbpf::ctx_refund(S->ctx, S->charged);
    delete S;
}

}  // namespace

extern "C" {

lbpf_status lbpf_server_create(lbpf_ctx *ctx, const lbpf_weights *weights,
                               const lbpf_server_cfg *cfg, lbpf_server **out) {
    using lbpf::set_last_error;
    if (!ctx || !weights || !cfg || !out) return set_last_error(LBPF_E_INVALID, "NULL argument");
    *out = nullptr;
    const lbpf_server_cfg c = *cfg;
    if (c.frame_w < 3 || c.frame_h < 3 || c.frame_w > kMaxSide || c.frame_h > kMaxSide)
        return set_last_error(LBPF_E_INVALID, "frame size out of range");
    if (c.n_slots < 1 || c.n_slots > kMaxSlots)
        return set_last_error(LBPF_E_INVALID, "n_slots out of range");
    if (c.max_batch_frames < 1 || c.max_batch_frames > c.n_slots)
        return set_last_error(LBPF_E_INVALID, "max_batch_frames out of range");
    if (c.max_boxes_per_frame < 1 || c.max_boxes_per_frame > kMaxBoxesPerFrame)
        return set_last_error(LBPF_E_INVALID, "max_boxes_per_frame out of range");
    if (c.inflight < 1 || c.inflight > kMaxInflight)
        return set_last_error(LBPF_E_INVALID, "inflight out of range");
    if (c.copy_streams < 1 || c.copy_streams > kMaxCopyStreams)
        return set_last_error(LBPF_E_INVALID, "copy_streams out of range");
    const size_t plane_px = (size_t)c.frame_w * (size_t)c.frame_h;
    if (c.budget_bytes < (int64_t)(3 * plane_px))
        return set_last_error(LBPF_E_INVALID, "budget_bytes cannot hold one frame");
    const int32_t max_boxes = c.max_batch_frames * c.max_boxes_per_frame;
    if (max_boxes > LBPF_MAX_BOXES_PER_CALL)
        return set_last_error(LBPF_E_INVALID, "max_batch_frames * max_boxes_per_frame too large");
    const int32_t D = lbpf_feature_dim(ctx);

    lbpf_server *S = new (std::nothrow) lbpf_server;
    if (!S) return set_last_error(LBPF_E_BUDGET, "out of host memory");
    S->ctx = ctx;
    S->w = weights;
    S->cfg = c;
    S->device = lbpf::ctx_device(ctx);
    S->plane_px = plane_px;
    S->frame_bytes = 3 * plane_px;
    S->max_boxes = max_boxes;
    auto bail = [&](lbpf_status s, const std::string &msg) {
        release(S);
        return set_last_error(s, msg);
    };
    auto hip_bail = [&](hipError_t e, const char *what) {
        release(S);
        return set_last_error(LBPF_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e = hipSetDevice(S->device);
    if (e != hipSuccess) return hip_bail(e, "hipSetDevice");
    const size_t slots_bytes = (size_t)c.n_slots * 3 * plane_px;
    const size_t set_bytes = (size_t)max_boxes * ((size_t)D * 4 + 4);
    const size_t want = slots_bytes + (size_t)c.inflight * set_bytes;
    if (!lbpf::ctx_charge(ctx, want)) return bail(LBPF_E_BUDGET, "server exceeds the HBM budget");
    S->charged = want;
    if ((e = hipMalloc(&S->d_grey, (size_t)c.n_slots * plane_px)) != hipSuccess)
        return hip_bail(e, "hipMalloc");
    if ((e = hipMalloc(&S->d_depth, (size_t)c.n_slots * 2 * plane_px)) != hipSuccess)
        return hip_bail(e, "hipMalloc");
    S->images.resize((size_t)c.n_slots);
    S->slot_ev.assign((size_t)c.n_slots, nullptr);
    for (int32_t i = 0; i < c.n_slots; ++i) {
        S->images[(size_t)i] = lbpf_image{S->d_grey + (size_t)i * plane_px,
                                          S->d_depth + (size_t)i * plane_px, c.frame_w,
                                          c.frame_h, c.frame_w, c.frame_w};
        if ((e = hipEventCreateWithFlags(&S->slot_ev[(size_t)i], hipEventDisableTiming)) !=
            hipSuccess)
            return hip_bail(e, "hipEventCreate");
        S->free_slots.push_back(i);
    }
    S->copy_streams.assign((size_t)c.copy_streams, nullptr);
    for (hipStream_t &cs : S->copy_streams)
        if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
            return hip_bail(e, "hipStreamCreate");
    S->sets.resize((size_t)c.inflight);
    for (int32_t i = 0; i < c.inflight; ++i) {
        Set &st = S->sets[(size_t)i];
        if ((e = hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_bail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming)) != hipSuccess)
            return hip_bail(e, "hipEventCreate");
        if ((e = hipMalloc(&st.hist, (size_t)max_boxes * (size_t)D * 4)) != hipSuccess)
            return hip_bail(e, "hipMalloc");
        if ((e = hipMalloc(&st.argmax, (size_t)max_boxes * 4)) != hipSuccess)
            return hip_bail(e, "hipMalloc");
        if ((e = hipHostMalloc(&st.argmax_host, (size_t)max_boxes * 4, hipHostMallocDefault)) !=
            hipSuccess)
            return hip_bail(e, "hipHostMalloc");
        const lbpf_status ps = lbpf_pipeline_create(ctx, weights, max_boxes, st.hist, nullptr,
                                                    st.argmax, st.argmax_host, &st.pipe);
        if (ps != LBPF_OK) {
            const std::string msg = lbpf_last_error();
            return bail(ps, msg);
        }
        S->free_sets.push_back(i);
    }
    S->t0 = Clock::now();
    try {
        S->thread = std::thread(run, S);
    } catch (...) {
        return bail(LBPF_E_HIP, "could not start the server thread");
    }
    *out = S;
    return LBPF_OK;
}

double lbpf_server_clock(const lbpf_server *S) { return S ? seconds_since(S->t0) : 0.0; }

lbpf_status lbpf_server_submit(lbpf_server *S, const lbpf_request *reqs, int32_t n) {
    using lbpf::set_last_error;
    if (!S) return set_last_error(LBPF_E_INVALID, "server is NULL");
    if (n < 0 || (n > 0 && !reqs)) return set_last_error(LBPF_E_INVALID, "bad request array");
    const lbpf_server_cfg &c = S->cfg;
    std::vector<Req> batch((size_t)n);
    double prev = -std::numeric_limits<double>::infinity();
    for (int32_t i = 0; i < n; ++i) {
        const lbpf_request &q = reqs[i];
        char buf[160];
        if (!q.grey || !q.depth) {
            snprintf(buf, sizeof buf, "request %d: NULL plane", i);
            return set_last_error(LBPF_E_INVALID, buf);
        }
        if (q.n_boxes < 0 || q.n_boxes > c.max_boxes_per_frame || (q.n_boxes > 0 && !q.boxes)) {
            snprintf(buf, sizeof buf, "request %d: box count %d out of range", i, q.n_boxes);
            return set_last_error(LBPF_E_INVALID, buf);
        }
        if (!std::isfinite(q.t_arrival) || q.t_arrival < prev) {
            snprintf(buf, sizeof buf, "request %d: arrival time decreases", i);
            return set_last_error(LBPF_E_INVALID, buf);
        }
        prev = q.t_arrival;
        for (int32_t k = 0; k < q.n_boxes; ++k) {
            const int32_t *b = q.boxes + 4 * k;
            if (b[2] < 3 || b[3] < 3 || b[2] > LBPF_MAX_SIDE || b[3] > LBPF_MAX_SIDE || b[0] < 0 ||
                b[1] < 0 || (int64_t)b[0] + b[2] > c.frame_w || (int64_t)b[1] + b[3] > c.frame_h) {
                snprintf(buf, sizeof buf, "request %d box %d (%d,%d,%d,%d) outside the frame", i,
                         k, b[0], b[1], b[2], b[3]);
                return set_last_error(LBPF_E_INVALID, buf);
            }
        }
        Req &r = batch[(size_t)i];
        r.id = q.id;
        r.t_arrival = q.t_arrival;
        r.grey = q.grey;
        r.depth = q.depth;
        r.boxes.assign(q.boxes, q.boxes + 4 * (size_t)q.n_boxes);
        r.y0 = c.frame_h;
        r.y1 = 0;
        for (int32_t k = 0; k < q.n_boxes; ++k) {
            r.y0 = std::min(r.y0, q.boxes[4 * k + 1]);
            r.y1 = std::max(r.y1, q.boxes[4 * k + 1] + q.boxes[4 * k + 3]);
        }
        if (r.y1 <= r.y0) r.y0 = r.y1 = 0;  // no boxes: nothing to upload
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->error != LBPF_OK) return set_last_error(S->error, S->error_msg);
        if (n > 0 && batch.front().t_arrival < S->last_arrival)
            return set_last_error(LBPF_E_INVALID, "arrival earlier than an already submitted one");
        for (Req &r : batch) S->pending.push_back(std::move(r));
        if (n > 0) S->last_arrival = S->pending.back().t_arrival;
        S->wake = true;
    }
    S->cv.notify_one();
    return LBPF_OK;
}

lbpf_status lbpf_server_poll(lbpf_server *S, lbpf_result *results, int32_t max_results,
                             int32_t *argmax, int32_t max_argmax, int32_t *n_out) {
    using lbpf::set_last_error;
    if (!S || !n_out || max_results < 0 || max_argmax < 0 || (max_results > 0 && !results) ||
        (max_argmax > 0 && !argmax))
        return set_last_error(LBPF_E_INVALID, "bad poll arguments");
    *n_out = 0;
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t nr = 0, na = 0;
    while (!S->done.empty() && nr < max_results) {
        const Done &d = S->done.front();
        const int32_t nb = (int32_t)d.argmax.size();
        if (na + nb > max_argmax) break;
        results[nr] = lbpf_result{d.id, d.t_arrival, d.t_done, nb, na};
        if (nb) std::memcpy(argmax + na, d.argmax.data(), sizeof(int32_t) * (size_t)nb);
        na += nb;
        ++nr;
        S->done.pop_front();
    }
    *n_out = nr;
    if (S->error != LBPF_OK) return set_last_error(S->error, S->error_msg);
    return LBPF_OK;
}

lbpf_status lbpf_server_get_stats(const lbpf_server *S, lbpf_server_stats *out) {
    if (!S || !out) return lbpf::set_last_error(LBPF_E_INVALID, "NULL argument");
    out->batches = S->n_batches.load();
    out->frames = S->n_frames.load();
    out->boxes = S->n_boxes.load();
    out->deferrals = S->n_deferrals.load();
    out->loop_iterations = S->n_iter.load();
    out->busy_seconds = S->busy_s.load();
    out->seconds = seconds_since(S->t0);
    return LBPF_OK;
}

void lbpf_server_destroy(lbpf_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop.store(true, std::memory_order_release);
        S->wake = true;
    }
    S->cv.notify_one();
    if (S->thread.joinable()) S->thread.join();
    release(S);
}

}  // extern "C"
