// C ABI of liblbpf.so (include/lbpf.h): contexts, host-side validation,
// pinned staging of box tables, weights and dispatch to the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx_internal.h"
#include "gram.h"
#include "lbpf_internal.h"

using namespace lbpf;

namespace {

thread_local std::string g_last_error;

lbpf_status fail(lbpf_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

lbpf_status fail_hip(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return LBPF_E_HIP;
}

#define HIP_TRY(expr, what)                        \
    do {                                           \
        hipError_t _e = (expr);                    \
        if (_e != hipSuccess) return fail_hip(_e, what); \
    } while (0)

constexpr int kRing = 4;

}  // namespace

lbpf_status lbpf::set_last_error(lbpf_status s, const std::string &msg) { return fail(s, msg); }

struct lbpf_ctx {
    int device = 0;
    int num_cus = 256;
    lbpf_feature_cfg cfg{};
    FeatParams fp{};
    size_t budget = 0;   // 0 = unbounded
    size_t used = 0;     // device bytes held by the context, its batches and weights
    uint8_t *d_bins = nullptr;
    CropDesc *h_stage[kRing] = {};
    CropDesc *d_stage[kRing] = {};
    hipEvent_t ev[kRing] = {};
    int ring_next = 0;
    float *d_scores = nullptr;  // scratch for argmax-only scoring
    size_t scores_elems = 0;
    int32_t *d_plain_median = nullptr;  // plain path: one crop's median
    uint32_t *d_plain_counts = nullptr; // plain path: one crop's counts
    std::vector<CropDesc> h_crops;      // host staging of resolved boxes
    hipEvent_t scratch_ev = nullptr;    // last use of d_scores / d_xq / d_sx
    hipEvent_t plain_ev = nullptr;      // last use of d_plain_median / d_plain_counts
    uint8_t *d_xq = nullptr;            // reduced-precision scoring: quantised feature rows
    float *d_sx = nullptr;              //   and their scales, kLpChunkRows rows
    size_t xq_bytes = 0;
    float *d_part = nullptr;            // FP32 scoring over split D: partial tiles
};

struct lbpf_batch {
    lbpf_ctx *ctx = nullptr;
    CropDesc *d_crops = nullptr;
    int32_t *d_order = nullptr;   // crop indices, largest area first
    uint32_t *d_queue = nullptr;  // persistent kernel's work queue (self-resetting)
    int32_t n = 0;
    size_t bytes = 0;
    LaunchCfg lc;
};

struct lbpf_graph {
    lbpf_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// A captured serving step (lbpf_pipeline_*): per replay the host-written box
// table is copied up, then features, (quantisation,) scores and argmax run
// with the batch size read from device memory, and the identities are copied
// back to the caller's pinned memory.
struct lbpf_pipeline {
    lbpf_ctx *ctx = nullptr;
    const lbpf_weights *w = nullptr;
    int32_t max_boxes = 0;
    uint8_t *h_stage = nullptr;  // pinned: CropDesc[max] | int32 order[max] | int32 n
    uint8_t *d_stage = nullptr;  // the same, on the device
    size_t stage_bytes = 0, off_order = 0, off_n = 0;
    uint32_t *d_queue = nullptr;  // persistent feature kernel's work queue
    float *d_scores = nullptr;    // scores when the caller passes none
    uint8_t *d_xq = nullptr;      // reduced precision: quantised rows, scales,
    float *d_sx = nullptr;        //   per-tile argmax pairs
    float *d_apart = nullptr;
    size_t apart_elems = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // end of the last replay (its staging may be reused)
    size_t bytes = 0;           // device bytes charged to the context
    std::vector<CropDesc> crops;
    std::vector<int32_t> order;
};

struct lbpf_weights {
    lbpf_ctx *ctx = nullptr;
    int32_t K = 0, D = 0;
    lbpf_precision prec = LBPF_FP32;
    float *W = nullptr;       // FP32 copy (FP32 precision only)
    float *b = nullptr;
    uint8_t *Wq = nullptr;    // quantised rows (reduced precision)
    float *sw = nullptr;      // their scales
    size_t bytes = 0;
};

namespace {

constexpr size_t kScoreScratchElems = size_t(16) << 20;  // 64 MiB of FP32 scores
constexpr size_t kPartElems = size_t(4) << 20;           // 16 MiB of split-D partial scores
constexpr int32_t kLpChunkRows = 16384;                  // feature rows quantised per pass

bool charge(lbpf_ctx *ctx, size_t bytes) {
    if (ctx->budget && ctx->used + bytes > ctx->budget) return false;
    ctx->used += bytes;
    return true;
}

// Resolve and validate a box table into crop descriptors.
lbpf_status resolve(const lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                    const lbpf_box *boxes, int32_t n_boxes, std::vector<CropDesc> &out) {
    if (n_boxes < 0 || n_images < 0) return fail(LBPF_E_INVALID, "negative count");
    if (n_boxes > 0 && (!boxes || !images || n_images == 0))
        return fail(LBPF_E_INVALID, "NULL image or box table");
    out.resize((size_t)n_boxes);
    for (int32_t i = 0; i < n_boxes; ++i) {
        const lbpf_box &b = boxes[i];
        char buf[160];
        if (b.image < 0 || b.image >= n_images) {
            snprintf(buf, sizeof buf, "box %d: image index %d out of range", i, b.image);
            return fail(LBPF_E_INVALID, buf);
        }
        const lbpf_image &im = images[b.image];
        if (!im.depth || (ctx->fp.use_grey && !im.grey)) {
            snprintf(buf, sizeof buf, "box %d: image %d has a NULL plane", i, b.image);
            return fail(LBPF_E_INVALID, buf);
        }
        if (im.width < 0 || im.height < 0 || im.depth_pitch < im.width ||
            (ctx->fp.use_grey && im.grey_pitch < im.width)) {
            snprintf(buf, sizeof buf, "image %d: bad size or pitch", b.image);
            return fail(LBPF_E_INVALID, buf);
        }
        if (b.w < 3 || b.h < 3 || b.w > LBPF_MAX_SIDE || b.h > LBPF_MAX_SIDE || b.x < 0 ||
            b.y < 0 || (int64_t)b.x + b.w > im.width || (int64_t)b.y + b.h > im.height) {
            snprintf(buf, sizeof buf, "box %d (%d,%d,%d,%d) invalid for image %d (%dx%d)", i,
                     b.x, b.y, b.w, b.h, b.image, im.width, im.height);
            return fail(LBPF_E_INVALID, buf);
        }
        CropDesc &c = out[(size_t)i];
        c.grey = im.grey ? im.grey + (size_t)b.y * im.grey_pitch + b.x : nullptr;
        c.depth = im.depth + (size_t)b.y * im.depth_pitch + b.x;
        c.grey_pitch = im.grey_pitch;
        c.depth_pitch = im.depth_pitch;
        c.w = (int16_t)b.w;
        c.h = (int16_t)b.h;
        // An image spans at least (height - 1) * pitch + width elements; the
        // furthest over-read is kOverRead past the crop's last row.
        const int64_t last = (int64_t)(b.y + b.h - 1);
        const bool g_ok = !im.grey || last * im.grey_pitch + b.x + b.w + kOverRead <=
                                          (int64_t)(im.height - 1) * im.grey_pitch + im.width;
        const bool d_ok = last * im.depth_pitch + b.x + b.w + kOverRead <=
                          (int64_t)(im.height - 1) * im.depth_pitch + im.width;
        c.flags = (g_ok && d_ok) ? kCropOverReadOk : 0u;
    }
    return LBPF_OK;
}

}  // namespace

bool lbpf::ctx_charge(lbpf_ctx *ctx, size_t bytes) { return charge(ctx, bytes); }
void lbpf::ctx_refund(lbpf_ctx *ctx, size_t bytes) { ctx->used -= bytes; }
int lbpf::ctx_device(const lbpf_ctx *ctx) { return ctx->device; }

extern "C" {

const char *lbpf_version(void) { return "lbpf 0.1.0 gfx950"; }

const char *lbpf_status_string(lbpf_status s) {
    switch (s) {
        case LBPF_OK: return "LBPF_OK";
        case LBPF_E_INVALID: return "LBPF_E_INVALID";
        case LBPF_E_BUDGET: return "LBPF_E_BUDGET";
        case LBPF_E_HIP: return "LBPF_E_HIP";
        case LBPF_E_UNSUPPORTED: return "LBPF_E_UNSUPPORTED";
    }
    return "LBPF_E_UNKNOWN";
}

const char *lbpf_last_error(void) { return g_last_error.c_str(); }

lbpf_status lbpf_create(lbpf_ctx **out, const lbpf_feature_cfg *cfg, size_t hbm_budget_bytes) {
    if (!out) return fail(LBPF_E_INVALID, "out is NULL");
    *out = nullptr;
    lbpf_feature_cfg c = cfg ? *cfg : lbpf_feature_cfg{8, 8, LBPF_MAP_U59, 150, LBPF_MOD_BOTH};
    if (c.grid_x < 1 || c.grid_y < 1 || c.grid_x * c.grid_y > 64)
        return fail(LBPF_E_INVALID, "grid must satisfy 1 <= grid_x*grid_y <= 64");
    if (c.mapping != LBPF_MAP_U59 && c.mapping != LBPF_MAP_FULL256)
        return fail(LBPF_E_INVALID, "unknown mapping");
    if (c.modality < LBPF_MOD_BOTH || c.modality > LBPF_MOD_DEPTH)
        return fail(LBPF_E_INVALID, "unknown modality");

    lbpf_ctx *ctx = new (std::nothrow) lbpf_ctx();
    if (!ctx) return fail(LBPF_E_BUDGET, "out of host memory");
    ctx->cfg = c;
    ctx->budget = hbm_budget_bytes;
    FeatParams &fp = ctx->fp;
    fp.grid_x = c.grid_x;
    fp.grid_y = c.grid_y;
    fp.nbins = c.mapping == LBPF_MAP_U59 ? 59 : 256;
    fp.window = c.depth_window_mm;
    fp.use_grey = c.modality != LBPF_MOD_DEPTH;
    fp.use_depth = c.modality != LBPF_MOD_GREY;
    fp.nch = fp.use_grey + fp.use_depth;
    fp.dim = fp.nch * c.grid_x * c.grid_y * fp.nbins;

    auto cleanup = [&](lbpf_status s) {
        lbpf_destroy(ctx);
        return s;
    };
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return cleanup(fail_hip(e, "hipGetDevice"));
    e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) return cleanup(fail_hip(e, "hipDeviceGetAttribute"));

    const size_t stage_bytes = sizeof(CropDesc) * LBPF_MAX_BOXES_PER_CALL;
    const size_t ws = 512 + kRing * stage_bytes + kScoreScratchElems * sizeof(float) +
                      sizeof(int32_t) + sizeof(uint32_t) * (size_t)fp.dim +
                      kPartElems * sizeof(float);
    if (!charge(ctx, ws)) return cleanup(fail(LBPF_E_BUDGET, "workspace exceeds the HBM budget"));

    // Tables: [0,256) code -> bin; [256,512) comparison byte -> bin (the
    // byte's layout is in features.hip).
    uint8_t table[512];
    if (c.mapping == LBPF_MAP_U59) {
        build_uniform59(table);
    } else {
        for (int i = 0; i < 256; ++i) table[i] = (uint8_t)i;
    }
    build_comparison_lut(table, table + 256);
    if ((e = hipMalloc(&ctx->d_bins, sizeof table)) != hipSuccess)
        return cleanup(fail_hip(e, "hipMalloc"));
    if ((e = hipMemcpy(ctx->d_bins, table, sizeof table, hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(fail_hip(e, "hipMemcpy"));
    for (int i = 0; i < kRing; ++i) {
        if ((e = hipHostMalloc((void **)&ctx->h_stage[i], stage_bytes, hipHostMallocDefault)) !=
            hipSuccess)
            return cleanup(fail_hip(e, "hipHostMalloc"));
        if ((e = hipMalloc((void **)&ctx->d_stage[i], stage_bytes)) != hipSuccess)
            return cleanup(fail_hip(e, "hipMalloc"));
        if ((e = hipEventCreateWithFlags(&ctx->ev[i], hipEventDisableTiming)) != hipSuccess)
            return cleanup(fail_hip(e, "hipEventCreate"));
    }
    if ((e = hipMalloc((void **)&ctx->d_scores, kScoreScratchElems * sizeof(float))) != hipSuccess)
        return cleanup(fail_hip(e, "hipMalloc"));
    if ((e = hipEventCreateWithFlags(&ctx->scratch_ev, hipEventDisableTiming)) != hipSuccess)
        return cleanup(fail_hip(e, "hipEventCreate"));
    if ((e = hipEventCreateWithFlags(&ctx->plain_ev, hipEventDisableTiming)) != hipSuccess)
        return cleanup(fail_hip(e, "hipEventCreate"));
    if ((e = hipMalloc((void **)&ctx->d_part, kPartElems * sizeof(float))) != hipSuccess)
        return cleanup(fail_hip(e, "hipMalloc"));
    if ((e = hipMalloc((void **)&ctx->d_plain_median, sizeof(int32_t))) != hipSuccess)
        return cleanup(fail_hip(e, "hipMalloc"));
    if ((e = hipMalloc((void **)&ctx->d_plain_counts, sizeof(uint32_t) * fp.dim)) != hipSuccess)
        return cleanup(fail_hip(e, "hipMalloc"));
    ctx->scores_elems = kScoreScratchElems;
    *out = ctx;
    return LBPF_OK;
}

void lbpf_destroy(lbpf_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    for (int i = 0; i < kRing; ++i) {
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
        if (ctx->h_stage[i]) (void)hipHostFree(ctx->h_stage[i]);
        if (ctx->d_stage[i]) (void)hipFree(ctx->d_stage[i]);
    }
    if (ctx->d_bins) (void)hipFree(ctx->d_bins);
    if (ctx->d_scores) (void)hipFree(ctx->d_scores);
    if (ctx->d_plain_median) (void)hipFree(ctx->d_plain_median);
    if (ctx->scratch_ev) (void)hipEventDestroy(ctx->scratch_ev);
    if (ctx->plain_ev) (void)hipEventDestroy(ctx->plain_ev);
    if (ctx->d_xq) (void)hipFree(ctx->d_xq);
    if (ctx->d_sx) (void)hipFree(ctx->d_sx);
    if (ctx->d_plain_counts) (void)hipFree(ctx->d_plain_counts);
    if (ctx->d_part) (void)hipFree(ctx->d_part);
    delete ctx;
}

int32_t lbpf_feature_dim(const lbpf_ctx *ctx) { return ctx ? ctx->fp.dim : -1; }

lbpf_status lbpf_features(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                          const lbpf_box *boxes, int32_t n_boxes, float *hist,
                          uint32_t *counts_opt, void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (n_boxes > LBPF_MAX_BOXES_PER_CALL)
        return fail(LBPF_E_BUDGET, "more boxes than LBPF_MAX_BOXES_PER_CALL");
    if (n_boxes > 0 && !hist) return fail(LBPF_E_INVALID, "hist is NULL");
    std::vector<CropDesc> crops;
    lbpf_status st = resolve(ctx, images, n_images, boxes, n_boxes, crops);
    if (st != LBPF_OK) return st;
    if (n_boxes == 0) return LBPF_OK;
    hipStream_t s = (hipStream_t)stream;
    const int slot = ctx->ring_next;
    ctx->ring_next = (slot + 1) % kRing;
    HIP_TRY(hipEventSynchronize(ctx->ev[slot]), "hipEventSynchronize");
    std::memcpy(ctx->h_stage[slot], crops.data(), sizeof(CropDesc) * crops.size());
    HIP_TRY(hipMemcpyAsync(ctx->d_stage[slot], ctx->h_stage[slot], sizeof(CropDesc) * crops.size(),
                           hipMemcpyHostToDevice, s),
            "hipMemcpyAsync");
    HIP_TRY(launch_features(ctx->d_stage[slot], n_boxes, ctx->fp, ctx->d_bins, hist, counts_opt, s),
            "feature kernel launch");
    HIP_TRY(hipEventRecord(ctx->ev[slot], s), "hipEventRecord");
    return LBPF_OK;
}

lbpf_status lbpf_batch_create(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                              const lbpf_box *boxes, int32_t n_boxes, lbpf_batch **out) {
    if (!ctx || !out) return fail(LBPF_E_INVALID, "NULL argument");
    *out = nullptr;
    std::vector<CropDesc> crops;
    lbpf_status st = resolve(ctx, images, n_images, boxes, n_boxes, crops);
    if (st != LBPF_OK) return st;
    const size_t nn = crops.size() ? crops.size() : 1;
    const size_t bytes = (sizeof(CropDesc) + sizeof(int32_t)) * nn + 2 * sizeof(uint32_t);
    if (!charge(ctx, bytes)) return fail(LBPF_E_BUDGET, "batch exceeds the HBM budget");
    lbpf_batch *b = new (std::nothrow) lbpf_batch();
    if (!b) {
        ctx->used -= bytes;
        return fail(LBPF_E_BUDGET, "out of host memory");
    }
    b->ctx = ctx;
    b->n = n_boxes;
    b->bytes = bytes;
    // Largest crops first: with a dynamic work queue this is longest-
    // processing-time-first scheduling; ties keep the input order.
    std::vector<int32_t> order(crops.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
        return (int64_t)crops[a].w * crops[a].h > (int64_t)crops[c].w * crops[c].h;
    });
    hipError_t e = hipMalloc((void **)&b->d_crops, sizeof(CropDesc) * nn);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_order, sizeof(int32_t) * nn);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_queue, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(b->d_queue, 0, 2 * sizeof(uint32_t));
    if (e == hipSuccess && n_boxes > 0)
        e = hipMemcpy(b->d_crops, crops.data(), sizeof(CropDesc) * crops.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && n_boxes > 0)
        e = hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * order.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        lbpf_batch_destroy(b);
        return fail_hip(e, "batch upload");
    }
    *out = b;
    return LBPF_OK;
}

void lbpf_batch_destroy(lbpf_batch *b) {
    if (!b) return;
    if (b->d_crops || b->d_order || b->d_queue) (void)hipDeviceSynchronize();
    if (b->d_crops) (void)hipFree(b->d_crops);
    if (b->d_order) (void)hipFree(b->d_order);
    if (b->d_queue) (void)hipFree(b->d_queue);
    if (b->ctx) b->ctx->used -= b->bytes;
    delete b;
}

int32_t lbpf_batch_size(const lbpf_batch *b) { return b ? b->n : -1; }

lbpf_status lbpf_features_batch(lbpf_ctx *ctx, const lbpf_batch *batch, float *hist,
                                uint32_t *counts_opt, void *stream) {
    if (!ctx || !batch) return fail(LBPF_E_INVALID, "NULL argument");
    if (batch->ctx != ctx) return fail(LBPF_E_INVALID, "batch belongs to another context");
    if (batch->n == 0) return LBPF_OK;
    if (!hist) return fail(LBPF_E_INVALID, "hist is NULL");
    HIP_TRY(launch_features(batch->d_crops, batch->n, ctx->fp, ctx->d_bins, hist, counts_opt,
                            (hipStream_t)stream, batch->lc, batch->d_order, batch->d_queue,
                            ctx->num_cus),
            "feature kernel launch");
    return LBPF_OK;
}

static bool launch_cfg_valid(const lbpf_launch_cfg &c) {
    return (c.persistent == 0 || c.persistent == 1) && c.wg_per_cu >= 1 && c.wg_per_cu <= 16 &&
           (c.row_prefetch == 2 || c.row_prefetch == 4 || c.row_prefetch == 8) && (c.sorted == 0 || c.sorted == 1);
}

lbpf_status lbpf_batch_set_launch(lbpf_batch *batch, const lbpf_launch_cfg *cfg) {
    if (!batch || !cfg || !launch_cfg_valid(*cfg)) return fail(LBPF_E_INVALID, "bad launch config");
    batch->lc.persistent = cfg->persistent;
    batch->lc.wg_per_cu = cfg->wg_per_cu;
    batch->lc.row_prefetch = cfg->row_prefetch;
    batch->lc.sorted = cfg->sorted;
    return LBPF_OK;
}

lbpf_status lbpf_batch_get_launch(const lbpf_batch *batch, lbpf_launch_cfg *cfg) {
    if (!batch || !cfg) return fail(LBPF_E_INVALID, "NULL argument");
    *cfg = lbpf_launch_cfg{batch->lc.persistent, batch->lc.wg_per_cu, batch->lc.row_prefetch,
                           batch->lc.sorted};
    return LBPF_OK;
}

lbpf_status lbpf_tune_batch(lbpf_ctx *ctx, lbpf_batch *batch, float *hist, int32_t reps,
                            lbpf_launch_cfg *best_out, float *best_us_out, void *stream) {
    if (!ctx || !batch || !hist || reps < 1) return fail(LBPF_E_INVALID, "bad tuning arguments");
    if (batch->ctx != ctx) return fail(LBPF_E_INVALID, "batch belongs to another context");
    hipStream_t s = (hipStream_t)stream;
    std::vector<lbpf_launch_cfg> cands;
    for (int pf : {2, 4, 8}) cands.push_back({0, 4, pf, 1});
    for (int m : {2, 4, 5, 6})
        for (int pf : {2, 4})
            for (int so : {0, 1}) cands.push_back({1, m, pf, so});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t er = hipEventCreate(&e1);
    if (er != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail_hip(er, "hipEventCreate");
    }
    const LaunchCfg saved = batch->lc;
    float best = 0.f;
    lbpf_launch_cfg best_cfg = cands[0];
    lbpf_status st = LBPF_OK;
    // Two rounds over the candidates, so a shape timed while the device was
    // still warming up (clocks, caches) gets a second chance; the fastest
    // average of a round wins.
    std::vector<lbpf_launch_cfg> rounds(cands);
    rounds.insert(rounds.end(), cands.begin(), cands.end());
    for (const auto &cand : rounds) {
        lbpf_batch_set_launch(batch, &cand);
        er = launch_features(batch->d_crops, batch->n, ctx->fp, ctx->d_bins, hist, nullptr, s,
                             batch->lc, batch->d_order, batch->d_queue, ctx->num_cus);
        if (er == hipSuccess) er = hipEventRecord(e0, s);
        for (int r = 0; r < reps && er == hipSuccess; ++r)
            er = launch_features(batch->d_crops, batch->n, ctx->fp, ctx->d_bins, hist, nullptr, s,
                                 batch->lc, batch->d_order, batch->d_queue, ctx->num_cus);
        if (er == hipSuccess) er = hipEventRecord(e1, s);
        if (er == hipSuccess) er = hipEventSynchronize(e1);
        float ms = 0.f;
        if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
        if (er != hipSuccess) {
            st = fail_hip(er, "tuning run");
            break;
        }
        const float us = 1000.f * ms / (float)reps;
        if (best == 0.f || us < best) {
            best = us;
            best_cfg = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    batch->lc = saved;
    if (st != LBPF_OK) return st;
    lbpf_batch_set_launch(batch, &best_cfg);
    if (best_out) *best_out = best_cfg;
    if (best_us_out) *best_us_out = best;
    return LBPF_OK;
}

lbpf_status lbpf_graph_create(lbpf_ctx *ctx, const lbpf_batch *batch, const lbpf_weights *w,
                              float *hist, float *scores_opt, int32_t *argmax_opt,
                              lbpf_graph **out) {
    if (!ctx || !batch || !hist || !out) return fail(LBPF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (batch->ctx != ctx || (w && w->ctx != ctx))
        return fail(LBPF_E_INVALID, "batch or weights belong to another context");
    if (w && !scores_opt && !argmax_opt) return fail(LBPF_E_INVALID, "no scoring output");
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    lbpf_graph *g = new (std::nothrow) lbpf_graph();
    if (!g) {
        (void)hipStreamDestroy(cs);
        return fail(LBPF_E_BUDGET, "out of host memory");
    }
    g->ctx = ctx;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    lbpf_status st = LBPF_OK;
    if (e == hipSuccess) {
        st = lbpf_features_batch(ctx, batch, hist, nullptr, cs);
        if (st == LBPF_OK && w) st = lbpf_score(ctx, hist, batch->n, w, scores_opt, argmax_opt, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (st == LBPF_OK && e2 != hipSuccess) st = fail_hip(e2, "hipStreamEndCapture");
    } else {
        st = fail_hip(e, "hipStreamBeginCapture");
    }
    if (st == LBPF_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = fail_hip(e, "hipGraphInstantiate");
    }
    (void)hipStreamDestroy(cs);
    if (st != LBPF_OK) {
        lbpf_graph_destroy(g);
        return st;
    }
    *out = g;
    return LBPF_OK;
}

lbpf_status lbpf_graph_launch(lbpf_graph *g, void *stream) {
    if (!g || !g->exec) return fail(LBPF_E_INVALID, "NULL graph");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
    return LBPF_OK;
}

void lbpf_graph_destroy(lbpf_graph *g) {
    if (!g) return;
    if (g->exec) {
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(g->exec);
    }
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

lbpf_status lbpf_weights_create(lbpf_ctx *ctx, const float *W, const float *b, int32_t K,
                                lbpf_precision precision, lbpf_weights **out, void *stream) {
    if (!ctx || !W || !b || !out || K < 1) return fail(LBPF_E_INVALID, "bad weights arguments");
    *out = nullptr;
    if (precision < LBPF_FP32 || precision > LBPF_F16X3)
        return fail(LBPF_E_UNSUPPORTED, "unknown precision");
    const int32_t D = ctx->fp.dim;
    const bool lp = precision != LBPF_FP32;
    const size_t bbytes = sizeof(float) * (size_t)K;
    const size_t wbytes = lp ? (size_t)K * lp_pitch(D, precision) + bbytes
                             : sizeof(float) * (size_t)K * D;
    // Reduced-precision weights need the context's feature quantisation
    // scratch: kLpChunkRows rows at this precision's feature pitch (at least
    // the BF16 one). It is allocated with the first such weights and grows
    // when wider ones arrive (split FP16 rows are twice as wide); its two
    // buffers are replaced as a pair, and on any failure the old pair stays
    // and the charge is refunded.
    const size_t xq_want =
        lp ? (size_t)kLpChunkRows * (size_t)std::max(lp_pitch_features(D, LBPF_BF16),
                                                     lp_pitch_features(D, precision))
           : 0;
    const bool grow = lp && (!ctx->d_xq || !ctx->d_sx || ctx->xq_bytes < xq_want);
    const size_t xq_need = grow ? xq_want : 0;
    const size_t sx_need = grow ? sizeof(float) * kLpChunkRows : 0;
    const size_t old_pair = (grow && ctx->d_xq) ? ctx->xq_bytes + sizeof(float) * kLpChunkRows : 0;
    if (!charge(ctx, wbytes + bbytes + xq_need + sx_need))
        return fail(LBPF_E_BUDGET, "weights exceed the HBM budget");
    if (grow) {
        uint8_t *xq = nullptr;
        float *sx = nullptr;
        hipError_t ea = hipMalloc((void **)&xq, xq_need);
        if (ea == hipSuccess) ea = hipMalloc((void **)&sx, sx_need);
        if (ea != hipSuccess) {
            if (xq) (void)hipFree(xq);
            ctx->used -= wbytes + bbytes + xq_need + sx_need;
            return fail_hip(ea, "quantisation scratch");
        }
        if (ctx->d_xq || ctx->d_sx) {
            // Scoring already queued may still read the old pair.
            (void)hipDeviceSynchronize();
            if (ctx->d_xq) (void)hipFree(ctx->d_xq);
            if (ctx->d_sx) (void)hipFree(ctx->d_sx);
            ctx->used -= old_pair;
        }
        ctx->d_xq = xq;
        ctx->d_sx = sx;
        ctx->xq_bytes = xq_need;
    }
    lbpf_weights *w = new (std::nothrow) lbpf_weights();
    if (!w) {
        ctx->used -= wbytes + bbytes;  // the scratch stays with the context
        return fail(LBPF_E_BUDGET, "out of host memory");
    }
    w->ctx = ctx;
    w->K = K;
    w->D = D;
    w->prec = precision;
    w->bytes = wbytes + bbytes;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMalloc((void **)&w->b, bbytes);
    if (e == hipSuccess) e = hipMemcpyAsync(w->b, b, bbytes, hipMemcpyDeviceToDevice, s);
    if (!lp) {
        if (e == hipSuccess) e = hipMalloc((void **)&w->W, sizeof(float) * (size_t)K * D);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w->W, W, sizeof(float) * (size_t)K * D, hipMemcpyDeviceToDevice, s);
    } else {
        if (e == hipSuccess) e = hipMalloc((void **)&w->Wq, (size_t)K * lp_pitch(D, precision));
        if (e == hipSuccess) e = hipMalloc((void **)&w->sw, bbytes);
        if (e == hipSuccess) e = launch_quant_rows(W, K, D, precision, w->Wq, w->sw, s, nullptr, true);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        lbpf_weights_destroy(w);
        return fail_hip(e, "weights upload");
    }
    *out = w;
    return LBPF_OK;
}

void lbpf_weights_destroy(lbpf_weights *w) {
    if (!w) return;
    if (w->W || w->b || w->Wq) (void)hipDeviceSynchronize();
    if (w->W) (void)hipFree(w->W);
    if (w->b) (void)hipFree(w->b);
    if (w->Wq) (void)hipFree(w->Wq);
    if (w->sw) (void)hipFree(w->sw);
    if (w->ctx) w->ctx->used -= w->bytes;
    delete w;
}

int32_t lbpf_weights_count(const lbpf_weights *w) { return w ? w->K : -1; }

lbpf_status lbpf_score(lbpf_ctx *ctx, const float *hist, int32_t N, const lbpf_weights *w,
                       float *scores_opt, int32_t *argmax_opt, void *stream) {
    if (!ctx || !w) return fail(LBPF_E_INVALID, "NULL argument");
    if (w->ctx != ctx) return fail(LBPF_E_INVALID, "weights belong to another context");
    if (N < 0) return fail(LBPF_E_INVALID, "N < 0");
    if (!scores_opt && !argmax_opt) return fail(LBPF_E_INVALID, "no output requested");
    if (N == 0) return LBPF_OK;
    if (!hist) return fail(LBPF_E_INVALID, "hist is NULL");
    hipStream_t s = (hipStream_t)stream;
    const size_t K = (size_t)w->K, D = (size_t)w->D;
    // Rows per pass: all of them when scores go to the caller's buffer,
    // otherwise as many as the context's score scratch holds. Reduced
    // precision passes are chunks of quantised rows; an argmax-only chunk
    // keeps only per-tile (score, identity) pairs in the scratch (the
    // small-product kernel blocks its rows to fit), so whole chunks run.
    int32_t rows = scores_opt ? N : (int32_t)std::max<size_t>(1, ctx->scores_elems / K);
    if (w->prec != LBPF_FP32) {
        const size_t tiles = (K + 255) / 256;
        if (!scores_opt && 2 * (size_t)kLpChunkRows * tiles <= ctx->scores_elems)
            rows = kLpChunkRows;
        rows = std::min(rows, kLpChunkRows);
    }
    // FP32 products too small to fill the GPU with 128 x 128 tiles split D
    // (partials in the context's scratch).
    const int32_t splits =
        w->prec == LBPF_FP32
            ? score_f32_splits(std::min(rows, N), w->K, w->D, ctx->num_cus, kPartElems)
            : 1;
    // Calls that use the context's scratch (reduced precision, argmax without
    // caller scores, split D) are ordered across streams by scratch_ev. Under
    // graph capture the graph's own order applies instead.
    const bool uses_scratch = w->prec != LBPF_FP32 || !scores_opt || splits > 1;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap), "hipStreamIsCapturing");
    const bool order = uses_scratch && cap == hipStreamCaptureStatusNone;
    if (order) HIP_TRY(hipStreamWaitEvent(s, ctx->scratch_ev, 0), "hipStreamWaitEvent");
    for (int32_t n0 = 0; n0 < N; n0 += rows) {
        const int32_t n = std::min(rows, N - n0);
        float *S = scores_opt ? scores_opt + (size_t)n0 * K : ctx->d_scores;
        if (w->prec != LBPF_FP32) {
            HIP_TRY(launch_quant_rows(hist + (size_t)n0 * D, n, w->D, w->prec, ctx->d_xq,
                                      ctx->d_sx, s),
                    "quantise launch");
            // The argmax comes from the GEMM's epilogue where it can; the
            // scratch then holds its per-tile pairs (and S nothing).
            HIP_TRY(launch_score_lp(ctx->d_xq, ctx->d_sx, n, w->Wq, w->sw, w->b, w->K, w->D,
                                    w->prec, scores_opt ? S : nullptr,
                                    argmax_opt ? argmax_opt + n0 : nullptr, ctx->d_scores,
                                    ctx->scores_elems, s),
                    "score launch");
            continue;
        }
        const int32_t sp = n == std::min(rows, N)
                               ? splits
                               : score_f32_splits(n, w->K, w->D, ctx->num_cus, kPartElems);
        HIP_TRY(launch_score_f32(hist + (size_t)n0 * D, n, w->W, w->b, w->K, w->D, S,
                                 argmax_opt ? argmax_opt + n0 : nullptr, s, sp, ctx->d_part),
                "score launch");
    }
    if (order) HIP_TRY(hipEventRecord(ctx->scratch_ev, s), "hipEventRecord");
    return LBPF_OK;
}

void lbpf_pipeline_destroy(lbpf_pipeline *p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    for (void *d : {(void *)p->d_stage, (void *)p->d_queue, (void *)p->d_scores, (void *)p->d_xq,
                    (void *)p->d_sx, (void *)p->d_apart})
        if (d) (void)hipFree(d);
    if (p->ctx) p->ctx->used -= p->bytes;
    delete p;
}

lbpf_status lbpf_pipeline_create(lbpf_ctx *ctx, const lbpf_weights *w, int32_t max_boxes,
                                 float *hist, float *scores_opt, int32_t *argmax,
                                 int32_t *argmax_host_opt, lbpf_pipeline **out) {
    if (!ctx || !w || !hist || !argmax || !out) return fail(LBPF_E_INVALID, "NULL argument");
    *out = nullptr;
    if (w->ctx != ctx) return fail(LBPF_E_INVALID, "weights belong to another context");
    if (max_boxes < 1 || max_boxes > LBPF_MAX_BOXES_PER_CALL)
        return fail(LBPF_E_BUDGET, "max_boxes outside 1..LBPF_MAX_BOXES_PER_CALL");
    if (!fast_path_ok(ctx->fp))
        return fail(LBPF_E_UNSUPPORTED, "pipelines need the default feature configuration "
                                        "(uniform-59 bins, both channels, window 1..255)");
    const int32_t K = w->K, D = w->D;
    const bool lp = w->prec != LBPF_FP32;
    if (!lp && (D % 32 != 0 || ((uintptr_t)hist & 15) || ((uintptr_t)w->W & 15)))
        return fail(LBPF_E_UNSUPPORTED, "FP32 pipelines need D % 32 == 0 and 16-byte aligned hist");
    lbpf_pipeline *p = new (std::nothrow) lbpf_pipeline();
    if (!p) return fail(LBPF_E_BUDGET, "out of host memory");
    p->ctx = ctx;
    p->w = w;
    p->max_boxes = max_boxes;
    const size_t mb = (size_t)max_boxes;
    p->off_order = sizeof(CropDesc) * mb;
    p->off_n = p->off_order + sizeof(int32_t) * mb;
    p->stage_bytes = p->off_n + sizeof(int32_t);
    const int32_t KT = (K + 255) / 256;
    p->apart_elems = lp ? 2 * mb * (size_t)KT : 0;
    const size_t need = p->stage_bytes + 2 * sizeof(uint32_t) +
                        (scores_opt ? 0 : sizeof(float) * mb * (size_t)K) +
                        (lp ? mb * (size_t)lp_pitch_features(D, w->prec) + sizeof(float) * mb +
                                  sizeof(float) * p->apart_elems
                            : 0);
    if (!charge(ctx, need)) {
        delete p;
        return fail(LBPF_E_BUDGET, "pipeline exceeds the HBM budget");
    }
    p->bytes = need;
    p->crops.reserve(mb);
    p->order.resize(mb);
    auto cleanup = [&](lbpf_status st) {
        lbpf_pipeline_destroy(p);
        return st;
    };
    hipError_t e = hipHostMalloc((void **)&p->h_stage, p->stage_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_stage, p->stage_bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_queue, 2 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(p->d_queue, 0, 2 * sizeof(uint32_t));
    if (e == hipSuccess && !scores_opt)
        e = hipMalloc((void **)&p->d_scores, sizeof(float) * mb * (size_t)K);
    if (e == hipSuccess && lp)
        e = hipMalloc((void **)&p->d_xq, mb * (size_t)lp_pitch_features(D, w->prec));
    if (e == hipSuccess && lp) e = hipMalloc((void **)&p->d_sx, sizeof(float) * mb);
    if (e == hipSuccess && lp) e = hipMalloc((void **)&p->d_apart, sizeof(float) * p->apart_elems);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return cleanup(fail_hip(e, "pipeline allocation"));
    std::memset(p->h_stage, 0, p->stage_bytes);  // n = 0 until the first launch

    float *S = scores_opt ? scores_opt : p->d_scores;
    const CropDesc *d_crops = reinterpret_cast<const CropDesc *>(p->d_stage);
    const int32_t *d_order = reinterpret_cast<const int32_t *>(p->d_stage + p->off_order);
    const int32_t *d_n = reinterpret_cast<const int32_t *>(p->d_stage + p->off_n);
    // The persistent feature kernel (4 workgroups per CU, 2 rows prefetched)
    // takes the crops in the order the host wrote: largest first.
    LaunchCfg lc;
    lc.persistent = 1;
    lc.wg_per_cu = 4;
    lc.row_prefetch = 2;
    lc.sorted = 1;
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return cleanup(fail_hip(e, "hipStreamCreate"));
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = hipMemcpyAsync(p->d_stage, p->h_stage, p->stage_bytes,
                                       hipMemcpyHostToDevice, cs);
        if (el == hipSuccess)
            el = launch_features(d_crops, max_boxes, ctx->fp, ctx->d_bins, hist, nullptr, cs, lc,
                                 d_order, p->d_queue, ctx->num_cus, d_n);
        if (el == hipSuccess && !lp)
            el = launch_score_f32(hist, max_boxes, w->W, w->b, K, D, S, argmax, cs, 1, nullptr, d_n);
        if (el == hipSuccess && lp)
            el = launch_quant_rows(hist, max_boxes, D, w->prec, p->d_xq, p->d_sx, cs, d_n);
        if (el == hipSuccess && lp)
            el = launch_score_lp(p->d_xq, p->d_sx, max_boxes, w->Wq, w->sw, w->b, K, D, w->prec, S,
                                 argmax, p->d_apart, p->apart_elems, cs, d_n);
        if (el == hipSuccess && argmax_host_opt)
            el = hipMemcpyAsync(argmax_host_opt, argmax, sizeof(int32_t) * mb,
                                hipMemcpyDeviceToHost, cs);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cs, &graph);
        p->graph = graph;
        e = el != hipSuccess ? el : ee;
    }
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return cleanup(fail_hip(e, "pipeline capture"));
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return cleanup(fail_hip(e, "hipGraphInstantiate"));
    *out = p;
    return LBPF_OK;
}

lbpf_status lbpf_pipeline_launch(lbpf_pipeline *p, const lbpf_image *images, int32_t n_images,
                                 const lbpf_box *boxes, int32_t n_boxes, void *stream) {
    if (!p) return fail(LBPF_E_INVALID, "pipeline is NULL");
    if (n_boxes > p->max_boxes) return fail(LBPF_E_BUDGET, "more boxes than the pipeline's max_boxes");
    lbpf_status st = resolve(p->ctx, images, n_images, boxes, n_boxes, p->crops);
    if (st != LBPF_OK) return st;
    // The previous replay reads the staging buffer: wait for it to finish
    // (a no-op when the caller already waited for its results).
    HIP_TRY(hipEventSynchronize(p->done), "hipEventSynchronize");
    const size_t n = (size_t)n_boxes;
    for (size_t i = 0; i < n; ++i) p->order[i] = (int32_t)i;
    std::stable_sort(p->order.begin(), p->order.begin() + n, [&](int32_t a, int32_t c) {
        return (int64_t)p->crops[a].w * p->crops[a].h > (int64_t)p->crops[c].w * p->crops[c].h;
    });
    std::memcpy(p->h_stage, p->crops.data(), sizeof(CropDesc) * n);
    std::memcpy(p->h_stage + p->off_order, p->order.data(), sizeof(int32_t) * n);
    const int32_t nb = n_boxes;
    std::memcpy(p->h_stage + p->off_n, &nb, sizeof nb);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipGraphLaunch(p->exec, s), "hipGraphLaunch");
    HIP_TRY(hipEventRecord(p->done, s), "hipEventRecord");
    return LBPF_OK;
}

int32_t lbpf_pipeline_max_boxes(const lbpf_pipeline *p) { return p ? p->max_boxes : -1; }

size_t lbpf_warp_crop_bytes(int32_t w, int32_t h) {
    if (w < 3 || h < 3 || w > LBPF_MAX_SIDE || h > LBPF_MAX_SIDE) return 0;
    const size_t px = (size_t)w * (size_t)h;
    // Each plane keeps kOverRead elements of slack past its last row, so the
    // feature kernels' row loads may run past the right edge.
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    return up(px + 2 * kOverRead) + up(2 * px + 4 * kOverRead);
}

lbpf_status lbpf_features_warped(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                                 const lbpf_warp_box *boxes, int32_t n_boxes, void *workspace,
                                 size_t workspace_bytes, float *hist, uint32_t *counts_opt,
                                 void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (n_boxes < 0 || n_images < 0) return fail(LBPF_E_INVALID, "negative count");
    if (n_boxes > LBPF_MAX_BOXES_PER_CALL)
        return fail(LBPF_E_BUDGET, "more boxes than LBPF_MAX_BOXES_PER_CALL");
    if (n_boxes == 0) return LBPF_OK;
    if (!boxes || !images || n_images == 0 || !hist)
        return fail(LBPF_E_INVALID, "NULL image table, box table or hist");
    if (!workspace || ((uintptr_t)workspace & 255u))
        return fail(LBPF_E_INVALID, "workspace is NULL or not 256-byte aligned");
    const bool grey = ctx->fp.use_grey != 0;
    // Range of one sampled coordinate over the crop: an affine function takes
    // its extremes at the corners and floor is monotone, so the corner
    // samples bound every sample.
    auto range = [](int32_t a, int32_t b, int32_t t, int32_t w, int32_t h, int64_t &lo,
                    int64_t &hi) {
        lo = INT64_MAX;
        hi = INT64_MIN;
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int64_t v = ((int64_t)a * (cx ? w - 1 : 0) + (int64_t)b * (cy ? h - 1 : 0) +
                                   t) >> 16;
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
    };
    size_t largest = 0;
    for (int32_t i = 0; i < n_boxes; ++i) {
        const lbpf_warp_box &b = boxes[i];
        char buf[200];
        if (b.image < 0 || b.image >= n_images) {
            snprintf(buf, sizeof buf, "warped box %d: image index %d out of range", i, b.image);
            return fail(LBPF_E_INVALID, buf);
        }
        const lbpf_image &im = images[b.image];
        if (!im.depth || (grey && !im.grey) || im.width < 1 || im.height < 1 ||
            im.depth_pitch < im.width || (grey && im.grey_pitch < im.width)) {
            snprintf(buf, sizeof buf, "warped box %d: image %d has a NULL plane or a bad size", i,
                     b.image);
            return fail(LBPF_E_INVALID, buf);
        }
        const size_t cb = lbpf_warp_crop_bytes(b.w, b.h);
        if (cb == 0) {
            snprintf(buf, sizeof buf, "warped box %d: side %dx%d outside 3..%d", i, b.w, b.h,
                     LBPF_MAX_SIDE);
            return fail(LBPF_E_INVALID, buf);
        }
        largest = std::max(largest, cb);
        for (int p = 0; p < (grey ? 2 : 1); ++p) {
            const lbpf_frame &f = p == 0 ? b.depth : b.grey;
            int64_t x0, x1, y0, y1;
            range(f.ux, f.vx, f.tx, b.w, b.h, x0, x1);
            range(f.uy, f.vy, f.ty, b.w, b.h, y0, y1);
            if (x0 < 0 || y0 < 0 || x1 >= im.width || y1 >= im.height) {
                snprintf(buf, sizeof buf,
                         "warped box %d: %s samples x %lld..%lld, y %lld..%lld leave the %dx%d image",
                         i, p == 0 ? "depth" : "grey", (long long)x0, (long long)x1,
                         (long long)y0, (long long)y1, im.width, im.height);
                return fail(LBPF_E_INVALID, buf);
            }
        }
    }
    if (workspace_bytes < largest)
        return fail(LBPF_E_INVALID, "workspace smaller than the largest warped crop");

    hipStream_t s = (hipStream_t)stream;
    const size_t D = (size_t)ctx->fp.dim;
    const size_t slot_bytes = sizeof(CropDesc) * LBPF_MAX_BOXES_PER_CALL;
    const int32_t max_group = (int32_t)((slot_bytes - 256) / (sizeof(CropDesc) + sizeof(WarpDesc)));
    uint8_t *ws = static_cast<uint8_t *>(workspace);
    int32_t first = 0;
    while (first < n_boxes) {
        // The group: boxes first .. last-1 whose crops fit the workspace.
        int32_t last = first;
        size_t used = 0;
        while (last < n_boxes && last - first < max_group) {
            const size_t cb = lbpf_warp_crop_bytes(boxes[last].w, boxes[last].h);
            if (used + cb > workspace_bytes) break;
            used += cb;
            ++last;
        }
        const int32_t n = last - first;
        const int slot = ctx->ring_next;
        ctx->ring_next = (slot + 1) % kRing;
        HIP_TRY(hipEventSynchronize(ctx->ev[slot]), "hipEventSynchronize");
        uint8_t *h = reinterpret_cast<uint8_t *>(ctx->h_stage[slot]);
        uint8_t *d = reinterpret_cast<uint8_t *>(ctx->d_stage[slot]);
        CropDesc *hc = reinterpret_cast<CropDesc *>(h);
        const size_t woff = (sizeof(CropDesc) * (size_t)n + 255) / 256 * 256;
        WarpDesc *hw = reinterpret_cast<WarpDesc *>(h + woff);
        size_t off = 0;
        for (int32_t j = 0; j < n; ++j) {
            const lbpf_warp_box &b = boxes[first + j];
            const lbpf_image &im = images[b.image];
            const size_t px = (size_t)b.w * (size_t)b.h;
            uint8_t *g_dst = ws + off;
            uint16_t *d_dst = reinterpret_cast<uint16_t *>(
                ws + off + (px + 2 * kOverRead + 255) / 256 * 256);
            off += lbpf_warp_crop_bytes(b.w, b.h);
            WarpDesc &wd = hw[j];
            wd.g_src = grey ? im.grey : nullptr;
            wd.d_src = im.depth;
            wd.g_dst = g_dst;
            wd.d_dst = d_dst;
            wd.g_pitch = im.grey_pitch;
            wd.d_pitch = im.depth_pitch;
            wd.src_w = im.width;
            wd.src_h = im.height;
            wd.w = b.w;
            wd.h = b.h;
            const lbpf_frame fr[2] = {b.grey, b.depth};
            for (int p = 0; p < 2; ++p) {
                int32_t *o = p == 0 ? wd.gf : wd.df;
                o[0] = fr[p].ux; o[1] = fr[p].uy; o[2] = fr[p].vx;
                o[3] = fr[p].vy; o[4] = fr[p].tx; o[5] = fr[p].ty;
            }
            CropDesc &c = hc[j];
            c.grey = grey ? g_dst : nullptr;
            c.depth = d_dst;
            c.grey_pitch = b.w;
            c.depth_pitch = b.w;
            c.w = (int16_t)b.w;
            c.h = (int16_t)b.h;
            c.flags = kCropOverReadOk;
        }
        HIP_TRY(hipMemcpyAsync(d, h, woff + sizeof(WarpDesc) * (size_t)n, hipMemcpyHostToDevice, s),
                "hipMemcpyAsync");
        HIP_TRY(launch_warp(reinterpret_cast<const WarpDesc *>(d + woff), n, s), "warp kernel launch");
        HIP_TRY(launch_features(reinterpret_cast<const CropDesc *>(d), n, ctx->fp, ctx->d_bins,
                                hist + (size_t)first * D,
                                counts_opt ? counts_opt + (size_t)first * D : nullptr, s),
                "feature kernel launch");
        HIP_TRY(hipEventRecord(ctx->ev[slot], s), "hipEventRecord");
        first = last;
    }
    return LBPF_OK;
}

lbpf_status lbpf_track(lbpf_ctx *ctx, const int32_t *prev, const int32_t *prev_stream,
                       int32_t P, const int32_t *cur, const int32_t *cur_stream, int32_t C,
                       int64_t gate2, int32_t *match, int32_t *owner, void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (P < 0 || C < 0) return fail(LBPF_E_INVALID, "negative count");
    if (P > kTrackMaxBoxes || C > kTrackMaxBoxes)
        return fail(LBPF_E_BUDGET, "more than 16384 tracks or boxes");
    if ((P > 0 && (!prev || !prev_stream || !match)) || (C > 0 && (!cur || !cur_stream || !owner)))
        return fail(LBPF_E_INVALID, "NULL box, stream or output array");
    auto ok = [](const int32_t *b, int32_t n) {
        for (int64_t i = 0; i < 4 * (int64_t)n; ++i) {
            if (b[i] < -kTrackMaxCoord || b[i] > kTrackMaxCoord) return false;
            if ((i & 3) >= 2 && b[i] < 0) return false;
        }
        return true;
    };
    if (!ok(prev, P) || !ok(cur, C))
        return fail(LBPF_E_INVALID, "box values must lie within +-32767 with w, h >= 0");
    if (gate2 > ((int64_t)1 << 36)) gate2 = 0;  // wider than any distance: no gate
    if (P == 0 && C == 0) return LBPF_OK;
    hipStream_t s = (hipStream_t)stream;
    const int slot = ctx->ring_next;
    ctx->ring_next = (slot + 1) % kRing;
    HIP_TRY(hipEventSynchronize(ctx->ev[slot]), "hipEventSynchronize");
    // Slot layout: prev [P][4], prev_stream [P], cur [C][4], cur_stream [C],
    // then 256-byte aligned u64 keys [C] (device only).
    uint8_t *h = reinterpret_cast<uint8_t *>(ctx->h_stage[slot]);
    uint8_t *d = reinterpret_cast<uint8_t *>(ctx->d_stage[slot]);
    const size_t o_ps = 16 * (size_t)P, o_cur = o_ps + 4 * (size_t)P, o_cs = o_cur + 16 * (size_t)C;
    const size_t bytes = o_cs + 4 * (size_t)C;
    const size_t o_keys = (bytes + 255) / 256 * 256;
    std::memcpy(h, prev, 16 * (size_t)P);
    std::memcpy(h + o_ps, prev_stream, 4 * (size_t)P);
    std::memcpy(h + o_cur, cur, 16 * (size_t)C);
    std::memcpy(h + o_cs, cur_stream, 4 * (size_t)C);
    HIP_TRY(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    HIP_TRY(launch_track(reinterpret_cast<const int32_t *>(d), reinterpret_cast<const int32_t *>(d + o_ps),
                         P, reinterpret_cast<const int32_t *>(d + o_cur),
                         reinterpret_cast<const int32_t *>(d + o_cs), C, gate2, match, owner,
                         reinterpret_cast<uint64_t *>(d + o_keys), s),
            "tracking kernel launch");
    HIP_TRY(hipEventRecord(ctx->ev[slot], s), "hipEventRecord");
    return LBPF_OK;
}

size_t lbpf_train_workspace_bytes(int32_t N) { return N > 0 ? train_workspace_bytes(N) : 0; }

lbpf_status lbpf_train_ovr(lbpf_ctx *ctx, const float *X, const int32_t *labels, int32_t N,
                           int32_t K, double C, double eps, int32_t max_epochs, uint64_t seed,
                           double *alpha_io, int32_t warm, float *W, float *b, double *W64_opt,
                           double *b64_opt, int32_t *epochs_opt, void *workspace,
                           size_t workspace_bytes, void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (!X || !labels || !W || !b || !workspace)
        return fail(LBPF_E_INVALID, "NULL X, labels, W, b or workspace");
    if (N < 1 || K < 1) return fail(LBPF_E_INVALID, "N and K must be >= 1");
    if (!(C > 0.0) || !(eps > 0.0) || max_epochs < 1)
        return fail(LBPF_E_INVALID, "C and eps must be > 0 and max_epochs >= 1");
    if (warm && !alpha_io) return fail(LBPF_E_INVALID, "warm start without alpha_io");
    if ((uintptr_t)workspace & 7u) return fail(LBPF_E_INVALID, "workspace not 8-byte aligned");
    if (workspace_bytes < train_workspace_bytes(N))
        return fail(LBPF_E_INVALID, "workspace smaller than lbpf_train_workspace_bytes(N)");
    if (ctx->fp.dim > kTrainMaxD || N > kTrainMaxN)
        return fail(LBPF_E_UNSUPPORTED, "training supports D <= 8192 and N <= 12288");
    HIP_TRY(launch_train(X, labels, N, ctx->fp.dim, K, C, eps, max_epochs, seed, alpha_io, warm,
                         W, b, W64_opt, b64_opt, epochs_opt, workspace, (hipStream_t)stream),
            "training kernel launch");
    return LBPF_OK;
}

size_t lbpf_train_gram_workspace_bytes(int32_t N, int32_t K) {
    return N > 0 && K > 0 ? train_gram_workspace_bytes(N, K) : 0;
}

lbpf_status lbpf_train_ovr_gram(lbpf_ctx *ctx, const float *X, const int32_t *labels, int32_t N,
                                int32_t K, double C, double eps, int32_t max_epochs,
                                uint64_t seed, float *alpha_io, int32_t warm, float *W, float *b,
                                int32_t *epochs_opt, void *workspace, size_t workspace_bytes,
                                void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (!X || !labels || !W || !b || !workspace)
        return fail(LBPF_E_INVALID, "NULL X, labels, W, b or workspace");
    if (N < 1 || K < 1) return fail(LBPF_E_INVALID, "N and K must be >= 1");
    if (!(C > 0.0) || !(eps > 0.0) || max_epochs < 1)
        return fail(LBPF_E_INVALID, "C and eps must be > 0 and max_epochs >= 1");
    if (warm && !alpha_io) return fail(LBPF_E_INVALID, "warm start without alpha_io");
    if ((uintptr_t)workspace & 15u) return fail(LBPF_E_INVALID, "workspace not 16-byte aligned");
    if (ctx->fp.dim > kTrainMaxD || N > kGramMaxN)
        return fail(LBPF_E_UNSUPPORTED, "Gram training supports D <= 8192 and N <= 8192");
    if (workspace_bytes < train_gram_workspace_bytes(N, K))
        return fail(LBPF_E_INVALID, "workspace smaller than lbpf_train_gram_workspace_bytes(N, K)");
    HIP_TRY(launch_train_gram(X, labels, N, ctx->fp.dim, K, (float)C, (float)eps, max_epochs, seed,
                              alpha_io, warm, W, b, epochs_opt, workspace, (hipStream_t)stream),
            "training kernel launch");
    return LBPF_OK;
}

lbpf_status lbpf_features_plain(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                                const lbpf_box *boxes, int32_t n_boxes, float *hist,
                                uint32_t *counts_opt, void *stream) {
    if (!ctx) return fail(LBPF_E_INVALID, "ctx is NULL");
    if (n_boxes > 0 && !hist) return fail(LBPF_E_INVALID, "hist is NULL");
    lbpf_status st = resolve(ctx, images, n_images, boxes, n_boxes, ctx->h_crops);
    if (st != LBPF_OK) return st;
    if (n_boxes == 0) return LBPF_OK;
    hipStream_t s = (hipStream_t)stream;
    const size_t D = (size_t)ctx->fp.dim;
    // Every crop uses the context's median word (and, without counts_opt, its
    // counts row): calls on different streams are ordered by plain_ev so they
    // never overlap. Under graph capture the graph's own order applies.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap), "hipStreamIsCapturing");
    const bool order = cap == hipStreamCaptureStatusNone;
    if (order) HIP_TRY(hipStreamWaitEvent(s, ctx->plain_ev, 0), "hipStreamWaitEvent");
    for (int32_t i = 0; i < n_boxes; ++i) {
        uint32_t *cnt = counts_opt ? counts_opt + (size_t)i * D : ctx->d_plain_counts;
        HIP_TRY(launch_plain_features(ctx->h_crops[(size_t)i], ctx->fp, ctx->d_bins,
                                      ctx->d_plain_median, cnt, hist + (size_t)i * D, s),
                "plain feature launch");
    }
    if (order) HIP_TRY(hipEventRecord(ctx->plain_ev, s), "hipEventRecord");
    return LBPF_OK;
}

lbpf_status lbpf_score_plain(lbpf_ctx *ctx, const float *hist, int32_t N, const lbpf_weights *w,
                             float *scores_opt, int32_t *argmax_opt, void *stream) {
    if (!ctx || !w) return fail(LBPF_E_INVALID, "NULL argument");
    if (w->ctx != ctx) return fail(LBPF_E_INVALID, "weights belong to another context");
    if (N < 0) return fail(LBPF_E_INVALID, "N < 0");
    if (!scores_opt && !argmax_opt) return fail(LBPF_E_INVALID, "no output requested");
    if (N > 0 && !hist) return fail(LBPF_E_INVALID, "hist is NULL");
    if (w->prec != LBPF_FP32) return fail(LBPF_E_UNSUPPORTED, "the plain path scores in FP32 only");
    if (N == 0) return LBPF_OK;
    hipStream_t s = (hipStream_t)stream;
    // Without caller scores every row goes through the context's score
    // scratch, which lbpf_score also uses: ordered by scratch_ev like it.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap), "hipStreamIsCapturing");
    const bool order = !scores_opt && cap == hipStreamCaptureStatusNone;
    if (order) HIP_TRY(hipStreamWaitEvent(s, ctx->scratch_ev, 0), "hipStreamWaitEvent");
    for (int32_t n = 0; n < N; ++n) {
        float *srow = scores_opt ? scores_opt + (size_t)n * w->K : ctx->d_scores;
        HIP_TRY(launch_plain_score(hist + (size_t)n * w->D, w->W, w->b, w->K, w->D, srow,
                                   argmax_opt ? argmax_opt + n : nullptr, s),
                "plain score launch");
    }
    if (order) HIP_TRY(hipEventRecord(ctx->scratch_ev, s), "hipEventRecord");
    return LBPF_OK;
}

lbpf_status lbpf_debug_codes(lbpf_ctx *ctx, const lbpf_image *image, const lbpf_box *box,
                             uint8_t *grey_codes, uint8_t *depth_codes, uint8_t *mask,
                             void *stream) {
    if (!ctx || !image || !box || !grey_codes || !depth_codes || !mask)
        return fail(LBPF_E_INVALID, "NULL argument");
    lbpf_box b = *box;
    b.image = 0;
    std::vector<CropDesc> crops;
    lbpf_status st = resolve(ctx, image, 1, &b, 1, crops);
    if (st != LBPF_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int slot = ctx->ring_next;
    ctx->ring_next = (slot + 1) % kRing;
    HIP_TRY(hipEventSynchronize(ctx->ev[slot]), "hipEventSynchronize");
    std::memcpy(ctx->h_stage[slot], crops.data(), sizeof(CropDesc));
    HIP_TRY(hipMemcpyAsync(ctx->d_stage[slot], ctx->h_stage[slot], sizeof(CropDesc),
                           hipMemcpyHostToDevice, s),
            "hipMemcpyAsync");
    HIP_TRY(launch_debug_codes(ctx->d_stage[slot], ctx->fp, grey_codes, depth_codes, mask, b.w,
                               b.h, s),
            "debug kernel launch");
    HIP_TRY(hipEventRecord(ctx->ev[slot], s), "hipEventRecord");
    return LBPF_OK;
}

}  // extern "C"
