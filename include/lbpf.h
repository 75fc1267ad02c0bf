/*
 * lbpf.h -- C ABI of liblbpf.so: depth-fused LBP face features and linear-SVM
 * scoring on AMD Instinct MI355X (gfx950), after Naik & Rathna, "Robust real
 * time face recognition and tracking on GPU using fusion of RGB and depth
 * image" (arXiv 1504.01883).
 *
 * The library computes, for face boxes given in co-registered grey (u8) and
 * depth (u16, millimetres, 0 = invalid) planes:
 *   1. the lower median m of the crop's non-zero depth (the depth region of
 *      interest that the paper's fusion relies on, abstract and Sec. 1);
 *   2. for every interior pixel whose depth d satisfies d != 0 and
 *      |d - m| < depth_window_mm, the 3x3 LBP code of the grey and of the
 *      depth plane (Sec. 2.4, Eq. 2, Fig. 7; neighbour p gets weight 2^p,
 *      bit set when the neighbour is >= the centre; p0 is the top-left
 *      neighbour and p runs clockwise);
 *   3. the uniform-59 bin of each code (58 uniform patterns in increasing
 *      order, then one bin for all others) or the raw 256-bin code;
 *   4. regional histograms over a grid_x x grid_y grid whose band r covers
 *      [floor(r*n/g), floor((r+1)*n/g)) of a side of length n (Sec. 2.4,
 *      Eq. 3), concatenated as [channel][ry][rx][bin], grey first;
 *   5. the L1-normalised feature x = count / T with T = channels * n_in,
 *      each element the correctly rounded single-precision quotient (0 when
 *      T = 0);
 *   6. SVM decision values S = X W^T + b for every enrolled identity and the
 *      best identity per crop (Sec. 2.5: one hyperplane per person; ties go
 *      to the lowest identity index).
 *
 * Conventions for every call:
 *   - Pointers documented as DEVICE point to GPU memory the caller allocated
 *     (hipMalloc or a torch CUDA tensor); HOST pointers are ordinary memory.
 *     The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls taking a stream are asynchronous: they return once the work is
 *     queued. Faults during execution surface at the caller's next
 *     synchronisation of that stream.
 *   - Every argument check happens before anything is queued: on an error
 *     return nothing was written and no work was queued.
 *   - lbpf_features / lbpf_features_batch / lbpf_score never allocate device
 *     memory; all scratch is owned by the context and sized at creation.
 *   - A context is used by one host thread at a time; several contexts may
 *     coexist. Work may be queued on several streams through one context:
 *     lbpf_features stages box tables through a small ring of buffers (it
 *     waits for the oldest slot before reusing it), and lbpf_score calls that
 *     use the context's scratch (reduced precision, argmax without caller
 *     scores, or FP32 products too small to fill the GPU, whose feature
 *     dimension is split over workgroups) are ordered across streams by an
 *     event the context keeps, so they never overlap each other; the plain
 *     comparator calls (lbpf_features_plain, and lbpf_score_plain without
 *     caller scores) are ordered the same way by events of their own;
 *     everything else may overlap. Inside a captured graph that ordering is
 *     the graph's, and a graph replay must not overlap eager scoring through
 *     the same context.
 */
#ifndef LBPF_H
#define LBPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbpf_status {
    LBPF_OK = 0,
    LBPF_E_INVALID = -1,     /* bad argument: NULL pointer, box outside its image, side < 3 ... */
    LBPF_E_BUDGET = -2,      /* request larger than the context's fixed capacity or budget */
    LBPF_E_HIP = -3,         /* a HIP runtime call failed; lbpf_last_error() has the detail */
    LBPF_E_UNSUPPORTED = -4  /* valid request the library does not implement */
} lbpf_status;

typedef enum lbpf_precision {
    LBPF_FP32 = 0,       /* FP32 operands, FP32 MFMA accumulation */
    LBPF_BF16 = 1,       /* BF16 operands (round to nearest even), FP32 accumulation */
    LBPF_FP16 = 2,       /* FP16 operands with per-row power-of-two scales */
    LBPF_FP8_E4M3 = 3,   /* OCP FP8 e4m3 operands with per-row amax/448 scales
                            (encoded as x * (448/amax) in FP32, RNE, saturating) */
    LBPF_F16X3 = 4       /* FP32 operands split into FP16 high and low parts (per-row
                            power-of-two scales); scores = hi hi + hi lo + lo hi on FP16
                            matrix cores with FP32 accumulation: FP32-level accuracy */
} lbpf_precision;

enum { LBPF_MAP_U59 = 0, LBPF_MAP_FULL256 = 1 };
enum { LBPF_MOD_BOTH = 0, LBPF_MOD_GREY = 1, LBPF_MOD_DEPTH = 2 };

/* One co-registered grey + depth image. grey and depth are DEVICE pointers to
 * row-major planes; pitches are in elements (bytes for grey, u16 for depth).
 * grey may be NULL only when the context's modality is LBPF_MOD_DEPTH. */
typedef struct lbpf_image {
    const uint8_t *grey;
    const uint16_t *depth;
    int32_t width, height, grey_pitch, depth_pitch;
} lbpf_image;

/* A face box in image `image`: the crop is columns [x, x+w) and rows [y, y+h)
 * of both planes (the paper maps the detected face to a rectangle of the
 * depth frame, Sec. 2.1). Requires 3 <= w, h <= LBPF_MAX_SIDE and the box
 * inside its image. */
typedef struct lbpf_box {
    int32_t image, x, y, w, h;
} lbpf_box;

#define LBPF_MAX_SIDE 1024

/* Feature configuration. grid_x * grid_y <= 64 and each >= 1; mapping is
 * LBPF_MAP_U59 (59 bins) or LBPF_MAP_FULL256 (256 bins, the paper's "0 to
 * 255" histogram, Sec. 3); depth_window_mm > 0 enables the depth mask with
 * that half-width, <= 0 counts every interior pixel; modality selects the
 * channels (Table 1 compares grey-only and depth-only inputs). */
typedef struct lbpf_feature_cfg {
    int32_t grid_x, grid_y;
    int32_t mapping;
    int32_t depth_window_mm;
    int32_t modality;
} lbpf_feature_cfg;

typedef struct lbpf_ctx lbpf_ctx;         /* workspace, pinned staging ring, lookup tables */
typedef struct lbpf_weights lbpf_weights; /* device-resident W, b and any quantised copy */
typedef struct lbpf_batch lbpf_batch;     /* device-resident, validated box table */

/* Library version string, e.g. "lbpf 0.1.0 gfx950". Never NULL. */
const char *lbpf_version(void);

/* Create a context on the current HIP device. cfg NULL selects the default
 * {8, 8, LBPF_MAP_U59, 150, LBPF_MOD_BOTH}. hbm_budget_bytes bounds the
 * device memory the context and its batches may hold (0 = no bound).
 * Allocates the context's fixed workspace (box staging for up to
 * LBPF_MAX_BOXES_PER_CALL boxes and the scoring scratch).
 * Returns LBPF_E_INVALID for a bad cfg, LBPF_E_BUDGET when the workspace alone
 * exceeds the budget, LBPF_E_HIP when an allocation fails. */
#define LBPF_MAX_BOXES_PER_CALL 65536
lbpf_status lbpf_create(lbpf_ctx **out, const lbpf_feature_cfg *cfg, size_t hbm_budget_bytes);

/* Release the context and its workspace (synchronises the device first).
 * NULL is allowed. Batches and weights created from it must be destroyed
 * before it. */
void lbpf_destroy(lbpf_ctx *ctx);

/* Feature dimension D = channels * grid_x * grid_y * bins (7552 for the
 * default configuration), or -1 for a NULL context. */
int32_t lbpf_feature_dim(const lbpf_ctx *ctx);

/* Features of n_boxes boxes. images (n_images entries) and boxes (n_boxes
 * entries) are HOST arrays; the planes they point to are DEVICE memory.
 * hist: DEVICE [n_boxes][D] FP32, L1-normalised (steps 1-5 above).
 * counts_opt: DEVICE [n_boxes][D] u32 raw histogram counts, or NULL.
 * The box table is validated on the host, copied through pinned memory and
 * the kernels are queued on `stream`. n_boxes = 0 is a no-op.
 * Errors: LBPF_E_INVALID (NULL pointers, a box outside its image or with a
 * side < 3 or > LBPF_MAX_SIDE, a NULL grey plane when grey is used),
 * LBPF_E_BUDGET (n_boxes > LBPF_MAX_BOXES_PER_CALL), LBPF_E_HIP. */
lbpf_status lbpf_features(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                          const lbpf_box *boxes, int32_t n_boxes, float *hist,
                          uint32_t *counts_opt, void *stream);

/* Validate a box table once and keep it in device memory, for repeated
 * launches over inputs that stay resident (benchmarks, hipGraph capture).
 * HOST arrays in, synchronous. The batch records the planes' DEVICE pointers:
 * the caller keeps them alive while the batch is used. Same errors as
 * lbpf_features, plus LBPF_E_BUDGET when the context's budget is exceeded. */
lbpf_status lbpf_batch_create(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                              const lbpf_box *boxes, int32_t n_boxes, lbpf_batch **out);
void lbpf_batch_destroy(lbpf_batch *batch);
int32_t lbpf_batch_size(const lbpf_batch *batch);

/* Features of a prepared batch: same outputs as lbpf_features, no host
 * staging and no allocation. hist and counts_opt are DEVICE [n][D]. */
lbpf_status lbpf_features_batch(lbpf_ctx *ctx, const lbpf_batch *batch, float *hist,
                                uint32_t *counts_opt, void *stream);

/* Sampling frame of one plane, after Eq. 1 (Sec. 2.1: p' = x u + y v + t, the
 * affine map that turns the mapped face region into a rectangle), in 16.16
 * fixed point: crop pixel (x, y) reads the plane pixel
 *     sx = floor((ux*x + vx*y + tx) / 65536),  sy = floor((uy*x + vy*y + ty) / 65536)
 * evaluated exactly in 64-bit integers (nearest sample, no interpolation).
 * The identity frame of box (x0, y0) is {65536, 0, 0, 65536, x0*65536,
 * y0*65536}; Sec. 3's resize of a w x h box to 200 x 200 is ux = w*65536/200,
 * vy = h*65536/200 with t offset by half a step. */
typedef struct lbpf_frame {
    int32_t ux, uy, vx, vy, tx, ty;
} lbpf_frame;

/* A warped face crop of w x h pixels (3 <= w, h <= LBPF_MAX_SIDE) sampled from
 * image `image`: grey through frame `grey` (ignored when the modality has no
 * grey channel), depth through frame `depth`. Every sample must lie inside
 * the image (checked on the four corners, which bound an affine map). */
typedef struct lbpf_warp_box {
    int32_t image, w, h;
    lbpf_frame grey, depth;
} lbpf_warp_box;

/* Device workspace bytes one warped w x h crop occupies (a multiple of 256);
 * 0 for sides outside 3..LBPF_MAX_SIDE. */
size_t lbpf_warp_crop_bytes(int32_t w, int32_t h);

/* Features of warped crops: the same outputs as lbpf_features for the crops
 * the frames sample (steps 1-5 run on the sampled w x h crop). images and
 * boxes are HOST arrays (planes DEVICE memory); hist / counts_opt are DEVICE
 * [n_boxes][D]. workspace is caller-owned DEVICE memory (256-byte aligned)
 * of workspace_bytes, at least lbpf_warp_crop_bytes of the largest crop: the
 * sampled crops are staged there and the call works through the boxes in
 * order, in groups whose crops fit it together (one sampling kernel and one
 * feature kernel per group, all on `stream`). The workspace must not be used
 * by other work until the call's work on `stream` has finished.
 * Errors: LBPF_E_INVALID (NULL pointers, bad sides, a sample outside the
 * image, misaligned or too small workspace), LBPF_E_BUDGET (more than
 * LBPF_MAX_BOXES_PER_CALL boxes), LBPF_E_HIP. */
lbpf_status lbpf_features_warped(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                                 const lbpf_warp_box *boxes, int32_t n_boxes, void *workspace,
                                 size_t workspace_bytes, float *hist, uint32_t *counts_opt,
                                 void *stream);

/* On-device training of the per-person hyperplanes (Sec. 2.5: max margin,
 * each person against all others; the paper trains on the CPU, Sec. 3).
 * For every class k in 0..K-1 (y_i = +1 where labels[i] == k, else -1):
 * L2-regularised hinge loss with cost C, the bias as an extra constant
 * feature 1, the features scaled by sigma = 1 / (lower median of the row
 * norms; 1 if that is 0), solved in FP64 by dual coordinate descent (Hsieh
 * et al. 2008). Epoch e of class k visits the samples in the Fisher-Yates
 * order (i = N-1 down to 1 swaps i with r mod (i+1)) drawn from the
 * splitmix64 stream seeded with seed ^ (k+1) * 0x5851F42D4C957F2D, draws
 * e(N-1) onwards; it stops after the first epoch whose largest projected
 * gradient is below eps, or after max_epochs.
 * X: DEVICE [N][D] FP32 features (D = lbpf_feature_dim, at most 8192);
 * labels: DEVICE [N] int32; 1 <= N <= 12288, K >= 1, C > 0, eps > 0,
 * max_epochs >= 1.
 * Outputs (DEVICE): W [K][D] and b [K] FP32 (sigma w and the bias weight,
 * rounded to nearest: ready for lbpf_weights_create), W64_opt / b64_opt the
 * same in FP64 (or NULL), epochs_opt [K] the epochs each class ran (or NULL).
 * alpha_io: DEVICE [K][N] FP64 dual variables, or NULL; with warm != 0 they
 * are the starting point (w is rebuilt from them: the incremental update
 * after new faces are labelled, new rows starting at 0); the final values are
 * written back whenever alpha_io is given.
 * workspace: DEVICE, lbpf_train_workspace_bytes(N) bytes, 8-byte aligned.
 * Errors: LBPF_E_INVALID, LBPF_E_UNSUPPORTED (D or N above the limits),
 * LBPF_E_HIP. */
size_t lbpf_train_workspace_bytes(int32_t N);
lbpf_status lbpf_train_ovr(lbpf_ctx *ctx, const float *X, const int32_t *labels, int32_t N,
                           int32_t K, double C, double eps, int32_t max_epochs, uint64_t seed,
                           double *alpha_io, int32_t warm, float *W, float *b, double *W64_opt,
                           double *b64_opt, int32_t *epochs_opt, void *workspace,
                           size_t workspace_bytes, void *stream);

/* The same training (Sec. 2.5: one max-margin hyperplane per person against
 * all others) on the Gram matrix, in FP32 throughout: G = X X^T of the
 * unscaled features on the FP32 matrix cores (the scoring GEMM with X as both
 * operands), sigma = 1 / (lower median of sqrt(G_ii); 1 if that is 0), then
 * per class the dual coordinate descent of lbpf_train_ovr (same problem,
 * same seeded sample order, same stopping rule) with the margins
 * y_i (sigma^2 sum_j alpha_j y_j G_ij + sum_j alpha_j y_j) kept for every
 * sample, so that the samples whose projected gradient is zero (which change
 * nothing) are passed over 64 at a time; W_k = sigma^2 sum_i alpha_ki y_ki x_i
 * and b_k = sum_i alpha_ki y_ki. Arguments as for lbpf_train_ovr, except:
 * 1 <= N <= 8192; alpha_io: DEVICE [K][N] FP32 (or NULL; warm != 0 needs it);
 * workspace: DEVICE, lbpf_train_gram_workspace_bytes(N, K) bytes (the N x N
 * Gram matrix among them), 16-byte aligned. Results agree with the FP64
 * trainer to FP32 accuracy, not bit for bit.
 * Errors: LBPF_E_INVALID, LBPF_E_UNSUPPORTED (D or N above the limits),
 * LBPF_E_HIP. */
size_t lbpf_train_gram_workspace_bytes(int32_t N, int32_t K);
lbpf_status lbpf_train_ovr_gram(lbpf_ctx *ctx, const float *X, const int32_t *labels, int32_t N,
                                int32_t K, double C, double eps, int32_t max_epochs,
                                uint64_t seed, float *alpha_io, int32_t warm, float *W, float *b,
                                int32_t *epochs_opt, void *workspace, size_t workspace_bytes,
                                void *stream);

/* Nearest-centre tracking (Sec. 2.3, Fig. 4): each face of the previous frame
 * (a track) is followed by the detection of the same stream whose box centre
 * is nearest to its previous centre. prev / cur: HOST int32 [P][4] / [C][4]
 * boxes (x, y, w, h), every value within +-32767 and w, h >= 0; prev_stream /
 * cur_stream: HOST int32 [P] / [C] stream (camera) ids. Distances are
 * squared Euclidean distances of the box centres, computed exactly;
 * gate2 > 0 ignores boxes farther than sqrt(gate2) pixels (<= 0: no gate).
 * Outputs (DEVICE int32): match [P] = the nearest current box for each track
 * (lowest index on ties) or -1; owner [C] = among the tracks matched to a box
 * the nearest one (lowest track index on ties), or -1 for a new face.
 * P, C <= 16384 (0 allowed). Errors: LBPF_E_INVALID, LBPF_E_BUDGET (sizes),
 * LBPF_E_HIP. */
lbpf_status lbpf_track(lbpf_ctx *ctx, const int32_t *prev, const int32_t *prev_stream,
                       int32_t P, const int32_t *cur, const int32_t *cur_stream, int32_t C,
                       int64_t gate2, int32_t *match, int32_t *owner, void *stream);

/* Launch shape of the fused feature kernel for one batch. persistent = 0:
 * one workgroup per crop; 1: wg_per_cu workgroups per compute unit take
 * crops from a device work queue (sorted = 1: largest crop first) until it is
 * empty. row_prefetch (2, 4 or 8) is how many rows ahead each lane loads. The
 * outputs do not depend on the launch shape. */
typedef struct lbpf_launch_cfg {
    int32_t persistent;
    int32_t wg_per_cu;
    int32_t row_prefetch;
    int32_t sorted;
} lbpf_launch_cfg;

/* Set / read a batch's launch shape (default {0, 4, 4, 1}). LBPF_E_INVALID
 * for values outside the ranges above. */
lbpf_status lbpf_batch_set_launch(lbpf_batch *batch, const lbpf_launch_cfg *cfg);
lbpf_status lbpf_batch_get_launch(const lbpf_batch *batch, lbpf_launch_cfg *cfg);

/* Autotuner: time every candidate launch shape on this batch (two rounds
 * over the candidates, each timing one warm-up launch then reps launches
 * with HIP events on `stream`; synchronous), keep the fastest average in
 * the batch and report it (best_out, best_us_out may be NULL). hist is a
 * DEVICE [n][D] FP32 scratch the runs write into. */
lbpf_status lbpf_tune_batch(lbpf_ctx *ctx, lbpf_batch *batch, float *hist, int32_t reps,
                            lbpf_launch_cfg *best_out, float *best_us_out, void *stream);

/* Capture features (+ optionally scores/argmax) of a batch into a HIP graph
 * and instantiate it; replays recompute everything from the batch's current
 * input planes. weights NULL captures the features only. hist, scores_opt,
 * argmax_opt are DEVICE outputs as for lbpf_features_batch / lbpf_score; the
 * caller keeps them alive. The graph holds no memset nodes: the persistent
 * kernel's work queue resets itself, so replays need nothing in between. */
typedef struct lbpf_graph lbpf_graph;
lbpf_status lbpf_graph_create(lbpf_ctx *ctx, const lbpf_batch *batch,
                              const lbpf_weights *weights, float *hist, float *scores_opt,
                              int32_t *argmax_opt, lbpf_graph **out);
lbpf_status lbpf_graph_launch(lbpf_graph *graph, void *stream);
void lbpf_graph_destroy(lbpf_graph *graph);

/* A serving step captured once as a HIP graph and replayed per batch (Sec. 3:
 * each frame's faces are detected, their features extracted and classified;
 * here for a batch of frames from many cameras at once). One replay copies
 * the batch's box table from the pipeline's pinned staging to the device,
 * runs the fused feature kernel (persistent, largest crop first), the scoring
 * of weights' precision (quantisation, GEMM, argmax) and copies the
 * identities back to host memory; every kernel reads the batch's box count
 * from device memory, so one graph serves batches of 0 .. max_boxes boxes.
 * Outputs are caller-owned: hist DEVICE [max_boxes][D] FP32, scores_opt
 * DEVICE [max_boxes][K] FP32 or NULL (then the pipeline keeps its own),
 * argmax DEVICE [max_boxes] int32, argmax_host_opt HOST [max_boxes] int32 in
 * pinned memory (hipHostMalloc or a pinned torch tensor) or NULL. Rows past
 * a batch's size are left unspecified. Requires the default feature
 * configuration (uniform-59, both channels, window 1..255) and, for FP32
 * weights, D % 32 == 0 and a 16-byte aligned hist. Allocates its staging and
 * scratch (charged to the context's budget). The weights must outlive the
 * pipeline. Errors: LBPF_E_INVALID, LBPF_E_BUDGET (max_boxes outside
 * 1..LBPF_MAX_BOXES_PER_CALL, budget), LBPF_E_UNSUPPORTED, LBPF_E_HIP. */
typedef struct lbpf_pipeline lbpf_pipeline;
lbpf_status lbpf_pipeline_create(lbpf_ctx *ctx, const lbpf_weights *weights, int32_t max_boxes,
                                 float *hist, float *scores_opt, int32_t *argmax,
                                 int32_t *argmax_host_opt, lbpf_pipeline **out);

/* Queue one batch on `stream`: the boxes (HOST array, validated like
 * lbpf_features, then written into the pinned staging in largest-first
 * order) over the images (HOST array of DEVICE planes, which must stay
 * valid until the replay has run), then one graph replay. Results
 * (hist[0 .. n_boxes), scores, argmax, argmax_host) are complete once
 * `stream` has passed this call. Launches on one pipeline must not overlap:
 * a launch first waits (on the host) for the previous one's replay to
 * finish. Errors: LBPF_E_INVALID (as lbpf_features), LBPF_E_BUDGET (more
 * than max_boxes boxes), LBPF_E_HIP. */
lbpf_status lbpf_pipeline_launch(lbpf_pipeline *pipeline, const lbpf_image *images,
                                 int32_t n_images, const lbpf_box *boxes, int32_t n_boxes,
                                 void *stream);
int32_t lbpf_pipeline_max_boxes(const lbpf_pipeline *pipeline);
void lbpf_pipeline_destroy(lbpf_pipeline *pipeline);

/* Native serving loop (Sec. 3's per-frame loop of detection, mapping,
 * features and classification, here for frames from many cameras at once):
 * a library thread admits frames, uploads them and runs batches, so that no
 * per-frame step needs the caller's thread.
 *
 * Every frame is frame_w x frame_h, a grey u8 plane and a depth u16 plane
 * with packed rows. The server owns n_slots device frame slots. Submitted
 * requests are released at their arrival time on the server clock, then
 * admitted first come, first served into a free slot while the bytes of all
 * admitted frames (3 frame_w frame_h each) stay within budget_bytes; a
 * request that does not fit waits, and nothing behind it overtakes it.
 * Admitted frames are copied host -> device on the server's copy streams
 * (only the rows their boxes span).
 * Whenever one of the `inflight` batch sets is free, up to max_batch_frames
 * admitted frames form a batch: one captured-pipeline replay
 * (lbpf_pipeline_*: box table, features, scores of the weights' precision,
 * argmax, identities copied to pinned host memory) on the set's own stream,
 * after the copies of its frames. Frames arriving while batches run join the
 * next batch (continuous batching). When the server thread sees a batch's
 * completion it frees the slots and records each request's result and
 * completion time. Requirements as for lbpf_pipeline_create. */
typedef struct lbpf_server lbpf_server;

typedef struct lbpf_server_cfg {
    int32_t frame_w, frame_h;     /* 3 .. 4096 each */
    int32_t n_slots;              /* device frame slots, 1 .. 4096 */
    int64_t budget_bytes;         /* >= one frame's 3 frame_w frame_h bytes */
    int32_t max_batch_frames;     /* 1 .. n_slots */
    int32_t max_boxes_per_frame;  /* 1 .. 64 */
    int32_t inflight;             /* batch sets (streams, pipelines), 1 .. 8 */
    int32_t copy_streams;         /* host -> device upload streams, 1 .. 8; frames go to
                                     them in turn (several copy engines at once) */
} lbpf_server_cfg;

/* One frame to serve. t_arrival: seconds on the server clock
 * (lbpf_server_clock); arrivals must not decrease across submissions.
 * grey, depth: HOST [frame_h][frame_w] planes, read by asynchronous copies,
 * so they should be pinned (hipHostMalloc, or pinned torch tensors); they
 * must stay valid and unchanged until the request's result has been polled.
 * boxes: HOST [n_boxes][4] int32 (x, y, w, h), each 3 <= w, h and inside the
 * frame; copied at submission. */
typedef struct lbpf_request {
    int64_t id;
    double t_arrival;
    const uint8_t *grey;
    const uint16_t *depth;
    const int32_t *boxes;
    int32_t n_boxes;
} lbpf_request;

/* A served frame: its identities (argmax over the enrolled identities, one
 * per box in submission order) are argmax[argmax_offset .. + n_boxes) of
 * the lbpf_server_poll call that returned it. t_done: server-clock time at
 * which the server thread saw the batch's completion. */
typedef struct lbpf_result {
    int64_t id;
    double t_arrival, t_done;
    int32_t n_boxes;
    int32_t argmax_offset;
} lbpf_result;

typedef struct lbpf_server_stats {
    int64_t batches, frames, boxes;
    int64_t deferrals;         /* loop iterations in which the budget or slots held a request back */
    int64_t loop_iterations;
    double busy_seconds;       /* server thread time outside idle waits */
    double seconds;            /* server clock now */
} lbpf_server_stats;

/* Allocates the frame slots, per batch set a stream, a pipeline and its
 * hist / argmax buffers (charged to the context's budget), and starts the
 * server thread. ctx and weights must outlive the server; while it runs,
 * other threads may use the context for calls that neither create nor
 * destroy objects. Errors: LBPF_E_INVALID (configuration out of range),
 * LBPF_E_BUDGET, LBPF_E_UNSUPPORTED (as lbpf_pipeline_create), LBPF_E_HIP. */
lbpf_status lbpf_server_create(lbpf_ctx *ctx, const lbpf_weights *weights,
                               const lbpf_server_cfg *cfg, lbpf_server **out);

/* Seconds since the server was created (steady clock). */
double lbpf_server_clock(const lbpf_server *server);

/* Queue n requests (HOST array). Validates all of them first: on
 * LBPF_E_INVALID (NULL plane, box count or box out of range, an arrival
 * earlier than one already submitted) none is queued. Thread-safe against
 * lbpf_server_poll. Also returns the server thread's error (LBPF_E_HIP) once
 * it has stopped on one. */
lbpf_status lbpf_server_submit(lbpf_server *server, const lbpf_request *requests, int32_t n);

/* Move up to max_results finished requests (oldest first) into results
 * (HOST) and their identities into argmax (HOST, max_argmax entries); stops
 * early when the next request's boxes would not fit. *n_out: results
 * written. Never blocks on the GPU. Errors: LBPF_E_INVALID (NULL, negative
 * sizes), LBPF_E_HIP (the server thread stopped on a HIP error; results
 * finished before it are still returned). */
lbpf_status lbpf_server_poll(lbpf_server *server, lbpf_result *results, int32_t max_results,
                             int32_t *argmax, int32_t max_argmax, int32_t *n_out);

lbpf_status lbpf_server_get_stats(const lbpf_server *server, lbpf_server_stats *out);

/* Stops the server: requests not yet in a batch are dropped, batches on the
 * device are waited for; then frees everything the server allocated. */
void lbpf_server_destroy(lbpf_server *server);

/* Enrol K identities: W DEVICE [K][D] FP32 row-major, b DEVICE [K] FP32.
 * The library copies them (and, for BF16/FP16/FP8, quantises them) into a
 * weights object it owns; the caller's buffers may be freed once `stream`
 * has finished. Synchronous with respect to the host. Errors: LBPF_E_INVALID
 * (K < 1, NULL), LBPF_E_UNSUPPORTED (precision not built), LBPF_E_BUDGET,
 * LBPF_E_HIP. */
lbpf_status lbpf_weights_create(lbpf_ctx *ctx, const float *W, const float *b, int32_t K,
                                lbpf_precision precision, lbpf_weights **out, void *stream);
void lbpf_weights_destroy(lbpf_weights *weights);
int32_t lbpf_weights_count(const lbpf_weights *weights);

/* Score N feature rows against every enrolled identity (step 6).
 * hist: DEVICE [N][D] FP32. scores_opt: DEVICE [N][K] FP32 or NULL.
 * argmax_opt: DEVICE [N] int32 or NULL (not both NULL). N = 0 is a no-op.
 * In FP32 the scores are accumulated in FP32 by MFMA (when the product has
 * too few 128 x 128 output tiles to fill the GPU, the feature dimension is
 * split into up to 4 equal ranges whose partial sums are added in range
 * order, so results are deterministic); in the reduced precisions the
 * operands are converted as documented for lbpf_precision and the products
 * accumulated in FP32. Errors: LBPF_E_INVALID, LBPF_E_HIP. */
lbpf_status lbpf_score(lbpf_ctx *ctx, const float *hist, int32_t N, const lbpf_weights *weights,
                       float *scores_opt, int32_t *argmax_opt, void *stream);

/* The plain unbatched FP32 GPU path, kept as the comparator of the fused
 * path: the same outputs, computed the straightforward way one crop at a
 * time (Sec. 3 extracts features face by face): per crop a median kernel, a
 * one-thread-per-pixel LBP kernel incrementing the crop's histogram with
 * global-memory atomics, and a normalisation kernel. Same arguments, results
 * (bit-exact) and errors as lbpf_features; counts_opt NULL uses a context
 * scratch row. Crops run in order on `stream`; every crop uses the context's
 * median scratch, so calls queued on different streams run one after the
 * other (ordered by an event the context keeps), never overlapped. */
lbpf_status lbpf_features_plain(lbpf_ctx *ctx, const lbpf_image *images, int32_t n_images,
                                const lbpf_box *boxes, int32_t n_boxes, float *hist,
                                uint32_t *counts_opt, void *stream);

/* Plain scoring: one GEMV kernel (one thread per identity, FP32 fused
 * multiply-adds) and one argmax kernel per feature row. Same arguments as
 * lbpf_score; FP32 weights only (LBPF_E_UNSUPPORTED otherwise). */
lbpf_status lbpf_score_plain(lbpf_ctx *ctx, const float *hist, int32_t N,
                             const lbpf_weights *weights, float *scores_opt,
                             int32_t *argmax_opt, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. FP32 scoring
 * (step 6) as lbpf_score with FP32 weights, without a context: hist DEVICE
 * [N][D] FP32, W DEVICE [K][D] FP32 row-major, b DEVICE [K] FP32 (the caller
 * owns all three), scores_opt DEVICE [N][K] FP32 or NULL, argmax_opt DEVICE
 * [N] int32 or NULL (not both NULL). The same kernels and results as
 * lbpf_score. The call allocates nothing: the scratch its kernels need (each
 * pass's scores when no score buffer is given, the partial tiles when the
 * feature dimension is split over workgroups) is a static device array of
 * LBPF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; argmax-only calls score in passes of
 * (LBPF_NOALLOC_SCRATCH_BYTES / 8) / K rows. Every call on one GPU shares
 * that GPU's array and nothing orders them: calls that overlap on one GPU
 * (other streams, other host threads) race and give wrong results.
 * N = 0 is a no-op. Errors: LBPF_E_INVALID (NULL pointers, N < 0, K < 1,
 * D < 1, no output), LBPF_E_BUDGET (argmax only with K above
 * LBPF_NOALLOC_SCRATCH_BYTES / 8), LBPF_E_HIP. */
#define LBPF_NOALLOC_SCRATCH_BYTES (16u << 20)
lbpf_status lbpf_score_noalloc(const float *hist, int32_t N, const float *W, const float *b,
                               int32_t K, int32_t D, float *scores_opt, int32_t *argmax_opt,
                               void *stream);

/* Test hook: per-pixel codes and mask of ONE box, for bit-exact checks.
 * image/box are HOST structs; grey_codes, depth_codes, mask are DEVICE
 * [box->h][box->w] u8 arrays. Interior pixels receive their grey code, depth
 * code and mask bit (1 = counted); border entries are written as 0. */
lbpf_status lbpf_debug_codes(lbpf_ctx *ctx, const lbpf_image *image, const lbpf_box *box,
                             uint8_t *grey_codes, uint8_t *depth_codes, uint8_t *mask,
                             void *stream);

/* Human-readable name of a status code. Never NULL. */
const char *lbpf_status_string(lbpf_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *lbpf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBPF_H */
