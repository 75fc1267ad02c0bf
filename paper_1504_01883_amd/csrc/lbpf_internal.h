// Internal declarations shared by the HIP sources of liblbpf.so.
// Nothing here is part of the public ABI (include/lbpf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbpf.h"

namespace lbpf {

// One face crop, resolved on the host from (image, box): plane pointers at
// the crop origin, pitches in elements, size, flags. 32 bytes, read once per
// workgroup.
struct CropDesc {
    const uint8_t *grey;
    const uint16_t *depth;
    int32_t grey_pitch, depth_pitch;
    int16_t w, h;
    uint32_t flags;
};
// Every row of the crop may be read up to kOverRead elements past its right
// edge in both planes without leaving the image (the bytes read there are
// never used).
constexpr uint32_t kCropOverReadOk = 1u;
constexpr int kOverRead = 7;
static_assert(sizeof(CropDesc) == 32, "CropDesc layout");

// Record `msg` as the calling thread's lbpf_last_error() and return s.
lbpf_status set_last_error(lbpf_status s, const std::string &msg);

// Feature geometry shared by every kernel launch of a context.
struct FeatParams {
    int32_t grid_x, grid_y;
    int32_t nbins;        // 59 or 256
    int32_t window;       // depth half-width in mm; <= 0 disables the mask
    int32_t use_grey, use_depth;
    int32_t nch;          // use_grey + use_depth
    int32_t dim;          // nch * grid_x * grid_y * nbins
};

// Code -> bin tables, built on the host by construction (tables.cpp).
void build_uniform59(uint8_t out[256]);
void build_comparison_lut(const uint8_t bin[256], uint8_t below[256]);
bool fast_path_ok(const FeatParams &fp);

// Launch shape of the fast feature kernel (chosen per batch by the tuner).
struct LaunchCfg {
    int32_t persistent = 0;    // 0: one workgroup per crop; 1: persistent work queue
    int32_t wg_per_cu = 4;     // persistent grid = wg_per_cu * CUs
    int32_t row_prefetch = 4;  // rows loaded ahead by each lane (2, 4 or 8)
    int32_t sorted = 1;        // persistent: take crops largest first
};

// Kernel launchers (features.hip). All return hipSuccess or the launch error.
// order / queue may be null (then the launch is one workgroup per crop).
hipError_t launch_features(const CropDesc *crops, int32_t n, const FeatParams &fp,
                           const uint8_t *d_tables, float *hist, uint32_t *counts,
                           hipStream_t s, const LaunchCfg &lc = LaunchCfg(),
                           const int32_t *order = nullptr, uint32_t *queue = nullptr,
                           int32_t num_cus = 256, const int32_t *n_dev = nullptr);
hipError_t launch_debug_codes(const CropDesc *crop, const FeatParams &fp, uint8_t *gcodes,
                              uint8_t *dcodes, uint8_t *mask, int32_t w, int32_t h,
                              hipStream_t s);

// The plain unbatched comparator (plain.hip): one crop / one row per call.
hipError_t launch_plain_features(const CropDesc &c, const FeatParams &fp, const uint8_t *bins,
                                 int32_t *median_scratch, uint32_t *counts, float *row,
                                 hipStream_t s);
hipError_t launch_plain_score(const float *x, const float *W, const float *b, int32_t K,
                              int32_t D, float *scores, int32_t *argmax, hipStream_t s);

// Reduced-precision scoring (score_lp.hip). Quantised weight rows have a
// pitch of lp_pitch(D, mode) bytes, feature rows lp_pitch_features(D, mode)
// (multiples of 128, zero padded; they differ for the split FP16 mode, whose
// segments are lp_seg(D) bytes).
int32_t lp_seg(int32_t D);
int32_t lp_pitch(int32_t D, int32_t mode);
int32_t lp_pitch_features(int32_t D, int32_t mode);
// n_dev (launchers below too): when not null, the kernels read the row count
// from this device word (at most the host count, which sizes the grid), so a
// captured graph serves batches of any size up to it.
// weights: quantise weight rows (split FP16: three segments) rather than
// feature rows.
hipError_t launch_quant_rows(const float *X, int32_t rows, int32_t D, int32_t mode, uint8_t *out,
                             float *scales, hipStream_t s, const int32_t *n_dev = nullptr,
                             bool weights = false);
// S: [N][K] scores, or null for argmax only; argmax: [N] or null. scratch
// (scratch_elems floats) holds the per-tile argmax pairs, or the scores when
// S is null and the pairs do not fit; it must hold N * K floats when S is
// null and 2 N ceil(K / 256) does not fit.
hipError_t launch_score_lp(const uint8_t *Xq, const float *sx, int32_t N, const uint8_t *Wq,
                           const float *sw, const float *b, int32_t K, int32_t D, int32_t mode,
                           float *S, int32_t *argmax, float *scratch, size_t scratch_elems,
                           hipStream_t s, const int32_t *n_dev = nullptr);

// Warped crops (warp.hip): each crop is sampled from its planes through two
// 16.16 fixed-point affine frames into a staging crop of pitch w, which the
// feature kernels then read as an ordinary image. 104 bytes.
struct WarpDesc {
    const uint8_t *g_src;   // grey plane at image pixel (0, 0); null if unused
    const uint16_t *d_src;  // depth plane at image pixel (0, 0)
    uint8_t *g_dst;         // staging grey crop, w * h bytes, pitch w
    uint16_t *d_dst;        // staging depth crop, w * h u16, pitch w
    int32_t g_pitch, d_pitch;
    int32_t src_w, src_h;   // plane size (samples are clamped into it)
    int32_t w, h;
    int32_t gf[6], df[6];   // frames (ux, uy, vx, vy, tx, ty)
};
static_assert(sizeof(WarpDesc) == 104, "WarpDesc layout");
hipError_t launch_warp(const WarpDesc *d, int32_t n, hipStream_t s);

// SVM training (train.hip): one-vs-rest dual coordinate descent in FP64, one
// workgroup per class. D <= kTrainMaxD, 1 <= N <= kTrainMaxN (alpha and the
// epoch's order live in LDS). workspace: train_workspace_bytes(N) bytes.
constexpr int32_t kTrainMaxD = 8192;
constexpr int32_t kTrainMaxN = 12288;
size_t train_workspace_bytes(int32_t N);
hipError_t launch_train(const float *X, const int32_t *labels, int32_t N, int32_t D, int32_t K,
                        double C, double eps, int32_t max_epochs, uint64_t seed, double *alpha,
                        int32_t warm, float *W, float *b, double *W64, double *b64,
                        int32_t *epochs, void *workspace, hipStream_t s);

// Nearest-centre tracking (track.hip). Boxes are int32 (x, y, w, h) with
// |coordinates| <= kTrackMaxCoord, so doubled-centre distances stay below
// 2^37 and (distance << 24) | track fits 64 bits; P <= kTrackMaxBoxes.
// keys: C u64 of scratch.
constexpr int32_t kTrackMaxCoord = 32767;
constexpr int32_t kTrackMaxBoxes = 16384;
hipError_t launch_track(const int32_t *prev, const int32_t *ps, int32_t P, const int32_t *cur,
                        const int32_t *cs, int32_t C, int64_t gate2, int32_t *match,
                        int32_t *owner, uint64_t *keys, hipStream_t s);

// Scoring (score.hip).
// FP32 scores. With D a multiple of 32 * splits and 16-byte aligned
// operands the 128 x 128-tile kernel runs over `splits` ranges of D (partials
// in part[splits][N][K], summed with the argmax by a second kernel); otherwise the 64 x 64-tile
// kernels run. splits: from score_f32_splits (1 when the tiles alone fill the
// GPU); 0 selects the 64 x 64-tile kernels.
int32_t score_f32_splits(int32_t N, int32_t K, int32_t D, int32_t num_cus, size_t part_elems);
// S is always written; argmax (may be null) gets each row's best identity.
hipError_t launch_score_f32(const float *X, int32_t N, const float *W, const float *b,
                            int32_t K, int32_t D, float *S, int32_t *argmax, hipStream_t s,
                            int32_t splits = 0, float *part = nullptr,
                            const int32_t *n_dev = nullptr);
hipError_t launch_argmax(const float *S, int32_t N, int32_t K, int32_t *argmax, hipStream_t s,
                         const int32_t *n_dev = nullptr);

}  // namespace lbpf
