// Fused depth-masked LBP + regional histogram + L1 normalisation, gfx950.
//
// One workgroup (4 wave64) per face crop; every step runs inside one launch:
//   1. exact lower median m of the crop's non-zero depth (the depth region of
//      interest of the paper's fusion);
//   2. for every interior pixel whose depth d satisfies d != 0 and
//      |d - m| < window, the 3x3 LBP code of the grey and of the depth plane
//      (Sec. 2.4, Eq. 2: neighbour p has weight 2^p and its bit is set when it
//      is >= the centre; p0 = top-left neighbour, then clockwise);
//   3. code -> uniform-59 bin through a 256-entry LDS table;
//   4. increments of the regional histograms (Eq. 3) held in LDS;
//   5. the row written once to HBM as count / T, T = channels * n_in, each
//      quotient the correctly rounded IEEE single division (and optionally the
//      raw counts).
//
// Kernels:
//   k_features_fast       -- the default configuration (uniform-59 bins, both
//                            channels, window 1..255 mm), one workgroup per
//                            crop. Crops up to 256 px wide take the lane path
//                            below; wider crops (and crops whose median lies
//                            within the window of 0) the per-pixel loop,
//                            inside the same launch.
//   k_features_persistent -- the same per crop, a fixed grid taking crops
//                            from a self-resetting work queue (ragged batches).
//   k_features_generic    -- every other configuration (256 bins, one
//                            channel, mask off, wide windows).
//
// Default configuration, per crop:
//   * Median: the four waves each estimate it from 64 pixels of a 16 x 16
//     sampling grid; one pass over the crop then histograms the 64 mm window
//     centred on the combined estimate (1 mm bins, LDS atomics) and counts
//     non-zero pixels and pixels above the window's start in packed 16-bit
//     registers; when the median falls in the window the histogram gives
//     it, otherwise an exact two-level radix select (high byte, then low
//     byte) runs.
//   * Codes: lanes own 4 adjacent columns and walk down a band of rows with a
//     3-row register window. Each pixel is packed as (grey | d' << 16) with
//     d' = clamp(d - (m - window), 0, 2 window) (0 for d = 0): clamping keeps
//     every comparison against an in-window centre unchanged and makes the
//     depth fit 9 bits, so ONE packed 16-bit subtraction per neighbour yields
//     both channels' comparisons: the sign bit of each 16-bit half. Byte
//     permutes gather the sign bits of two neighbours per instruction and
//     masked AND-ORs merge them into one word holding both channels'
//     comparison bytes. Halo columns come from the neighbouring lanes through
//     DPP wave shifts.
//   * Counters: one LDS word per (cell, bin), the grey count in its low 16
//     bits and the depth count in its high 16 bits.
//   * Normalisation: count / T is tabulated once per crop for every count a
//     cell can hold, then the row is written by table lookup.
#include "lbpf_internal.h"

#include <algorithm>

namespace lbpf {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kFastMaxW = 256;    // 64 lanes x 4 columns
constexpr int kQuot = 1088;       // tabulated quotients (cells up to 32 x 34 px)
constexpr int kU59 = 59;

// Neighbour p of the centre (y, x) is (y + kDy[p], x + kDx[p]).
__constant__ int8_t kDy[8] = {-1, -1, -1, 0, 1, 1, 1, 0};
__constant__ int8_t kDx[8] = {-1, 0, 1, 1, 1, 0, -1, -1};

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub_sat(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t ld_u32(const void *p) {
    uint32_t v;
    __builtin_memcpy(&v, p, 4);
    return v;
}
__device__ __forceinline__ uint2 ld_u64(const void *p) {
    uint2 v;
    __builtin_memcpy(&v, p, 8);
    return v;
}
__device__ __forceinline__ uint4 ld_u128(const void *p) {
    uint4 v;
    __builtin_memcpy(&v, p, 16);
    return v;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct MedianScratch {
    uint32_t hist[256];
    int32_t bin;
    uint32_t rank;
    uint32_t est[kWaves];  // the waves' median estimates
};

// On wave 0: find the bin of a 256-bin LDS histogram that holds 0-based rank
// `rank`, and the rank inside that bin. rank >= total leaves ms.bin at -1.
__device__ __forceinline__ void select_bin(MedianScratch &ms, uint32_t rank, int lane) {
    const uint32_t c0 = ms.hist[4 * lane + 0], c1 = ms.hist[4 * lane + 1],
                   c2 = ms.hist[4 * lane + 2], c3 = ms.hist[4 * lane + 3];
    const uint32_t s = c0 + c1 + c2 + c3;
    const uint32_t incl = wave_inclusive_scan(s, lane);
    const uint32_t excl = incl - s;
    if (lane == 0) ms.bin = -1;
    if (excl <= rank && rank < incl) {
        uint32_t r = rank - excl;
        int b = 4 * lane;
        if (r >= c0) {
            r -= c0;
            b += 1;
            if (r >= c1) {
                r -= c1;
                b += 1;
                if (r >= c2) {
                    r -= c2;
                    b += 1;
                }
            }
        }
        ms.bin = b;
        ms.rank = r;
    }
}

// Load the 8 depth pixels x0..x0+7 of a row (zeros past the crop's width).
__device__ __forceinline__ void load8(const uint16_t *row, int x0, int w, uint32_t v[8]) {
    if (x0 + 8 <= w) {
        const uint4 q = ld_u128(row + x0);
        v[0] = q.x & 0xFFFFu; v[1] = q.x >> 16;
        v[2] = q.y & 0xFFFFu; v[3] = q.y >> 16;
        v[4] = q.z & 0xFFFFu; v[5] = q.z >> 16;
        v[6] = q.w & 0xFFFFu; v[7] = q.w >> 16;
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (x0 + i < w) ? row[x0 + i] : 0u;
    }
}

// Exact lower median of the non-zero depth values of the crop, -1 if none.
// All threads of the block call it.
__device__ __noinline__ int32_t crop_median(const CropDesc c, MedianScratch &ms) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cpr = (c.w + 7) >> 3;              // 8-pixel chunks per row (<= 128)
    const int rows_par = kThreads / cpr;         // rows visited in parallel
    const int cx = tid % cpr, ry0 = tid / cpr;
    const bool act = ry0 < rows_par;
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    __syncthreads();
    if (act) {
        for (int y = ry0; y < c.h; y += rows_par) {
            uint32_t v[8];
            load8(c.depth + (size_t)y * c.depth_pitch, 8 * cx, c.w, v);
            const uint32_t key = (v[3] ? v[3] : v[4]) >> 8;
            uint32_t same = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) same += (v[i] != 0 && (v[i] >> 8) == key) ? 1u : 0u;
            if (same) atomicAdd(&ms.hist[key], same);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (v[i] != 0 && (v[i] >> 8) != key) atomicAdd(&ms.hist[v[i] >> 8], 1u);
        }
    }
    __syncthreads();
    if (wave == 0) {
        const uint32_t tot = wave_sum(ms.hist[4 * lane] + ms.hist[4 * lane + 1] +
                                      ms.hist[4 * lane + 2] + ms.hist[4 * lane + 3]);
        if (tot > 0) {
            select_bin(ms, (tot - 1) / 2, lane);
        } else if (lane == 0) {
            ms.bin = -1;
        }
    }
    __syncthreads();
    const int32_t hi = ms.bin;
    const uint32_t rank_in_hi = ms.rank;
    if (hi < 0) return -1;
    __syncthreads();
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    __syncthreads();
    if (act) {
        for (int y = ry0; y < c.h; y += rows_par) {
            uint32_t v[8];
            load8(c.depth + (size_t)y * c.depth_pitch, 8 * cx, c.w, v);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                if (v[i] != 0 && (int32_t)(v[i] >> 8) == hi) atomicAdd(&ms.hist[v[i] & 255u], 1u);
        }
    }
    __syncthreads();
    if (wave == 0) select_bin(ms, rank_in_hi, lane);
    __syncthreads();
    const int32_t m = (hi << 8) | ms.bin;
    __syncthreads();
    return m;
}

__device__ __forceinline__ bool centre_in_mask(uint32_t d, int32_t m, int32_t window) {
    if (window <= 0) return true;
    if (m < 0 || d == 0) return false;
    const int32_t diff = (int32_t)d - m;
    return diff < window && -diff < window;
}

template <typename T>
__device__ __forceinline__ uint32_t lbp_code(const T *p, int32_t pitch, int y, int x) {
    const uint32_t c = p[(size_t)y * pitch + x];
    uint32_t code = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t g = p[(size_t)(y + kDy[k]) * pitch + (x + kDx[k])];
        code |= (g >= c ? 1u : 0u) << k;
    }
    return code;
}

// Per-pixel histogram loop for any crop and configuration: each thread takes
// pixels in row order and increments its bins with LDS atomics.
// With `packed` (both channels in use) the counters are the fast path's: one
// word per (cell, bin), grey count in the low half, depth count in the high.
template <int kNW = kWaves>
__device__ void lbp_hist_generic(const CropDesc c, const FeatParams &fp, int32_t m,
                                 const uint8_t *sh_bin, const uint8_t *sh_rowband,
                                 const uint8_t *sh_colband, uint32_t *sh_hist,
                                 bool packed = false) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cells = fp.grid_x * fp.grid_y;
    const int nb = fp.nbins;
    for (int y = 1 + wave; y <= c.h - 2; y += kNW) {
        const int rowcell = sh_rowband[y] * fp.grid_x;
        for (int x = 1 + lane; x <= c.w - 2; x += 64) {
            const uint32_t dc = c.depth[(size_t)y * c.depth_pitch + x];
            if (!centre_in_mask(dc, m, fp.window)) continue;
            const int cell = rowcell + sh_colband[x];
            int ch = 0;
            if (fp.use_grey) {
                const uint32_t code = lbp_code(c.grey, c.grey_pitch, y, x);
                atomicAdd(&sh_hist[cell * nb + sh_bin[code]], 1u);
                ch = 1;
            }
            if (fp.use_depth) {
                const uint32_t code = lbp_code(c.depth, c.depth_pitch, y, x);
                if (packed)
                    atomicAdd(&sh_hist[cell * nb + sh_bin[code]], 0x10000u);
                else
                    atomicAdd(&sh_hist[(ch * cells + cell) * nb + sh_bin[code]], 1u);
            }
        }
    }
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Load through the global address space at a 32-bit byte offset from a
// workgroup-uniform base (global_load with an SGPR base). Unaligned
// addresses are fine on gfx950.
template <typename T>
__device__ __forceinline__ T gld(const void *base, uint32_t byte_off) {
    typedef __attribute__((address_space(1))) const T gT;
    return *(const gT *)((const __attribute__((address_space(1))) char *)base + byte_off);
}

// Streaming (non-temporal) store: the feature rows are not read again by this
// kernel, and kept out of L2's reuse they do not evict the depth lines that
// the code pass reads a second time.
template <typename T>
__device__ __forceinline__ void st_nt(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}
// (a & m) | c with m in an SGPR: one VALU instruction (gfx9 VOP3 takes no
// literal, so the compiler would otherwise split it into AND + OR).
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t m, uint32_t c) {
    uint32_t r;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(m), "v"(c));
    return r;
}

// a + b + c in one instruction; written out because the compiler otherwise
// shares a + b between two such sums and spends three adds on them.
__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

// Depth pixels x0..x0+7 of crop row y as four u16 pairs; pixels at x >= w
// read as 0. A chunk that ends past the right edge of a crop that may not be
// over-read is loaded from column w - 8 instead (crops at least 8 wide), and
// the pixels before x0 are zeroed as well: the median pass does not count a
// zero, so every pixel still counts once, and the chunk is one load.
__device__ __forceinline__ u32x4 depth_chunk(const CropDesc &c, int y, int x0) {
    const bool inside = (c.flags & kCropOverReadOk) || x0 + 8 <= c.w;
    if (inside || c.w >= 8) {
        const int xs = inside ? x0 : c.w - 8;
        u32x4 q = gld<u32x4>(c.depth, ((uint32_t)y * (uint32_t)c.depth_pitch + (uint32_t)xs) * 2u);
        if (x0 + 8 > c.w) {
            // Element e (column xs + e) is kept iff x0 <= xs + e < w.
            const int lo = x0 - xs, hi = c.w - xs;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t keep = (2 * i >= lo && 2 * i < hi ? 0x0000FFFFu : 0u) |
                                      (2 * i + 1 >= lo && 2 * i + 1 < hi ? 0xFFFF0000u : 0u);
                q[i] &= keep;
            }
        }
        return q;
    }
    const uint16_t *row = c.depth + (size_t)y * c.depth_pitch;
    u32x4 q;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t a = (x0 + 2 * i < c.w) ? row[x0 + 2 * i] : 0u;
        const uint32_t b = (x0 + 2 * i + 1 < c.w) ? row[x0 + 2 * i + 1] : 0u;
        q[i] = a | (b << 16);
    }
    return q;
}

constexpr int kMedBatch = 8;  // 16-byte chunks in flight per thread

// Width (mm) of the median pass's 1 mm window histogram, centred on the
// estimate.
constexpr uint32_t kMedWin = 64;

// One u16 pair of the median pass: per-half counts of v >= lo (ge2) and of
// v != 0 (nz2), and the 1 mm window histogram of [lo, lo + kMedWin). one2
// holds 0x10001 (kept opaque to the compiler, see crop_median_fast).
__device__ __forceinline__ void median_count(uint32_t q, uint32_t lolo, uint32_t lm1,
                                             uint32_t one2, uint32_t &ge2, uint32_t &nz2,
                                             MedianScratch &ms) {
    // v >= lo iff v - (lo - 1) saturates above 0 (lo >= 1, so 0 is not).
    ge2 += pk_min(pk_sub_sat(q, lm1), one2);
    nz2 += pk_min(q, one2);
    const uint32_t t = pk_sub(q, lolo);  // v - lo; >= kMedWin for v = 0
    const uint32_t t0 = t & 0xFFFFu, t1 = t >> 16;
    if (t0 < kMedWin) atomicAdd(&ms.hist[t0], 1u);
    if (t1 < kMedWin) atomicAdd(&ms.hist[t1], 1u);
}

// End of the median pass for a block of kNW waves: totals over the block,
// then the lower median's rank looked up in the window histogram. Returns
// the median, -1 when the crop has no depth, -2 when the median lies outside
// [lo, lo + kMedWin) (the caller then runs the exact radix select). All threads
// call it; it ends with a barrier.
template <int kNW>
__device__ __forceinline__ int32_t median_finish(MedianScratch &ms, uint32_t *sh_red,
                                                 uint32_t ge2, uint32_t nz2, int32_t lo) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nnz = wave_sum((nz2 & 0xFFFFu) + (nz2 >> 16));
    const uint32_t below = nnz - wave_sum((ge2 & 0xFFFFu) + (ge2 >> 16));
    if (lane == 0) {
        sh_red[wave] = below;
        sh_red[kNW + wave] = nnz;
    }
    __syncthreads();
    uint32_t tb = 0, tn = 0;
#pragma unroll
    for (int i = 0; i < kNW; ++i) {
        tb += sh_red[i];
        tn += sh_red[kNW + i];
    }
    if (tn == 0) return -1;  // uniform: every thread sees the same totals
    const uint32_t rank = (tn - 1) / 2;
    if (wave == 0) {
        if (rank >= tb) {
            select_bin(ms, rank - tb, lane);  // -1 when the rank lies above the window
        } else if (lane == 0) {
            ms.bin = -1;
        }
    }
    __syncthreads();
    const int32_t bin = ms.bin;
    __syncthreads();
    (void)tid;
    return bin >= 0 ? lo + bin : -2;
}

// One wave's 64-sample estimate of the median: the lower median of the
// non-zero values among `v` (one per lane), or 1000 when all are zero. A binary
// search over the value range finds the smallest t with more than `rank`
// non-zero samples <= t, each count a ballot (16 steps of one compare).
__device__ __forceinline__ uint32_t median_estimate(uint32_t v) {
    const int nz = __popcll(__ballot(v != 0));
    if (nz == 0) return 1000u;
    const uint32_t rank = (uint32_t)(nz - 1) / 2;
    const uint32_t vm1 = v - 1u;  // v = 0 wraps above every bound
    uint32_t lo = 1, hi = 65535;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint32_t)__popcll(__ballot(vm1 < mid)) > rank)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Exact lower median of the crop's non-zero depth, -1 if none.
//  1. Each wave estimates it as the lower median of the non-zero values
//     among 64 pixels of a 16 x 16 sampling grid (wave w takes the grid rows
//     w, w + 4, ...); the estimate is the mean of the middle two of the four.
//  2. One pass over the crop: a 1 mm histogram of the kMedWin values
//     [lo, lo + kMedWin) centred on the estimate (LDS atomics), and
//     per-thread counts of the non-zero pixels and of those below the window
//     (packed 16-bit arithmetic, no atomics).
//  3. When the median's rank falls inside the window, the window histogram
//     gives it exactly; otherwise the two-level radix select runs.
// All threads of the block call it.
__device__ __forceinline__ int32_t crop_median_fast(const CropDesc &c, MedianScratch &ms,
                                                   uint32_t *sh_red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cpr = (c.w + 7) >> 3;
    const int rows_par = kThreads / cpr;
    const int cx = tid % cpr, ry0 = tid / cpr;
    const int nk = ry0 < rows_par ? (c.h - ry0 + rows_par - 1) / rows_par : 0;
    const int x0 = 8 * cx;
    // The first batch of chunks does not depend on the estimate: issue its
    // loads before the estimate is taken so the two latencies overlap.
    u32x4 buf[kMedBatch];
#pragma unroll
    for (int u = 0; u < kMedBatch; ++u)
        if (nk > 0) buf[u] = depth_chunk(c, ry0 + min(u, nk - 1) * rows_par, x0);
    // select_bin scans all 256 bins; the pass fills the first kMedWin.
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    {
        // Wave w samples grid rows w, w + 4, ... of a 16 x 16 grid over the
        // crop, so each wave's estimate covers the whole crop.
        const int gr = 4 * (lane >> 4) + wave, gc = lane & 15;
        const int sy = ((2 * gr + 1) * c.h) >> 5, sx = ((2 * gc + 1) * c.w) >> 5;
        const uint32_t e = median_estimate(c.depth[(size_t)sy * c.depth_pitch + sx]);
        if (lane == 0) ms.est[wave] = e;
    }
    __syncthreads();
    // The mean of the middle two of the four wave estimates.
    const uint32_t ea = min(ms.est[0], ms.est[1]), eb = max(ms.est[0], ms.est[1]);
    const uint32_t ec = min(ms.est[2], ms.est[3]), ed = max(ms.est[2], ms.est[3]);
    const int32_t est = (int32_t)((max(ea, ec) + min(eb, ed)) >> 1);
    const int32_t lo = min(max(est - (int32_t)kMedWin / 2, 1), 65536 - (int32_t)kMedWin);
    const uint32_t lolo = (uint32_t)lo * 0x10001u;
    const uint32_t lm1 = (uint32_t)(lo - 1) * 0x10001u;
    // A 1 in each half that the compiler cannot see: with a visible constant
    // it turns each packed min below into two compares and selects.
    uint32_t one2 = 0x10001u;
    asm volatile("" : "+s"(one2));

    uint32_t ge2 = 0, nz2 = 0;  // per-half counts of v >= lo and of v != 0
    for (int kb = 0; kb < nk; kb += kMedBatch) {
        if (kb > 0) {
#pragma unroll
            for (int u = 0; u < kMedBatch; ++u)
                buf[u] = depth_chunk(c, ry0 + min(kb + u, nk - 1) * rows_par, x0);
        }
#pragma unroll
        for (int u = 0; u < kMedBatch; ++u) {
            if (kb + u >= nk) break;
#pragma unroll
            for (int i = 0; i < 4; ++i) median_count(buf[u][i], lolo, lm1, one2, ge2, nz2, ms);
        }
    }
    const int32_t r = median_finish<kWaves>(ms, sh_red, ge2, nz2, lo);
    return r != -2 ? r : crop_median(c, ms);
}

// Columns x0..x0+3 of one row as loaded: grey bytes in G, depth u16 pairs
// in Z0 (x0, x0+1) and Z1 (x0+2, x0+3). Every lane issues the same two loads,
// from column xl = x0, or, for a lane that hangs over the right edge of a crop
// that may not be over-read, from xl = w - 4; make_row then shifts that
// lane's columns down by s = x0 - xl. Columns past the crop are never used.
struct RawRow {
    uint32_t G, Z0, Z1;
};

__device__ __forceinline__ RawRow load_row(const CropDesc &c, int y, int xl) {
    RawRow r;
    r.G = gld<uint32_t>(c.grey, (uint32_t)y * (uint32_t)c.grey_pitch + (uint32_t)xl);
    const u32x2 z =
        gld<u32x2>(c.depth, ((uint32_t)y * (uint32_t)c.depth_pitch + (uint32_t)xl) * 2u);
    r.Z0 = z.x;
    r.Z1 = z.y;
    return r;
}

// load_row at byte offsets goff (grey plane) and doff (depth plane) from the
// crop's origin.
__device__ __forceinline__ RawRow load_row_at(const CropDesc &c, uint32_t goff, uint32_t doff) {
    RawRow r;
    r.G = gld<uint32_t>(c.grey, goff);
    const u32x2 z = gld<u32x2>(c.depth, doff);
    r.Z0 = z.x;
    r.Z1 = z.y;
    return r;
}

// d' = clamp(d - lo, 0, span) on a pair of u16, for lo >= 0 (so d = 0 maps
// to 0).
__device__ __forceinline__ uint32_t to_window(uint32_t z, uint32_t lolo, uint32_t span2) {
    return pk_min(pk_sub_sat(z, lolo), span2);
}

// Row of 6 packed pixels (grey | d' << 16): columns [x0-1, x0 .. x0+3, x0+4].
struct Row6 {
    uint32_t p[6];
};

// s8 = 8 s and s16 = 16 s for the column shift s of load_row.
__device__ __forceinline__ Row6 make_row(const RawRow &raw, uint32_t lolo, uint32_t span2,
                                         uint32_t s8, uint32_t s16) {
    const uint32_t G = raw.G >> s8;
    const uint64_t Z = ((((uint64_t)raw.Z1) << 32) | raw.Z0) >> s16;
    const uint32_t D0 = to_window((uint32_t)Z, lolo, span2);
    const uint32_t D1 = to_window((uint32_t)(Z >> 32), lolo, span2);
    Row6 r;
    r.p[1] = __builtin_amdgcn_perm(G, D0, 0x01000C04u);
    r.p[2] = __builtin_amdgcn_perm(G, D0, 0x03020C05u);
    r.p[3] = __builtin_amdgcn_perm(G, D1, 0x01000C06u);
    r.p[4] = __builtin_amdgcn_perm(G, D1, 0x03020C07u);
    // Left halo = previous lane's last pixel, right halo = next lane's first.
    // bound_ctrl: the lane with no source (0, resp. 63) reads 0, and no old
    // value has to be set up first.
    r.p[0] = __builtin_amdgcn_mov_dpp(r.p[4], 0x138, 0xF, 0xF, true);  // wave_shr:1
    r.p[5] = __builtin_amdgcn_mov_dpp(r.p[1], 0x130, 0xF, 0xF, true);  // wave_shl:1
    return r;
}

// Byte 0 | byte 1 and byte 2 | byte 3 of x, one SDWA instruction each.
__device__ __forceinline__ uint32_t or_b01(uint32_t x) {
    uint32_t r;
    asm("v_or_b32_sdwa %0, %1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_0 src1_sel:BYTE_1"
        : "=v"(r)
        : "v"(x));
    return r;
}
__device__ __forceinline__ uint32_t or_b23(uint32_t x) {
    uint32_t r;
    asm("v_or_b32_sdwa %0, %1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_2 src1_sel:BYTE_3"
        : "=v"(r)
        : "v"(x));
    return r;
}

// Comparison bits of the centre B[j] against its 8 neighbours in rows A
// (y-1), B (y), C (y+1). A set bit means the neighbour is BELOW the centre:
// the sign of the packed 16-bit difference neighbour - centre, bit 15 for
// grey and bit 31 for depth. v_perm's selectors 8-11 replicate those sign
// bits into whole bytes, so each perm gathers the four signs of two
// neighbours (bytes: grey of the first, grey of the second, depth of the
// first, depth of the second); the masks then keep bit p for neighbour p.
// Grey index = byte 0 | byte 1, depth index = byte 2 | byte 3 (or_b01,
// or_b23): bit p <-> neighbour p in both.
__device__ __forceinline__ uint32_t compare_bits(const Row6 &A, const Row6 &B, const Row6 &C, int j) {
    const uint32_t c = B.p[j];
    // All eight differences first: a packed result read by the very next
    // instruction costs a wait state on gfx950.
    const uint32_t d0 = pk_sub(A.p[j - 1], c), d1 = pk_sub(A.p[j], c), d2 = pk_sub(A.p[j + 1], c);
    const uint32_t d3 = pk_sub(B.p[j + 1], c), d4 = pk_sub(C.p[j + 1], c), d5 = pk_sub(C.p[j], c);
    const uint32_t d6 = pk_sub(C.p[j - 1], c), d7 = pk_sub(B.p[j - 1], c);
    // perm(hi, lo, sel): 8 = sign of lo[15], 9 = lo[31], 10 = hi[15], 11 = hi[31].
    constexpr uint32_t kSel = 0x090B080Au;
    uint32_t acc = __builtin_amdgcn_perm(d0, d1, kSel) & 0x02010201u;
    acc = and_or(__builtin_amdgcn_perm(d2, d3, kSel), 0x08040804u, acc);
    acc = and_or(__builtin_amdgcn_perm(d4, d5, kSel), 0x20102010u, acc);
    acc = and_or(__builtin_amdgcn_perm(d6, d7, kSel), 0x80408040u, acc);
    return acc;
}

// LDS of the fast path, about 23 KB: six workgroups fit a CU's LDS.
struct FastShared {
    // cells * 59 words: the grey count of (cell, bin) in the low half, the
    // depth count in the high half (a cell holds fewer than 65536 pixels).
    __attribute__((aligned(16))) uint32_t hist[64 * kU59];
    MedianScratch ms;
    uint8_t bin[256];    // code -> bin
    uint8_t lut[256];    // comparison byte (bit p: neighbour p below) -> 4 x bin
    uint8_t rowband[LBPF_MAX_SIDE];
    uint8_t colband[LBPF_MAX_SIDE];
    uint16_t rowoff[LBPF_MAX_SIDE];  // byte offset of row y's band in hist
    float q[kQuot];
    uint32_t red[2 * kWaves];
    int32_t next;
};

__device__ __forceinline__ void load_tables(FastShared &sh, const uint8_t *tables) {
    for (int i = threadIdx.x; i < 256; i += kThreads) {
        sh.bin[i] = tables[i];
        sh.lut[i] = (uint8_t)(4 * tables[256 + i]);  // bins <= 58: byte offsets fit
    }
}

// Normalisation and output of one crop by a block of kNT threads, after the
// counting (the caller's barrier): n_in = total of the grey counts, T = 2 n_in,
// grey count / T to out[0 .. half), depth count / T to out[half .. 2 half),
// raw counts to cout when it is not null. maxc bounds every count, so when it
// is below kQuot the quotients are tabulated once in q. red holds kNT / 64
// words.
template <int kNT>
__device__ __forceinline__ void finish_crop(const uint32_t *hist, int half, int maxc, float *q,
                                            uint32_t *red, float *out, uint32_t *cout) {
    constexpr int kNW = kNT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t part = 0;
    for (int i = tid; i < half; i += kNT) part += hist[i] & 0xFFFFu;
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    uint32_t n_in = 0;
#pragma unroll
    for (int i = 0; i < kNW; ++i) n_in += red[i];
    const float T = (float)(2u * n_in);
    const bool tab = maxc < kQuot;
    if (tab) {
        for (int v = tid; v <= maxc; v += kNT) q[v] = n_in ? (float)v / T : 0.0f;
        __syncthreads();
    }
    const bool vec = (half & 3) == 0 && ((uintptr_t)out & 15) == 0 && ((uintptr_t)cout & 15) == 0;
    if (vec && tab) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        for (int i = 4 * tid; i < half; i += 4 * kNT) {
            const u32x4 v = *reinterpret_cast<const u32x4 *>(&hist[i]);
            const u32x4 g = v & 0xFFFFu, d = v >> 16;
            st_nt(reinterpret_cast<f32x4 *>(out + i), f32x4{q[g.x], q[g.y], q[g.z], q[g.w]});
            st_nt(reinterpret_cast<f32x4 *>(out + half + i), f32x4{q[d.x], q[d.y], q[d.z], q[d.w]});
            if (cout) {
                *reinterpret_cast<u32x4 *>(cout + i) = g;
                *reinterpret_cast<u32x4 *>(cout + half + i) = d;
            }
        }
    } else {
        for (int i = tid; i < half; i += kNT) {
            const uint32_t v = hist[i], g = v & 0xFFFFu, d = v >> 16;
            out[i] = tab ? q[g] : (n_in ? (float)g / T : 0.0f);
            out[half + i] = tab ? q[d] : (n_in ? (float)d / T : 0.0f);
            if (cout) {
                cout[i] = g;
                cout[half + i] = d;
            }
        }
    }
}

// Features of one crop by the whole workgroup: row `out` (and `cout` when
// not null) of length fp.dim. The tables must already be in LDS; the caller
// separates consecutive crops with a barrier. kPF = rows loaded ahead.
template <int kPF, bool kEarly>
__device__ void fast_crop(const CropDesc &cd, const FeatParams &fp, FastShared &sh, float *out,
                          uint32_t *cout) {
    // A private copy: the descriptor then lives in registers and is not
    // re-read after every LDS atomic that might alias it.
    const CropDesc c = cd;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int w = c.w, h = c.h;
    const int gx = fp.grid_x, gy = fp.grid_y, cells = gx * gy;

    const int half = cells * kU59;  // words of sh.hist; half of dim
    // 64 * 59 is a multiple of 4, so the rounded-up clear stays in the array.
    for (int i = 4 * tid; i < half; i += 4 * kThreads)
        *reinterpret_cast<u32x4 *>(&sh.hist[i]) = u32x4{0u, 0u, 0u, 0u};
    // Coordinate y lies in band floor(((y + 1) g - 1) / n) of a side of length n.
    for (int y = tid; y < h; y += kThreads) {
        const int band = ((y + 1) * gy - 1) / h;
        sh.rowband[y] = (uint8_t)band;
        sh.rowoff[y] = (uint16_t)(band * gx * kU59 * 4);  // < 64 * 59 * 4
    }
    for (int x = tid; x < w; x += kThreads) sh.colband[x] = (uint8_t)(((x + 1) * gx - 1) / w);

    // Stream geometry of the code phase. Its first rows do not depend on the
    // median: with kEarly their loads are issued now and land while the
    // median is computed (at the price of registers held across it).
    // The lane loads need w >= 4 unless the crop may be over-read.
    const bool fast = w <= kFastMaxW && (w >= 4 || (c.flags & kCropOverReadOk));
    const int L = (w + 3) >> 2;           // lanes per stream (<= 64 when fast)
    const int spw = fast ? 64 / L : 1;    // streams per wave
    const int sw = lane / L;              // stream of this lane within the wave
    const int x0 = 4 * (lane - sw * L);
    const int S = kWaves * spw;
    const int s = wave * spw + (sw < spw ? sw : 0);
    const int rows = h - 2;
    // Stream s owns rows yb .. yb + n_own - 1. Every lane of the block steps
    // through n_step >= n_own rows, so the row loop is uniform; the rows past
    // a lane's own are loaded and coded but not counted. They stay inside the
    // crop: floor(s R / S) + ceil(R / S) <= R, so the last centre row
    // yb + n_step - 1 <= h - 2 and its lower neighbour row <= h - 1.
    const int yb = 1 + (s * rows) / S;
    const int n_own = (fast && sw < spw) ? 1 + ((s + 1) * rows) / S - yb : 0;
    const int n_step = (rows + S - 1) / S;
    const bool full = (c.flags & kCropOverReadOk) || x0 + 4 <= w;
    const int xl = full ? x0 : w - 4;
    const uint32_t s8 = 8u * (uint32_t)(x0 - xl), s16 = 2u * s8;
    RawRow rawA, rawB, ring[kPF];
    auto prime = [&]() {
        rawA = load_row(c, yb - 1, xl);
        rawB = load_row(c, yb, xl);
#pragma unroll
        for (int u = 0; u < kPF; ++u) ring[u] = load_row(c, min(yb + 1 + u, h - 1), xl);
    };
    if (kEarly && fast) prime();

    // Ends with a barrier; the same value in every lane.
    const int32_t m = __builtin_amdgcn_readfirstlane(crop_median_fast(c, sh.ms, sh.red));
    const int32_t lo = m - fp.window;
    // The packed window arithmetic needs lo >= 0: a crop whose median lies
    // within the window of 0 takes the generic path.
    if (fast && (m < 0 || lo >= 0)) {
        if (m >= 0) {
            if (!kEarly) prime();
            const uint32_t lolo = (uint32_t)lo * 0x10001u;
            const uint32_t span2 = (uint32_t)(2 * fp.window) * 0x10001u;
            const uint32_t in_hi = (uint32_t)(2 * fp.window - 1) << 16;

            // Per column: histogram column offset (bytes) and in-window
            // threshold (0 for border or out-of-crop columns: never counted).
            // A pixel counts when its packed word plus the row's bias is
            // below the threshold: the bias subtracts 1 from d' in rows the
            // lane owns (so 1 <= d' < 2 window passes) and lifts d' above
            // every threshold in the others.
            uint32_t col4[4], thr[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int x = x0 + k;
                col4[k] = (uint32_t)(sh.colband[min(x, w - 1)] * kU59) * 4u;
                thr[k] = (x >= 1 && x <= w - 2) ? in_hi : 0u;
            }
            char *hbase = reinterpret_cast<char *>(sh.hist);

            Row6 A = make_row(rawA, lolo, span2, s8, s16);
            Row6 B = make_row(rawB, lolo, span2, s8, s16);
            // Byte offsets of the next row to refill, kept running so the loop
            // has no multiplies; rows past h - 1 clamp to it (the offsets
            // grow with the row).
            const uint32_t gstep = (uint32_t)c.grey_pitch, dstep = 2u * (uint32_t)c.depth_pitch;
            const uint32_t r0 = (uint32_t)(yb + 1 + kPF), rl = (uint32_t)(h - 1);
            uint32_t gnext = r0 * gstep + (uint32_t)xl, dnext = r0 * dstep + 2u * (uint32_t)xl;
            const uint32_t gmax = rl * gstep + (uint32_t)xl, dmax = rl * dstep + 2u * (uint32_t)xl;
            // One row: code the centre row B against A and C = the row in
            // `slot`, count it, then refill `slot` kPF rows ahead.
            auto step = [&](const int tt, RawRow &slot, const bool refill) {
                const int yy = yb + tt;
                const Row6 C = make_row(slot, lolo, span2, s8, s16);
                if (refill) slot = load_row_at(c, min(gnext, gmax), min(dnext, dmax));
                gnext += gstep;
                dnext += dstep;
                const uint32_t bias = tt < n_own ? 0xFFFF0000u : 0x7FFF0000u;
                const uint32_t row4 = sh.rowoff[yy];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t bits = compare_bits(A, B, C, k + 1);
                    if (B.p[k + 1] + bias < thr[k]) {
                        // The table holds 4 x bin: byte offsets.
                        const uint32_t og = sh.lut[or_b01(bits)];
                        const uint32_t od = sh.lut[or_b23(bits)];
                        atomicAdd(reinterpret_cast<uint32_t *>(hbase + add3(row4, col4[k], og)), 1u);
                        atomicAdd(reinterpret_cast<uint32_t *>(hbase + add3(row4, col4[k], od)),
                                  0x10000u);
                    }
                }
                A = B;
                B = C;
            };
            // Whole groups of kPF rows in a loop with no other exit, so the
            // wait for each ring slot counts exactly the loads issued after
            // it; then the remaining rows, which need no refill.
            int t = 0;
            for (; t + kPF <= n_step; t += kPF) {
#pragma unroll
                for (int u = 0; u < kPF; ++u) step(t + u, ring[u], true);
            }
#pragma unroll
            for (int u = 0; u < kPF - 1; ++u) {
                if (t + u >= n_step) break;  // uniform
                step(t + u, ring[u], false);
            }
        }
    } else {
        lbp_hist_generic(c, fp, m, sh.bin, sh.rowband, sh.colband, sh.hist, true);
    }
    __syncthreads();

    finish_crop<kThreads>(sh.hist, half, ((h + gy - 1) / gy) * ((w + gx - 1) / gx), sh.q, sh.red,
                          out, cout);
}

// One workgroup per crop.
template <int kPF>
__global__ __launch_bounds__(kThreads) void k_features_fast(const CropDesc *__restrict__ crops,
                                                            FeatParams fp,
                                                            const uint8_t *__restrict__ tables,
                                                            float *__restrict__ hist,
                                                            uint32_t *__restrict__ counts) {
    __shared__ FastShared sh;
    load_tables(sh, tables);
    const size_t i = blockIdx.x;
    fast_crop<kPF, true>(crops[i], fp, sh, hist + i * fp.dim, counts ? counts + i * fp.dim : nullptr);
}

// Persistent: a fixed grid of workgroups takes crops from a work queue in the
// order `order` (largest first balances ragged batches) until it runs dry.
// queue[0] is the next position, queue[1] counts finished workgroups; the
// last workgroup to finish resets both, so the kernel can be relaunched (or
// replayed from a graph) with no memset in between.
template <int kPF>
__global__ __launch_bounds__(kThreads, 4) void k_features_persistent(
    const CropDesc *__restrict__ crops, const int32_t *__restrict__ order, int32_t n,
    FeatParams fp, const uint8_t *__restrict__ tables, float *__restrict__ hist,
    uint32_t *__restrict__ counts, uint32_t *__restrict__ queue,
    const int32_t *__restrict__ n_dev) {
    __shared__ FastShared sh;
    if (n_dev) n = *n_dev;  // a batch count kept in device memory (graph replays)
    load_tables(sh, tables);
    if (threadIdx.x == 0) sh.next = (int32_t)atomicAdd(&queue[0], 1u);
    __syncthreads();
    for (;;) {
        // Every thread read the same j; readfirstlane tells the compiler so,
        // and the crop's descriptor is then fetched with scalar loads.
        const int32_t j = __builtin_amdgcn_readfirstlane(sh.next);
        if (j >= n) break;
        // The next position is taken now and published after this crop, so
        // the atomic's latency overlaps the crop (a workgroup takes one
        // position past the end on its way out).
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(&queue[0], 1u);
        const size_t i = order ? (size_t)order[j] : (size_t)j;
        fast_crop<kPF, false>(crops[i], fp, sh, hist + i * fp.dim, counts ? counts + i * fp.dim : nullptr);
        if (threadIdx.x == 0) sh.next = (int32_t)next;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1u) == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
        }
    }
}

// Any configuration: dynamic LDS holds fp.dim counters.
__global__ __launch_bounds__(kThreads) void k_features_generic(const CropDesc *__restrict__ crops,
                                                               FeatParams fp,
                                                               const uint8_t *__restrict__ tables,
                                                               float *__restrict__ hist,
                                                               uint32_t *__restrict__ counts) {
    extern __shared__ uint32_t sh_hist[];
    __shared__ MedianScratch ms;
    __shared__ uint8_t sh_bin[256];
    __shared__ uint8_t sh_rowband[LBPF_MAX_SIDE];
    __shared__ uint8_t sh_colband[LBPF_MAX_SIDE];
    __shared__ uint32_t sh_red[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const CropDesc c = crops[blockIdx.x];

    for (int i = tid; i < fp.dim; i += kThreads) sh_hist[i] = 0;
    for (int i = tid; i < 256; i += kThreads) sh_bin[i] = tables[i];
    for (int y = tid; y < c.h; y += kThreads) sh_rowband[y] = (uint8_t)(((y + 1) * fp.grid_y - 1) / c.h);
    for (int x = tid; x < c.w; x += kThreads) sh_colband[x] = (uint8_t)(((x + 1) * fp.grid_x - 1) / c.w);
    __syncthreads();
    const int32_t m = fp.window > 0 ? crop_median(c, ms) : -1;

    lbp_hist_generic(c, fp, m, sh_bin, sh_rowband, sh_colband, sh_hist);
    __syncthreads();

    const int per_ch = fp.grid_x * fp.grid_y * fp.nbins;
    uint32_t part = 0;
    for (int i = tid; i < per_ch; i += kThreads) part += sh_hist[i];
    part = wave_sum(part);
    if (lane == 0) sh_red[wave] = part;
    __syncthreads();
    uint32_t n_in = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) n_in += sh_red[w];
    const float T = (float)(fp.nch * n_in);

    float *out = hist + (size_t)blockIdx.x * fp.dim;
    uint32_t *cout = counts ? counts + (size_t)blockIdx.x * fp.dim : nullptr;
    for (int i = tid; i < fp.dim; i += kThreads) {
        const uint32_t v = sh_hist[i];
        out[i] = n_in ? (float)v / T : 0.0f;
        if (cout) cout[i] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_debug_codes(const CropDesc *__restrict__ crop,
                                                          FeatParams fp, uint8_t *gcodes,
                                                          uint8_t *dcodes, uint8_t *mask) {
    __shared__ MedianScratch ms;
    const CropDesc c = *crop;
    const int32_t m = fp.window > 0 ? crop_median(c, ms) : -1;
    for (int i = threadIdx.x; i < c.w * c.h; i += kThreads) {
        const int y = i / c.w, x = i % c.w;
        uint8_t g = 0, d = 0, k = 0;
        if (y >= 1 && y <= c.h - 2 && x >= 1 && x <= c.w - 2) {
            if (c.grey) g = (uint8_t)lbp_code(c.grey, c.grey_pitch, y, x);
            d = (uint8_t)lbp_code(c.depth, c.depth_pitch, y, x);
            k = centre_in_mask(c.depth[(size_t)y * c.depth_pitch + x], m, fp.window) ? 1 : 0;
        }
        gcodes[i] = g;
        dcodes[i] = d;
        mask[i] = k;
    }
}

}  // namespace

bool fast_path_ok(const FeatParams &fp) {
    // Packed 16-bit counters: a cell of the largest crop holds < 65536 pixels.
    const int64_t cell_max = (int64_t)((LBPF_MAX_SIDE + fp.grid_x - 1) / fp.grid_x) *
                             ((LBPF_MAX_SIDE + fp.grid_y - 1) / fp.grid_y);
    return fp.nbins == kU59 && fp.use_grey && fp.use_depth && fp.window >= 1 &&
           fp.window <= 255 && fp.grid_x * fp.grid_y <= 64 && cell_max < 65536;
}

hipError_t launch_features(const CropDesc *crops, int32_t n, const FeatParams &fp,
                           const uint8_t *d_tables, float *hist, uint32_t *counts,
                           hipStream_t s, const LaunchCfg &lc, const int32_t *order,
                           uint32_t *queue, int32_t num_cus, const int32_t *n_dev) {
    if (n <= 0) return hipSuccess;
    if (fast_path_ok(fp)) {
        const int pf = lc.row_prefetch <= 2 ? 2 : (lc.row_prefetch <= 4 ? 4 : 8);
        if (lc.persistent && queue) {
            const int grid = std::min<int>(n, std::max(1, lc.wg_per_cu) * num_cus);
            const int32_t *ord = lc.sorted ? order : nullptr;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, crops, ord, n, fp,
                                   d_tables, hist, counts, queue, n_dev);
            };
            if (pf == 2) go(k_features_persistent<2>);
            else if (pf == 4) go(k_features_persistent<4>);
            else go(k_features_persistent<8>);
        } else {
            if (n_dev) return hipErrorInvalidValue;  // device counts: the persistent kernel only
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(n), dim3(kThreads), 0, s, crops, fp, d_tables, hist,
                                   counts);
            };
            if (pf == 2) go(k_features_fast<2>);
            else if (pf == 4) go(k_features_fast<4>);
            else go(k_features_fast<8>);
        }
        return hipGetLastError();
    }
    if (n_dev) return hipErrorInvalidValue;  // device counts: the fast configuration only
    const size_t shmem = (size_t)fp.dim * sizeof(uint32_t);
    // Above 64 KiB of dynamic LDS (the 256-bin mapping) the kernel must opt in.
    static size_t shmem_limit = 64 * 1024;
    if (shmem > shmem_limit) {
        hipError_t e = hipFuncSetAttribute((const void *)k_features_generic,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shmem);
        if (e != hipSuccess) return e;
        shmem_limit = shmem;
    }
    hipLaunchKernelGGL(k_features_generic, dim3(n), dim3(kThreads), shmem, s, crops, fp,
                       d_tables, hist, counts);
    return hipGetLastError();
}

hipError_t launch_debug_codes(const CropDesc *crop, const FeatParams &fp, uint8_t *gcodes,
                              uint8_t *dcodes, uint8_t *mask, int32_t, int32_t, hipStream_t s) {
    hipLaunchKernelGGL(k_debug_codes, dim3(1), dim3(kThreads), 0, s, crop, fp, gcodes, dcodes,
                       mask);
    return hipGetLastError();
}

}  // namespace lbpf
