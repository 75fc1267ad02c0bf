// Fused depth-masked LBP + regional histogram + L1 normalisation, gfx950.
//
// One workgroup (4 wave64) per face crop; every step runs inside one launch:
//   1. exact lower median m of the crop's non-zero depth (the depth region of
//      interest of the paper's fusion), by a two-level radix select: a 256-bin
//      histogram of the high bytes, then of the low bytes inside the selected
//      high byte;
//   2. for every interior pixel whose depth d satisfies d != 0 and
//      |d - m| < window, the 3x3 LBP code of the grey and of the depth plane
//      (Sec. 2.4, Eq. 2: neighbour p has weight 2^p and its bit is set when it
//      is >= the centre; p0 = top-left neighbour, then clockwise);
//   3. code -> uniform-59 bin through a 256-entry LDS table;
//   4. increments of the [channel][ry][rx][bin] regional histogram (Eq. 3)
//      held in LDS;
//   5. the row written once to HBM as count / T, T = channels * n_in, each
//      quotient the correctly rounded IEEE single division (and optionally the
//      raw counts).
//
// Two kernels:
//   k_features_fast  -- the default configuration (uniform-59 bins, both
//                       channels, window 1..255 mm). Crops up to 256 px wide
//                       take the fast path below; wider crops fall back to the
//                       generic per-pixel loop inside the same launch.
//   k_features_generic -- every other configuration (256 bins, one channel,
//                       mask off, wide windows).
//
// Fast path, per crop:
//   * Median: each thread loads 8 depth pixels per 16-byte load and adds them
//     to the high-byte histogram as one count for the pixels sharing the
//     first pixel's high byte (smooth depth makes that the common case) plus
//     one count per other pixel, so contention on the LDS atomics stays low.
//   * Codes: lanes own 4 adjacent columns and walk down a band of rows with a
//     3-row register window. Each pixel is packed as (grey | d' << 16) with
//     d' = clamp(d - (m - window), 0, 2 window) (0 for d = 0): clamping keeps
//     every comparison against an in-window centre unchanged and makes the
//     depth fit 9 bits, so ONE packed 16-bit subtraction per neighbour yields
//     both channels' comparisons. For a negative difference the high bits of
//     each 16-bit half are all ones (bits 8..15 for grey, 9..15 for d'), so
//     one AND-OR per neighbour deposits the grey bit and the depth bit into
//     distinct positions of one accumulator. Halo columns come from the
//     neighbouring lanes through DPP wave shifts.
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
__device__ int32_t crop_median(const CropDesc &c, MedianScratch &ms) {
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
__device__ void lbp_hist_generic(const CropDesc &c, const FeatParams &fp, int32_t m,
                                 const uint8_t *sh_bin, const uint8_t *sh_rowband,
                                 const uint8_t *sh_colband, uint32_t *sh_hist) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cells = fp.grid_x * fp.grid_y;
    const int nb = fp.nbins;
    for (int y = 1 + wave; y <= c.h - 2; y += kWaves) {
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

// (a & m) | c with m in an SGPR: one VALU instruction (gfx9 VOP3 takes no
// literal, so the compiler would otherwise split it into AND + OR).
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t m, uint32_t c) {
    uint32_t r;
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(m), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

// Depth pixels x0..x0+7 of crop row y as four u16 pairs; pixels at x >= w
// read as 0.
__device__ __forceinline__ u32x4 depth_chunk(const CropDesc &c, int y, int x0) {
    if ((c.flags & kCropOverReadOk) || x0 + 8 <= c.w) {
        u32x4 q = gld<u32x4>(c.depth, ((uint32_t)y * (uint32_t)c.depth_pitch + (uint32_t)x0) * 2u);
        if (x0 + 8 > c.w) {
            const int valid = c.w - x0;  // 1..7
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t keep = (2 * i + 1 < valid ? 0xFFFF0000u : 0u) |
                                      (2 * i < valid ? 0x0000FFFFu : 0u);
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

// Ascending bitonic sort of one value per lane across a wave.
__device__ __forceinline__ uint32_t wave_sort64(uint32_t x, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t y = __shfl_xor(x, j, 64);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            x = keep_min ? min(x, y) : max(x, y);
        }
    }
    return x;
}

// Exact lower median of the crop's non-zero depth, -1 if none.
//  1. Wave 0 estimates it: the lower median of the non-zero values among 64
//     pixels on an 8 x 8 grid.
//  2. One pass over the crop: a 1 mm histogram of the 256 values
//     [lo, lo + 256) around the estimate (LDS atomics on well-spread
//     addresses), and per-thread counts of the non-zero pixels and of those
//     below the window (packed 16-bit arithmetic, no atomics).
//  3. When the median's rank falls inside the window, the window histogram
//     gives it exactly; otherwise the two-level radix select runs.
// All threads of the block call it.
__device__ int32_t crop_median_fast(const CropDesc &c, MedianScratch &ms, uint32_t *sh_red) {
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
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    if (wave == 0) {
        const int sy = ((2 * (lane >> 3) + 1) * c.h) >> 4;
        const int sx = ((2 * (lane & 7) + 1) * c.w) >> 4;
        const uint32_t v = c.depth[(size_t)sy * c.depth_pitch + sx];
        const uint32_t sorted = wave_sort64(v ? v : 0x10000u, lane);  // zeros last
        const int nz = __popcll(__ballot(v != 0));
        const uint32_t est = __shfl(sorted, nz > 0 ? (nz - 1) / 2 : 0, 64);
        if (lane == 0) ms.rank = nz > 0 ? est : 1000u;
    }
    __syncthreads();
    const int32_t lo = min(max((int32_t)ms.rank - 128, 1), 65536 - 256);
    const uint32_t lolo = (uint32_t)lo * 0x10001u;
    const uint32_t lm1 = (uint32_t)(lo - 1) * 0x10001u;

    uint32_t below2 = 0, nz2 = 0;  // per-half counts
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
            for (int i = 0; i < 4; ++i) {
                const uint32_t q = buf[u][i];
                // below: 1 <= v < lo, i.e. v - 1 < lo - 1 (v = 0 wraps high).
                below2 += pk_min(pk_sub_sat(lm1, pk_sub(q, 0x10001u)), 0x10001u);
                nz2 += pk_min(q, 0x10001u);
                const uint32_t t = pk_sub(q, lolo);  // v - lo; >= 256 for v = 0
                const uint32_t t0 = t & 0xFFFFu, t1 = t >> 16;
                if (t0 < 256u) atomicAdd(&ms.hist[t0], 1u);
                if (t1 < 256u) atomicAdd(&ms.hist[t1], 1u);
            }
        }
    }
    const uint32_t below = wave_sum((below2 & 0xFFFFu) + (below2 >> 16));
    const uint32_t nnz = wave_sum((nz2 & 0xFFFFu) + (nz2 >> 16));
    if (lane == 0) {
        sh_red[wave] = below;
        sh_red[kWaves + wave] = nnz;
    }
    __syncthreads();
    uint32_t tb = 0, tn = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        tb += sh_red[i];
        tn += sh_red[kWaves + i];
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
    if (bin >= 0) return lo + bin;
    return crop_median(c, ms);
}

// Columns x0..x0+3 of one row: grey bytes in G, depth u16 pairs in Z0
// (x0, x0+1) and Z1 (x0+2, x0+3). With `full` the 4 columns are loaded as is
// (columns past the crop are never used); otherwise they are clamped to w-1.
struct RawRow {
    uint32_t G, Z0, Z1;
};

__device__ __forceinline__ RawRow load_row(const CropDesc &c, int y, int x0, bool full) {
    RawRow r;
    if (full) {
        r.G = gld<uint32_t>(c.grey, (uint32_t)y * (uint32_t)c.grey_pitch + (uint32_t)x0);
        const u32x2 z =
            gld<u32x2>(c.depth, ((uint32_t)y * (uint32_t)c.depth_pitch + (uint32_t)x0) * 2u);
        r.Z0 = z.x;
        r.Z1 = z.y;
    } else {
        const uint8_t *grow = c.grey + (size_t)y * c.grey_pitch;
        const uint16_t *drow = c.depth + (size_t)y * c.depth_pitch;
        const int xa = min(x0, c.w - 1), x1 = min(x0 + 1, c.w - 1), x2 = min(x0 + 2, c.w - 1),
                  x3 = min(x0 + 3, c.w - 1);
        r.G = (uint32_t)grow[xa] | ((uint32_t)grow[x1] << 8) | ((uint32_t)grow[x2] << 16) |
              ((uint32_t)grow[x3] << 24);
        r.Z0 = (uint32_t)drow[xa] | ((uint32_t)drow[x1] << 16);
        r.Z1 = (uint32_t)drow[x2] | ((uint32_t)drow[x3] << 16);
    }
    return r;
}

// d' = 0 for d == 0, else clamp(d - lo, 0, span), on a pair of u16.
__device__ __forceinline__ uint32_t to_window(uint32_t z, int32_t lo, uint32_t lolo, uint32_t span2) {
    if (lo >= 0) return pk_min(pk_sub_sat(z, lolo), span2);
    const uint32_t a = z & 0xFFFFu, b = z >> 16;
    const int32_t span = (int32_t)(span2 & 0xFFFFu);
    const uint32_t da = a ? (uint32_t)min((int32_t)a - lo, span) : 0u;
    const uint32_t db = b ? (uint32_t)min((int32_t)b - lo, span) : 0u;
    return da | (db << 16);
}

// Row of 6 packed pixels (grey | d' << 16): columns [x0-1, x0 .. x0+3, x0+4].
struct Row6 {
    uint32_t p[6];
};

__device__ __forceinline__ Row6 make_row(const RawRow &raw, int32_t lo, uint32_t lolo,
                                         uint32_t span2) {
    const uint32_t D0 = to_window(raw.Z0, lo, lolo, span2);
    const uint32_t D1 = to_window(raw.Z1, lo, lolo, span2);
    Row6 r;
    r.p[1] = __builtin_amdgcn_perm(raw.G, D0, 0x01000C04u);
    r.p[2] = __builtin_amdgcn_perm(raw.G, D0, 0x03020C05u);
    r.p[3] = __builtin_amdgcn_perm(raw.G, D1, 0x01000C06u);
    r.p[4] = __builtin_amdgcn_perm(raw.G, D1, 0x03020C07u);
    // Left halo = previous lane's last pixel, right halo = next lane's first.
    r.p[0] = __builtin_amdgcn_update_dpp(0u, r.p[4], 0x138, 0xF, 0xF, false);  // wave_shr:1
    r.p[5] = __builtin_amdgcn_update_dpp(0u, r.p[1], 0x130, 0xF, 0xF, false);  // wave_shl:1
    return r;
}

// Comparison bits of the centre B[j] against its 8 neighbours in rows A
// (y-1), B (y), C (y+1): grey bit of neighbour p at 8+p, depth bit of
// neighbour p at 25+p (p < 7) and of p7 at 24. A set bit means the
// neighbour is BELOW the centre. For a negative 16-bit difference every bit
// from 8 (grey, |diff| < 256) or 9 (depth, |diff| < 512) up is set.
__device__ __forceinline__ uint32_t compare_bits(const Row6 &A, const Row6 &B, const Row6 &C, int j) {
    const uint32_t c = B.p[j];
    // All eight differences first: a packed result read by the very next
    // instruction costs a wait state on gfx950.
    const uint32_t d0 = pk_sub(A.p[j - 1], c), d1 = pk_sub(A.p[j], c), d2 = pk_sub(A.p[j + 1], c);
    const uint32_t d3 = pk_sub(B.p[j + 1], c), d4 = pk_sub(C.p[j + 1], c), d5 = pk_sub(C.p[j], c);
    const uint32_t d6 = pk_sub(C.p[j - 1], c), d7 = pk_sub(B.p[j - 1], c);
    uint32_t acc = d0 & 0x02000100u;
    acc = and_or(d1, 0x04000200u, acc);
    acc = and_or(d2, 0x08000400u, acc);
    acc = and_or(d3, 0x10000800u, acc);
    acc = and_or(d4, 0x20001000u, acc);
    acc = and_or(d5, 0x40002000u, acc);
    acc = and_or(d6, 0x80004000u, acc);
    acc = and_or(d7, 0x00008000u, acc);
    acc = and_or(d7 >> 7, 0x01000000u, acc);
    return acc;
}

// LDS of the fast path; 38.7 KB, so four workgroups fit a CU.
struct FastShared {
    // fp.dim = 2 * cells * 59 counters, then 64 per-lane discard slots.
    __attribute__((aligned(16))) uint32_t hist[2 * 64 * kU59 + 64];
    MedianScratch ms;
    uint8_t bin[256];    // code -> bin
    uint8_t lut_g[256];  // grey comparison byte -> bin
    uint8_t lut_d[256];  // depth comparison byte -> bin
    uint8_t rowband[LBPF_MAX_SIDE];
    uint8_t colband[LBPF_MAX_SIDE];
    float q[kQuot];
    uint32_t red[2 * kWaves];
    int32_t next;
};

__device__ __forceinline__ void load_tables(FastShared &sh, const uint8_t *tables) {
    for (int i = threadIdx.x; i < 256; i += kThreads) {
        sh.bin[i] = tables[i];
        sh.lut_g[i] = tables[256 + i];
        sh.lut_d[i] = tables[512 + i];
    }
}

// Features of one crop by the whole workgroup: row `out` (and `cout` when
// not null) of length fp.dim. The tables must already be in LDS; the caller
// separates consecutive crops with a barrier. kPF = rows loaded ahead.
template <int kPF, bool kEarly>
__device__ void fast_crop(const CropDesc &c, const FeatParams &fp, FastShared &sh, float *out,
                          uint32_t *cout) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int w = c.w, h = c.h;
    const int gx = fp.grid_x, gy = fp.grid_y, cells = gx * gy;
    const int dim = fp.dim;

    for (int i = tid; i < dim + 64; i += kThreads) sh.hist[i] = 0;
    // Coordinate y lies in band floor(((y + 1) g - 1) / n) of a side of length n.
    for (int y = tid; y < h; y += kThreads) sh.rowband[y] = (uint8_t)(((y + 1) * gy - 1) / h);
    for (int x = tid; x < w; x += kThreads) sh.colband[x] = (uint8_t)(((x + 1) * gx - 1) / w);

    // Stream geometry of the code phase. Its first rows do not depend on the
    // median: with kEarly their loads are issued now and land while the
    // median is computed (at the price of registers held across it).
    const bool fast = w <= kFastMaxW;
    const int L = (w + 3) >> 2;           // lanes per stream (<= 64 when fast)
    const int spw = fast ? 64 / L : 1;    // streams per wave
    const int sw = lane / L;              // stream of this lane within the wave
    const int x0 = 4 * (lane - sw * L);
    const int S = kWaves * spw;
    const int s = wave * spw + (sw < spw ? sw : 0);
    const int rows = h - 2;
    const int yb = 1 + (s * rows) / S;
    const int ye = (fast && sw < spw) ? 1 + ((s + 1) * rows) / S : yb;
    const bool full = (c.flags & kCropOverReadOk) || x0 + 4 <= w;
    RawRow rawA, rawB, ring[kPF];
    auto prime = [&]() {
        rawA = load_row(c, yb - 1, x0, full);
        rawB = load_row(c, yb, x0, full);
#pragma unroll
        for (int u = 0; u < kPF; ++u) ring[u] = load_row(c, min(yb + 1 + u, h - 1), x0, full);
    };
    if (kEarly && yb < ye) prime();

    const int32_t m = crop_median_fast(c, sh.ms, sh.red);  // ends with a barrier

    if (fast) {
        if (m >= 0 && yb < ye) {
            if (!kEarly) prime();
            const int32_t lo = m - fp.window;
            const uint32_t lolo = (uint32_t)(lo & 0xFFFF) * 0x10001u;
            const uint32_t span2 = (uint32_t)(2 * fp.window) * 0x10001u;
            const uint32_t in_hi = (uint32_t)(2 * fp.window - 1) << 16;

            // Per column: histogram column offset (bytes) and in-window
            // threshold (0 for border or out-of-crop columns: never counted).
            uint32_t col4[4], thr[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int x = x0 + k;
                col4[k] = (uint32_t)(sh.colband[min(x, w - 1)] * kU59) * 4u;
                thr[k] = (x >= 1 && x <= w - 2) ? in_hi : 0u;
            }
            const uint32_t dep4 = (uint32_t)(cells * kU59) * 4u;
            char *hbase = reinterpret_cast<char *>(sh.hist);

            Row6 A = make_row(rawA, lo, lolo, span2);
            Row6 B = make_row(rawB, lo, lolo, span2);
            for (int y = yb; y < ye; y += kPF) {
#pragma unroll
                for (int u = 0; u < kPF; ++u) {
                    const int yy = y + u;
                    if (yy >= ye) break;
                    const Row6 C = make_row(ring[u], lo, lolo, span2);
                    ring[u] = load_row(c, min(yy + 1 + kPF, h - 1), x0, full);
                    const uint32_t row4 = (uint32_t)(sh.rowband[yy] * gx * kU59) * 4u;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t bits = compare_bits(A, B, C, k + 1);
                        if (B.p[k + 1] - 0x10000u < thr[k]) {
                            const uint32_t base = row4 + col4[k];
                            const uint32_t bg = sh.lut_g[(bits >> 8) & 0xFFu];
                            const uint32_t bd = sh.lut_d[bits >> 24];
                            atomicAdd(reinterpret_cast<uint32_t *>(hbase + base + 4u * bg), 1u);
                            atomicAdd(reinterpret_cast<uint32_t *>(hbase + dep4 + base + 4u * bd), 1u);
                        }
                    }
                    A = B;
                    B = C;
                }
            }
        }
    } else {
        lbp_hist_generic(c, fp, m, sh.bin, sh.rowband, sh.colband, sh.hist);
    }
    __syncthreads();

    // n_in = total of the grey half; T = 2 n_in.
    uint32_t part = 0;
    for (int i = tid; i < cells * kU59; i += kThreads) part += sh.hist[i];
    part = wave_sum(part);
    if (lane == 0) sh.red[wave] = part;
    __syncthreads();
    uint32_t n_in = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) n_in += sh.red[i];
    const float T = (float)(2u * n_in);
    const int maxc = ((h + gy - 1) / gy) * ((w + gx - 1) / gx);  // cell capacity bound
    const bool tab = maxc < kQuot;
    if (tab) {
        for (int v = tid; v <= maxc; v += kThreads) sh.q[v] = n_in ? (float)v / T : 0.0f;
        __syncthreads();
    }
    const bool vec = (dim & 3) == 0 && ((uintptr_t)out & 15) == 0 && ((uintptr_t)cout & 15) == 0;
    if (vec && tab) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        for (int i = 4 * tid; i < dim; i += 4 * kThreads) {
            const u32x4 v = *reinterpret_cast<const u32x4 *>(&sh.hist[i]);
            const f32x4 f = {sh.q[v.x], sh.q[v.y], sh.q[v.z], sh.q[v.w]};
            *reinterpret_cast<f32x4 *>(out + i) = f;
            if (cout) *reinterpret_cast<u32x4 *>(cout + i) = v;
        }
    } else {
        for (int i = tid; i < dim; i += kThreads) {
            const uint32_t v = sh.hist[i];
            out[i] = tab ? sh.q[v] : (n_in ? (float)v / T : 0.0f);
            if (cout) cout[i] = v;
        }
    }
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
__global__ __launch_bounds__(kThreads) void k_features_persistent(
    const CropDesc *__restrict__ crops, const int32_t *__restrict__ order, int32_t n,
    FeatParams fp, const uint8_t *__restrict__ tables, float *__restrict__ hist,
    uint32_t *__restrict__ counts, uint32_t *__restrict__ queue) {
    __shared__ FastShared sh;
    load_tables(sh, tables);
    for (;;) {
        if (threadIdx.x == 0) sh.next = (int32_t)atomicAdd(&queue[0], 1u);
        __syncthreads();
        const int32_t j = sh.next;
        if (j >= n) break;  // uniform: every thread read the same j
        const size_t i = order ? (size_t)order[j] : (size_t)j;
        fast_crop<kPF, false>(crops[i], fp, sh, hist + i * fp.dim, counts ? counts + i * fp.dim : nullptr);
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
    return fp.nbins == kU59 && fp.use_grey && fp.use_depth && fp.window >= 1 &&
           fp.window <= 255 && fp.grid_x * fp.grid_y <= 64;
}

hipError_t launch_features(const CropDesc *crops, int32_t n, const FeatParams &fp,
                           const uint8_t *d_tables, float *hist, uint32_t *counts,
                           hipStream_t s, const LaunchCfg &lc, const int32_t *order,
                           uint32_t *queue, int32_t num_cus) {
    if (n <= 0) return hipSuccess;
    if (fast_path_ok(fp)) {
        const int pf = lc.row_prefetch <= 2 ? 2 : (lc.row_prefetch <= 4 ? 4 : 8);
        if (lc.persistent && queue) {
            const int grid = std::min<int>(n, std::max(1, lc.wg_per_cu) * num_cus);
            const int32_t *ord = lc.sorted ? order : nullptr;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, crops, ord, n, fp,
                                   d_tables, hist, counts, queue);
            };
            if (pf == 2) go(k_features_persistent<2>);
            else if (pf == 4) go(k_features_persistent<4>);
            else go(k_features_persistent<8>);
        } else {
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
