// Fused depth-masked LBP + regional histogram + L1 normalisation, gfx950.
//
// One workgroup (4 wave64) per face crop. Steps, all inside one launch:
//   1. exact lower median of the crop's non-zero depth by a two-level radix
//      select (high byte, then low byte) over 256-bin LDS histograms;
//   2. for every interior pixel inside the depth window, the 3x3 LBP code of
//      the grey and of the depth plane (Sec. 2.4, Eq. 2; p0 = top-left
//      neighbour, clockwise, bit set when neighbour >= centre);
//   3. code -> bin through a 256-entry LDS table (uniform-59 or identity);
//   4. increments of the [channel][ry][rx][bin] histogram, kept in LDS;
//   5. the row written once to HBM as count / T (IEEE single division) and,
//      optionally, as raw counts.
#include "lbpf_internal.h"

namespace lbpf {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Neighbour p of the centre (y, x) is (y + kDy[p], x + kDx[p]).
__constant__ int8_t kDy[8] = {-1, -1, -1, 0, 1, 1, 1, 0};
__constant__ int8_t kDx[8] = {-1, 0, 1, 1, 1, 0, -1, -1};

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Given a 256-bin histogram in LDS and a 0-based rank, find the bin holding
// that rank and the rank inside the bin. Runs on wave 0 only.
__device__ __forceinline__ void select_bin(const uint32_t *h, uint32_t rank, int lane,
                                           int32_t *out_bin, uint32_t *out_rank,
                                           uint32_t *out_total) {
    uint32_t c0 = h[4 * lane + 0], c1 = h[4 * lane + 1], c2 = h[4 * lane + 2],
             c3 = h[4 * lane + 3];
    uint32_t s = c0 + c1 + c2 + c3;
    uint32_t incl = wave_inclusive_scan(s, lane);
    uint32_t excl = incl - s;
    uint32_t total = __shfl(incl, 63, 64);
    if (lane == 0) *out_total = total;
    if (rank < total && excl <= rank && rank < incl) {
        uint32_t r = rank - excl;
        int b = 4 * lane;
        if (r >= c0) { r -= c0; b += 1;
            if (r >= c1) { r -= c1; b += 1;
                if (r >= c2) { r -= c2; b += 1; } } }
        *out_bin = b;
        *out_rank = r;
    }
}

struct MedianScratch {
    uint32_t hist[256];
    int32_t bin;
    uint32_t rank;
    uint32_t total;
};

// Exact lower median of the non-zero depth of the crop, or -1 when every
// depth pixel is 0. All threads of the block must call it.
__device__ int32_t crop_median(const CropDesc &c, MedianScratch &ms) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    __syncthreads();
    for (int y = wave; y < c.h; y += kWaves) {
        const uint16_t *row = c.depth + (size_t)y * c.depth_pitch;
        for (int x = lane; x < c.w; x += 64) {
            uint32_t d = row[x];
            if (d != 0) atomicAdd(&ms.hist[d >> 8], 1u);
        }
    }
    __syncthreads();
    if (wave == 0) {
        // rank (n-1)/2 of the non-zero values; the total is found in the scan.
        uint32_t s = ms.hist[4 * lane] + ms.hist[4 * lane + 1] + ms.hist[4 * lane + 2] +
                     ms.hist[4 * lane + 3];
        uint32_t tot = s;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) tot += __shfl_xor(tot, off, 64);
        if (lane == 0) ms.bin = -1;
        if (tot > 0) select_bin(ms.hist, (tot - 1) / 2, lane, &ms.bin, &ms.rank, &ms.total);
    }
    __syncthreads();
    const int32_t hi = ms.bin;
    if (hi < 0) return -1;
    const uint32_t rank_in_hi = ms.rank;
    __syncthreads();
    for (int i = tid; i < 256; i += kThreads) ms.hist[i] = 0;
    __syncthreads();
    for (int y = wave; y < c.h; y += kWaves) {
        const uint16_t *row = c.depth + (size_t)y * c.depth_pitch;
        for (int x = lane; x < c.w; x += 64) {
            uint32_t d = row[x];
            if (d != 0 && (int32_t)(d >> 8) == hi) atomicAdd(&ms.hist[d & 255u], 1u);
        }
    }
    __syncthreads();
    if (wave == 0) select_bin(ms.hist, rank_in_hi, lane, &ms.bin, &ms.rank, &ms.total);
    __syncthreads();
    int32_t m = (hi << 8) | ms.bin;
    __syncthreads();
    return m;
}

__device__ __forceinline__ bool centre_in_mask(uint32_t d, int32_t m, int32_t window) {
    if (window <= 0) return true;
    if (m < 0 || d == 0) return false;
    int32_t diff = (int32_t)d - m;
    return diff < window && -diff < window;
}

template <typename T>
__device__ __forceinline__ uint32_t lbp_code(const T *p, int32_t pitch, int y, int x) {
    const uint32_t c = p[(size_t)y * pitch + x];
    uint32_t code = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint32_t g = p[(size_t)(y + kDy[k]) * pitch + (x + kDx[k])];
        code |= (g >= c ? 1u : 0u) << k;
    }
    return code;
}

__global__ __launch_bounds__(kThreads) void k_features_v1(const CropDesc *__restrict__ crops,
                                                          FeatParams fp,
                                                          const uint8_t *__restrict__ bin_table,
                                                          float *__restrict__ hist,
                                                          uint32_t *__restrict__ counts) {
    extern __shared__ uint32_t sh_hist[];  // fp.dim counters
    __shared__ MedianScratch ms;
    __shared__ uint8_t sh_bin[256];
    __shared__ uint8_t sh_rowband[LBPF_MAX_SIDE];
    __shared__ uint8_t sh_colband[LBPF_MAX_SIDE];
    __shared__ uint32_t sh_nin[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const CropDesc c = crops[blockIdx.x];

    for (int i = tid; i < fp.dim; i += kThreads) sh_hist[i] = 0;
    for (int i = tid; i < 256; i += kThreads) sh_bin[i] = bin_table[i];
    // Band of each row/column: band r covers [floor(r n / g), floor((r+1) n / g)),
    // so coordinate y lies in band floor(((y + 1) g - 1) / n).
    for (int y = tid; y < c.h; y += kThreads) sh_rowband[y] = (uint8_t)(((y + 1) * fp.grid_y - 1) / c.h);
    for (int x = tid; x < c.w; x += kThreads) sh_colband[x] = (uint8_t)(((x + 1) * fp.grid_x - 1) / c.w);

    const int32_t m = fp.window > 0 ? crop_median(c, ms) : -1;
    __syncthreads();

    const int cells = fp.grid_x * fp.grid_y;
    const int nb = fp.nbins;
    uint32_t n_in = 0;
    for (int y = 1 + wave; y <= c.h - 2; y += kWaves) {
        const int rowcell = sh_rowband[y] * fp.grid_x;
        for (int x = 1 + lane; x <= c.w - 2; x += 64) {
            uint32_t dc = c.depth[(size_t)y * c.depth_pitch + x];
            if (!centre_in_mask(dc, m, fp.window)) continue;
            n_in += 1;
            const int cell = rowcell + sh_colband[x];
            int ch = 0;
            if (fp.use_grey) {
                uint32_t code = lbp_code(c.grey, c.grey_pitch, y, x);
                atomicAdd(&sh_hist[cell * nb + sh_bin[code]], 1u);
                ch = 1;
            }
            if (fp.use_depth) {
                uint32_t code = lbp_code(c.depth, c.depth_pitch, y, x);
                atomicAdd(&sh_hist[(ch * cells + cell) * nb + sh_bin[code]], 1u);
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n_in += __shfl_xor(n_in, off, 64);
    if (lane == 0) sh_nin[wave] = n_in;
    __syncthreads();
    uint32_t total_in = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) total_in += sh_nin[w];
    const float T = (float)(fp.nch * total_in);

    float *out = hist + (size_t)blockIdx.x * fp.dim;
    uint32_t *cout = counts ? counts + (size_t)blockIdx.x * fp.dim : nullptr;
    for (int i = tid; i < fp.dim; i += kThreads) {
        uint32_t v = sh_hist[i];
        out[i] = total_in ? (float)v / T : 0.0f;
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
        int y = i / c.w, x = i % c.w;
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

hipError_t launch_features(const CropDesc *crops, int32_t n, const FeatParams &fp,
                           const uint8_t *d_bin_table, float *hist, uint32_t *counts,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t shmem = (size_t)fp.dim * sizeof(uint32_t);
    // Above 64 KiB of dynamic LDS (the 256-bin mapping) the kernel must opt in.
    static size_t shmem_limit = 64 * 1024;
    if (shmem > shmem_limit) {
        hipError_t e = hipFuncSetAttribute((const void *)k_features_v1,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)shmem);
        if (e != hipSuccess) return e;
        shmem_limit = shmem;
    }
    hipLaunchKernelGGL(k_features_v1, dim3(n), dim3(kThreads), shmem, s, crops, fp, d_bin_table,
                       hist, counts);
    return hipGetLastError();
}

hipError_t launch_debug_codes(const CropDesc *crop, const FeatParams &fp, uint8_t *gcodes,
                              uint8_t *dcodes, uint8_t *mask, int32_t, int32_t, hipStream_t s) {
    hipLaunchKernelGGL(k_debug_codes, dim3(1), dim3(kThreads), 0, s, crop, fp, gcodes, dcodes,
                       mask);
    return hipGetLastError();
}

}  // namespace lbpf
