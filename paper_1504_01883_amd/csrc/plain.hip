// The plain, unbatched FP32 GPU path: the comparator the fused path is
// measured against. It computes the same results (bit-exact features, FP32
// scores) the straightforward way, one face at a time, as the paper's
// per-face GPU feature extraction did (Sec. 3): per crop
//   1. one workgroup finds the depth median (two-level radix select);
//   2. one thread per interior pixel computes both LBP codes and increments
//      the crop's histogram with global-memory atomics;
//   3. one thread per element normalises the counts into the feature row;
//   4. one wave per identity computes its decision value (a GEMV), and one
//      wave takes the argmax.
// Five launches per crop, no shared memory beyond the median's.
#include "lbpf_internal.h"

namespace lbpf {

namespace {

constexpr int kThreads = 256;

__constant__ int8_t kPDy[8] = {-1, -1, -1, 0, 1, 1, 1, 0};
__constant__ int8_t kPDx[8] = {-1, 0, 1, 1, 1, 0, -1, -1};

template <typename T>
__device__ __forceinline__ uint32_t plain_code(const T *p, int32_t pitch, int y, int x) {
    const uint32_t c = p[(size_t)y * pitch + x];
    uint32_t code = 0;
    for (int k = 0; k < 8; ++k) {
        const uint32_t g = p[(size_t)(y + kPDy[k]) * pitch + (x + kPDx[k])];
        if (g >= c) code |= 1u << k;
    }
    return code;
}

// Median by a two-level radix select over 256-bin shared histograms; the
// bin holding the rank is found by one wave with a prefix scan.
__device__ __forceinline__ void plain_select(const uint32_t *h, uint32_t rank, int32_t *sel,
                                             uint32_t *sel_rank) {
    const int lane = threadIdx.x;
    uint32_t c[4], s = 0;
    for (int j = 0; j < 4; ++j) {
        c[j] = h[4 * lane + j];
        s += c[j];
    }
    uint32_t incl = s;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    uint32_t acc = incl - s;
    if (lane == 0) *sel = -1;
    if (acc <= rank && rank < incl) {
        for (int j = 0; j < 4; ++j) {
            if (rank < acc + c[j]) {
                *sel = 4 * lane + j;
                *sel_rank = rank - acc;
                break;
            }
            acc += c[j];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_plain_median(CropDesc c, int32_t *median) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t total;
    __shared__ int32_t sel;
    __shared__ uint32_t sel_rank;
    const int tid = threadIdx.x;
    int32_t hi = -1;
    uint32_t rank = 0;
    for (int level = 0; level < 2; ++level) {
        h[tid] = 0;
        if (tid == 0) total = 0;
        __syncthreads();
        uint32_t nz = 0;
        for (int y = 0; y < c.h; ++y)
            for (int x = tid; x < c.w; x += kThreads) {
                const uint32_t d = c.depth[(size_t)y * c.depth_pitch + x];
                if (d == 0) continue;
                nz += 1;
                if (level == 0) atomicAdd(&h[d >> 8], 1u);
                else if ((int32_t)(d >> 8) == hi) atomicAdd(&h[d & 255u], 1u);
            }
        if (level == 0) atomicAdd(&total, nz);
        __syncthreads();
        if (tid < 64) plain_select(h, level == 0 ? (total ? (total - 1) / 2 : 1u << 31) : rank, &sel,
                                   &sel_rank);
        __syncthreads();
        if (level == 0) {
            hi = sel;
            rank = sel_rank;
            if (hi < 0) break;
        }
        __syncthreads();
    }
    if (tid == 0) *median = hi < 0 ? -1 : (hi << 8) | sel;
}

__global__ __launch_bounds__(kThreads) void k_plain_hist(CropDesc c, FeatParams fp,
                                                         const uint8_t *bin_table,
                                                         const int32_t *median,
                                                         uint32_t *counts) {
    const int iw = c.w - 2, ih = c.h - 2;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= iw * ih) return;
    const int y = 1 + i / iw, x = 1 + i % iw;
    const int32_t m = *median;
    const uint32_t d = c.depth[(size_t)y * c.depth_pitch + x];
    if (fp.window > 0) {
        if (m < 0 || d == 0) return;
        const int32_t diff = (int32_t)d - m;
        if (!(diff < fp.window && -diff < fp.window)) return;
    }
    const int ry = ((y + 1) * fp.grid_y - 1) / c.h, rx = ((x + 1) * fp.grid_x - 1) / c.w;
    const int cell = ry * fp.grid_x + rx, cells = fp.grid_x * fp.grid_y;
    int ch = 0;
    if (fp.use_grey) {
        atomicAdd(&counts[cell * fp.nbins + bin_table[plain_code(c.grey, c.grey_pitch, y, x)]], 1u);
        ch = 1;
    }
    if (fp.use_depth)
        atomicAdd(&counts[(ch * cells + cell) * fp.nbins +
                          bin_table[plain_code(c.depth, c.depth_pitch, y, x)]],
                  1u);
}

// T = channels * n_in = the sum of all counts; one block sums, all divide.
__global__ __launch_bounds__(kThreads) void k_plain_normalise(const uint32_t *counts, int32_t dim,
                                                              float *row) {
    __shared__ uint32_t part[kThreads];
    uint32_t s = 0;
    for (int i = threadIdx.x; i < dim; i += kThreads) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    const uint32_t T = part[0];
    for (int i = threadIdx.x; i < dim; i += kThreads)
        row[i] = T ? (float)counts[i] / (float)T : 0.0f;
}

// One wave per identity: lanes stride over the row (coalesced), then a
// butterfly sum.
__global__ __launch_bounds__(kThreads) void k_plain_gemv(const float *x, const float *W,
                                                         const float *b, int32_t K, int32_t D,
                                                         float *s) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (k >= K) return;
    const float *w = W + (size_t)k * D;
    float acc = 0.0f;
    for (int d = lane; d < D; d += 64) acc = fmaf(w[d], x[d], acc);
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) s[k] = acc + b[k];
}

__global__ __launch_bounds__(64) void k_plain_argmax(const float *s, int32_t K, int32_t *out) {
    float best = -INFINITY;
    int32_t arg = K;
    for (int32_t k = threadIdx.x; k < K; k += 64) {
        if (s[k] > best || arg == K) {
            best = s[k];
            arg = k;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int32_t oa = __shfl_xor(arg, off, 64);
        if (ob > best || (ob == best && oa < arg)) {
            best = ob;
            arg = oa;
        }
    }
    if (threadIdx.x == 0) *out = arg;
}

}  // namespace

hipError_t launch_plain_features(const CropDesc &c, const FeatParams &fp, const uint8_t *bins,
                                 int32_t *median_scratch, uint32_t *counts, float *row,
                                 hipStream_t s) {
    hipError_t e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * fp.dim, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plain_median, dim3(1), dim3(kThreads), 0, s, c, median_scratch);
    const int interior = (c.w - 2) * (c.h - 2);
    hipLaunchKernelGGL(k_plain_hist, dim3((interior + kThreads - 1) / kThreads), dim3(kThreads), 0,
                       s, c, fp, bins, median_scratch, counts);
    hipLaunchKernelGGL(k_plain_normalise, dim3(1), dim3(kThreads), 0, s, counts, fp.dim, row);
    return hipGetLastError();
}

hipError_t launch_plain_score(const float *x, const float *W, const float *b, int32_t K,
                              int32_t D, float *scores, int32_t *argmax, hipStream_t s) {
    const int per_block = kThreads / 64;
    hipLaunchKernelGGL(k_plain_gemv, dim3((K + per_block - 1) / per_block), dim3(kThreads), 0, s,
                       x, W, b, K, D, scores);
    if (argmax) hipLaunchKernelGGL(k_plain_argmax, dim3(1), dim3(64), 0, s, scores, K, argmax);
    return hipGetLastError();
}

}  // namespace lbpf
