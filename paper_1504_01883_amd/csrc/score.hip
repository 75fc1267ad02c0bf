// SVM decision values S = X W^T + b on gfx950 matrix cores, and the per-row
// argmax (Sec. 2.5: one hyperplane per enrolled person, the largest decision
// value names the person).
//
// FP32 path: v_mfma_f32_16x16x4f32 (D[m][n] += sum_k A[m][k] B[k][n] over a
// 16 x 16 x 4 block; lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// and receives D[4 (l / 16) + t][l % 16], t = 0..3). Operands go straight
// from global memory (L2) into VGPRs as float4: lane l loads row (l % 16) of
// a block at columns d0 + 4 (l / 16) .. +3, and MFMA c (c = 0..3) consumes
// component c, so four MFMAs cover 16 consecutive d exactly once for both
// operands.
#include "lbpf_internal.h"

namespace lbpf {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;

// Four consecutive operands d .. d+3 of row `row` (zeros past `nrows` rows or
// past `d_end`); `ld` is the row stride. kVec: 16-byte aligned rows and
// d_end a multiple of 4, so a quad is either fully inside or fully outside.
template <bool kVec>
__device__ __forceinline__ floatx4 load_frag(const float *__restrict__ base, int32_t row,
                                             int32_t nrows, int32_t d_end, int32_t d, int32_t ld) {
    floatx4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < nrows) {
        const float *p = base + (size_t)row * ld + d;
        if (kVec) {
            if (d + 3 < d_end) v = *reinterpret_cast<const floatx4 *>(p);
        } else {
            if (d + 0 < d_end) v.x = p[0];
            if (d + 1 < d_end) v.y = p[1];
            if (d + 2 < d_end) v.z = p[2];
            if (d + 3 < d_end) v.w = p[3];
        }
    }
    return v;
}

// A workgroup of 8 wave64 owns a 64 x 64 tile of S. Wave w computes rows
// 32 (w & 1) .. +32 of the tile over one quarter of the feature dimension
// (w >> 1), as 2 x 4 blocks of 16 x 16; the quarters are summed in a fixed
// order through LDS at the end. Two waves per SIMD hide each other's load
// latency. Each iteration covers 32 feature columns (2 sub-steps of
// 16) and the operands of the next iteration are loaded before the MFMAs of
// the current one are issued, so a global load has a full iteration of MFMA
// work (64 instructions) to land.
template <bool kVec>
__global__ __launch_bounds__(512) void k_score_f32(const float *__restrict__ X, int32_t N,
                                                   const float *__restrict__ W,
                                                   const float *__restrict__ bias, int32_t K,
                                                   int32_t D, float *__restrict__ S) {
    __shared__ floatx4 partial[3][2][2][4][64];  // [quarter-1][row half][i][j][lane]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int rh = wave & 1, kq = wave >> 1;
    const int32_t n0 = blockIdx.x * kTile + rh * 32;
    const int32_t k0 = blockIdx.y * kTile;
    const int32_t dq = ((D + 127) / 128) * 32;  // quarter length, a multiple of 32
    const int32_t d_begin = min(kq * dq, D);
    const int32_t d_end = min(d_begin + dq, D);

    floatx4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    // Operands of one 32-column iteration: [sub-step][block].
    floatx4 xa[2][2], wb[2][4];
    auto load_iter = [&](int32_t d, floatx4 (&xo)[2][2], floatx4 (&wo)[2][4]) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int32_t du = d + 16 * u + 4 * q;
#pragma unroll
            for (int i = 0; i < 2; ++i) xo[u][i] = load_frag<kVec>(X, n0 + 16 * i + r, N, d_end, du, D);
#pragma unroll
            for (int j = 0; j < 4; ++j) wo[u][j] = load_frag<kVec>(W, k0 + 16 * j + r, K, d_end, du, D);
        }
    };
    load_iter(d_begin, xa, wb);
    for (int32_t d0 = d_begin; d0 < d_end; d0 += 32) {
        floatx4 xn[2][2], wn[2][4];
        load_iter(d0 + 32, xn, wn);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[u][i][c], wb[u][j][c],
                                                                         acc[i][j], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int i = 0; i < 2; ++i) xa[u][i] = xn[u][i];
#pragma unroll
            for (int j = 0; j < 4; ++j) wb[u][j] = wn[u][j];
        }
    }

    // Waves of quarters 1..3 hand their sums to the quarter-0 wave of the same rows.
    if (kq > 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) partial[kq - 1][rh][i][j][lane] = acc[i][j];
    }
    __syncthreads();
    if (kq > 0) return;
    // Lane l holds S[n0 + 16 i + 4 q + t][k0 + 16 j + r] in acc[i][j][t].
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int32_t k = k0 + 16 * j + r;
        if (k >= K) continue;
        const float bk = bias[k];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const floatx4 s = ((acc[i][j] + partial[0][rh][i][j][lane]) +
                               partial[1][rh][i][j][lane]) + partial[2][rh][i][j][lane];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int32_t n = n0 + 16 * i + 4 * q + t;
                if (n < N) S[(size_t)n * K + k] = s[t] + bk;
            }
        }
    }
}

// One wave per row: lanes scan k = lane, lane + 64, ... keeping the first
// (lowest k) maximum, then a butterfly picks the larger value, or the lower
// index on equal values.
__global__ __launch_bounds__(256) void k_argmax(const float *__restrict__ S, int32_t N, int32_t K,
                                                int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int32_t n = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (n >= N) return;
    const float *row = S + (size_t)n * K;
    float best = -INFINITY;
    int32_t arg = K;  // larger than any valid index
    for (int32_t k = lane; k < K; k += 64) {
        float v = row[k];
        if (v > best || arg == K) {
            best = v;
            arg = k;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        float ob = __shfl_xor(best, off, 64);
        int32_t oa = __shfl_xor(arg, off, 64);
        if (ob > best || (ob == best && oa < arg)) {
            best = ob;
            arg = oa;
        }
    }
    if (lane == 0) out[n] = arg;
}

}  // namespace

hipError_t launch_score_f32(const float *X, int32_t N, const float *W, const float *b, int32_t K,
                            int32_t D, float *S, hipStream_t s) {
    if (N <= 0 || K <= 0) return hipSuccess;
    dim3 grid((N + kTile - 1) / kTile, (K + kTile - 1) / kTile);
    const bool vec = (D % 4 == 0) && ((uintptr_t)X % 16 == 0) && ((uintptr_t)W % 16 == 0);
    if (vec)
        hipLaunchKernelGGL(k_score_f32<true>, grid, dim3(512), 0, s, X, N, W, b, K, D, S);
    else
        hipLaunchKernelGGL(k_score_f32<false>, grid, dim3(512), 0, s, X, N, W, b, K, D, S);
    return hipGetLastError();
}

hipError_t launch_argmax(const float *S, int32_t N, int32_t K, int32_t *argmax, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_argmax, dim3((N + 3) / 4), dim3(256), 0, s, S, N, K, argmax);
    return hipGetLastError();
}

}  // namespace lbpf
