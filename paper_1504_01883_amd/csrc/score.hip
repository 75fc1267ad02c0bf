// SVM decision values S = X W^T + b on gfx950 matrix cores, and the per-row
// argmax (Sec. 2.5: one hyperplane per enrolled person, the largest decision
// value names the person).
//
// FP32 path: v_mfma_f32_16x16x4f32. A workgroup of 4 wave64 owns a 64 x 64
// tile of S (64 crops x 64 identities); each wave owns a 32 x 32 sub-tile as
// 2 x 2 MFMA blocks. Operands go straight from global memory (L2) into VGPRs
// as float4: lane l loads row (l % 16) of a block at columns d0 + 4 (l / 16)
// .. +3, and MFMA c (c = 0..3) consumes component c, so the four MFMAs of a
// step cover 16 consecutive d exactly once for both operands.
#include "lbpf_internal.h"

namespace lbpf {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;

template <bool kVec>
__device__ __forceinline__ floatx4 load_frag(const float *__restrict__ base, int32_t row,
                                             int32_t nrows, int32_t D, int32_t d) {
    floatx4 v = {0.f, 0.f, 0.f, 0.f};
    if (row < nrows) {
        const float *p = base + (size_t)row * D + d;
        if (kVec) {
            if (d + 3 < D) {
                v = *reinterpret_cast<const floatx4 *>(p);
            }
        } else {
            if (d + 0 < D) v.x = p[0];
            if (d + 1 < D) v.y = p[1];
            if (d + 2 < D) v.z = p[2];
            if (d + 3 < D) v.w = p[3];
        }
    }
    return v;
}

template <bool kVec>
__global__ __launch_bounds__(256) void k_score_f32(const float *__restrict__ X, int32_t N,
                                                   const float *__restrict__ W,
                                                   const float *__restrict__ bias, int32_t K,
                                                   int32_t D, float *__restrict__ S) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int32_t n0 = blockIdx.x * kTile + (wave >> 1) * 32;
    const int32_t k0 = blockIdx.y * kTile + (wave & 1) * 32;

    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    floatx4 xa[2], wb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) xa[i] = load_frag<kVec>(X, n0 + 16 * i + r, N, D, 4 * q);
#pragma unroll
    for (int j = 0; j < 2; ++j) wb[j] = load_frag<kVec>(W, k0 + 16 * j + r, K, D, 4 * q);

    for (int32_t d0 = 0; d0 < D; d0 += 16) {
        floatx4 xn[2], wn[2];
        const int32_t dn = d0 + 16 + 4 * q;
#pragma unroll
        for (int i = 0; i < 2; ++i) xn[i] = load_frag<kVec>(X, n0 + 16 * i + r, N, D, dn);
#pragma unroll
        for (int j = 0; j < 2; ++j) wn[j] = load_frag<kVec>(W, k0 + 16 * j + r, K, D, dn);
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[i][c], wb[j][c],
                                                                     acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 2; ++i) xa[i] = xn[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) wb[j] = wn[j];
    }

    // Lane l holds S[n0 + 16 i + 4 q + t][k0 + 16 j + r] in acc[i][j][t].
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int32_t k = k0 + 16 * j + r;
        if (k >= K) continue;
        const float bk = bias[k];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int32_t n = n0 + 16 * i + 4 * q + t;
                if (n < N) S[(size_t)n * K + k] = acc[i][j][t] + bk;
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
        hipLaunchKernelGGL(k_score_f32<true>, grid, dim3(256), 0, s, X, N, W, b, K, D, S);
    else
        hipLaunchKernelGGL(k_score_f32<false>, grid, dim3(256), 0, s, X, N, W, b, K, D, S);
    return hipGetLastError();
}

hipError_t launch_argmax(const float *S, int32_t N, int32_t K, int32_t *argmax, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_argmax, dim3((N + 3) / 4), dim3(256), 0, s, S, N, K, argmax);
    return hipGetLastError();
}

}  // namespace lbpf
