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

// --- FP32, LDS ring --------------------------------------------------------------
//
// For D a multiple of 32 and 16-byte aligned operands. A workgroup of 8 waves
// owns a 64 x 64 tile of S; waves 0-3 take the first half of the feature
// dimension and waves 4-7 the second (two waves per SIMD), and wave t of a
// half computes the 32 x 32 block (rows 32 (t & 1), columns 32 (t >> 1)) with
// v_mfma_f32_32x32x2f32 (lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32];
// D: register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32).
// Each half streams 64-byte slices of its 64 X rows and 64 W rows through a
// ring of kRing LDS stages with global_load_lds_dwordx4 (wave t copies 32 rows
// of X (t < 2) or W (t >= 2), two 1 KB instructions per stage), issued
// kRing - 1 stages ahead; each stage's fragments are read into registers one
// stage before they are multiplied, so the MFMAs after a barrier never wait
// for LDS. Chunk c (16 bytes) of row r sits at position
// c ^ ((r >> 1) & 3) of the row so that fragment reads of 8 consecutive rows
// hit 8 bank groups. A lane reads a 16-byte chunk (4 consecutive d) of its
// row and feeds its components to 4 MFMAs: step s pairs d = 4 q + s of lanes
// with l / 32 = q, so every d of the slice is used once by both operands.
// At the end the second half's blocks go through LDS and are added to the
// first half's in a fixed order, then the bias.

constexpr int kRing = 8;
constexpr int kSliceB = 64;                        // bytes per row and stage
constexpr int kHalfStage = 2 * 64 * kSliceB;       // X rows then W rows: 8 KB

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void glb_void_t;
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int kVm>
__device__ __forceinline__ void wait_vm() {
    static_assert(kVm >= 0 && kVm < 64, "vmcnt range");
    // gfx9 s_waitcnt: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8], vmcnt[15:14].
    __builtin_amdgcn_s_waitcnt((kVm & 15) | (7 << 4) | (15 << 8) | ((kVm >> 4) << 14));
}

// Wait until at most 2 * `younger` of this wave's copies are in flight.
__device__ __forceinline__ void wait_stage(int younger) {
    switch (younger) {
        case 0: wait_vm<0>(); break;
        case 1: wait_vm<2>(); break;
        case 2: wait_vm<4>(); break;
        case 3: wait_vm<6>(); break;
        case 4: wait_vm<8>(); break;
        case 5: wait_vm<10>(); break;
        default: wait_vm<12>(); break;
    }
}

// Barrier that orders LDS only: this wave's LDS reads have returned
// (lgkmcnt 0) before it arrives. __syncthreads would also drain the copies of
// the stages still in flight.
__device__ __forceinline__ void barrier_lds() {
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ int fswz(int row, int chunk) { return chunk ^ ((row >> 1) & 3); }

__global__ __launch_bounds__(512) void k_score_f32_ring(const float *__restrict__ X, int32_t N,
                                                        const float *__restrict__ W,
                                                        const float *__restrict__ bias,
                                                        int32_t K, int32_t D,
                                                        float *__restrict__ S) {
    __shared__ __attribute__((aligned(1024))) uint8_t lds[2 * kRing * kHalfStage];  // 128 KB
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int half = wave >> 2, t = wave & 3;
    const int32_t n0 = blockIdx.x * kTile, k0 = blockIdx.y * kTile;
    const int32_t dh = D / 2;
    const int nst = dh / (kSliceB / 4);
    uint8_t *ring = lds + half * kRing * kHalfStage;

    // Copy role: 32 rows of X (t < 2) or W (t >= 2); lane i -> row i / 4 of
    // each 16-row kilobyte, position i % 4.
    const bool isx = t < 2;
    const float *mat = isx ? X : W;
    const int32_t lim = isx ? N : K, base = isx ? n0 : k0;
    const int rr = lane >> 2, pos = lane & 3;
    const float *src[2];
    int dst_off[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int row = (t & 1) * 32 + j * 16 + rr;  // 0..63 within X or W
        const int32_t g = min(base + row, lim - 1);
        src[j] = mat + (size_t)g * D + (size_t)half * dh + 4 * fswz(row, pos);
        dst_off[j] = (isx ? 0 : 64 * kSliceB) + ((t & 1) * 32 + j * 16) * kSliceB;
    }
    auto copy = [&](int st) {
        uint8_t *stage = ring + (st % kRing) * kHalfStage;
#pragma unroll
        for (int j = 0; j < 2; ++j)
            __builtin_amdgcn_global_load_lds((glb_void_t *)(src[j] + st * (kSliceB / 4)),
                                             (lds_void_t *)(stage + dst_off[j]), 16, 0, 0);
    };

    const int fr = lane & 31, fq = lane >> 5;
    const int ra = (t & 1) * 32 + fr, rb = (t >> 1) * 32 + fr;
    // Byte offsets of this lane's fragments within a stage, chunk pair c.
    int oa[2], ob[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        oa[c] = ra * kSliceB + 16 * fswz(ra, 2 * c + fq);
        ob[c] = 64 * kSliceB + rb * kSliceB + 16 * fswz(rb, 2 * c + fq);
    }
    auto read = [&](int st, floatx4 (&a)[2], floatx4 (&b)[2]) {
        const uint8_t *stage = ring + (st % kRing) * kHalfStage;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            a[c] = *reinterpret_cast<const floatx4 *>(stage + oa[c]);
            b[c] = *reinterpret_cast<const floatx4 *>(stage + ob[c]);
        }
    };
    // Four independent accumulator chains (chunk pair c, parity of the
    // component), interleaved so that an accumulator recurs only every fourth
    // MFMA of the wave; summed at the end.
    floatx16 acc4[4] = {{}, {}, {}, {}};
    auto mma = [&](const floatx4 (&a)[2], const floatx4 (&b)[2]) {
        acc4[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0].x, b[0].x, acc4[0], 0, 0, 0);
        acc4[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1].x, b[1].x, acc4[1], 0, 0, 0);
        acc4[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0].y, b[0].y, acc4[2], 0, 0, 0);
        acc4[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1].y, b[1].y, acc4[3], 0, 0, 0);
        acc4[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0].z, b[0].z, acc4[0], 0, 0, 0);
        acc4[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1].z, b[1].z, acc4[1], 0, 0, 0);
        acc4[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0].w, b[0].w, acc4[2], 0, 0, 0);
        acc4[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1].w, b[1].w, acc4[3], 0, 0, 0);
    };
    // Iteration st: make stage st + 1 visible, start the copy of stage
    // st + kRing - 1 (into the buffer stage st - 1 used, whose fragments were
    // read an iteration earlier), read stage st + 1's fragments, multiply stage
    // st's (read during the previous iteration).
    // Called for st + 1 < nst only: the last stage is multiplied on its own,
    // so that no path without a barrier joins the steady-state loop (that
    // join would make the compiler wait for the fresh fragment reads).
    auto step = [&](int st, const floatx4 (&ca)[2], const floatx4 (&cb)[2], floatx4 (&na)[2],
                    floatx4 (&nb)[2]) {
        wait_stage(min(nst - 2 - st, kRing - 3));
        barrier_lds();
        if (st + kRing - 1 < nst) copy(st + kRing - 1);
        read(st + 1, na, nb);
        mma(ca, cb);
    };
#pragma unroll
    for (int st = 0; st < kRing - 1; ++st)
        if (st < nst) copy(st);
    floatx4 a0[2], b0[2], a1[2], b1[2];
    wait_stage(min(nst - 1, kRing - 2));
    barrier_lds();
    read(0, a0, b0);
    int st = 0;
    for (; st + 2 < nst; st += 2) {
        step(st, a0, b0, a1, b1);
        step(st + 1, a1, b1, a0, b0);
    }
    if (st + 1 < nst) {  // two stages left
        step(st, a0, b0, a1, b1);
        mma(a1, b1);
    } else {
        mma(a0, b0);
    }

    const floatx16 acc = (acc4[0] + acc4[1]) + (acc4[2] + acc4[3]);
    // Second half -> LDS -> added to the first half's block.
    __syncthreads();
    floatx16 *part = reinterpret_cast<floatx16 *>(lds);
    if (half == 1) part[t * 64 + lane] = acc;
    __syncthreads();
    if (half == 0) {
        const floatx16 o = part[t * 64 + lane];
        const int32_t k = k0 + (t >> 1) * 32 + (lane & 31);
        if (k < K) {
            const float bk = bias[k];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int32_t n = n0 + (t & 1) * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (n < N) S[(size_t)n * K + k] = (acc[r] + o[r]) + bk;
            }
        }
    }
}

}  // namespace

hipError_t launch_score_f32(const float *X, int32_t N, const float *W, const float *b, int32_t K,
                            int32_t D, float *S, hipStream_t s) {
    if (N <= 0 || K <= 0) return hipSuccess;
    dim3 grid((N + kTile - 1) / kTile, (K + kTile - 1) / kTile);
    const bool vec = (D % 4 == 0) && ((uintptr_t)X % 16 == 0) && ((uintptr_t)W % 16 == 0);
    if (vec && D % 32 == 0) {
        hipLaunchKernelGGL(k_score_f32_ring, grid, dim3(512), 0, s, X, N, W, b, K, D, S);
        return hipGetLastError();
    }
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
