// SVM decision values S = X W^T + b on gfx950 matrix cores, and the per-row
// argmax (Sec. 2.5: one hyperplane per enrolled person, the largest decision
// value names the person).
//
// FP32 paths:
//   * k_score_f32_split (D a multiple of 32 per split, 16-byte aligned rows):
//     128 x 128 tiles streamed through LDS, described at the kernel;
//   * k_score_f32 (any D): v_mfma_f32_16x16x4f32 (D[m][n] += sum_k A[m][k]
//     B[k][n] over a 16 x 16 x 4 block; lane l supplies A[l % 16][l / 16] and
//     B[l / 16][l % 16] and receives D[4 (l / 16) + t][l % 16], t = 0..3).
//     Operands go straight from global memory (L2) into VGPRs as float4: lane
//     l loads row (l % 16) of a block at columns d0 + 4 (l / 16) .. +3, and
//     MFMA c (c = 0..3) consumes component c, so four MFMAs cover 16
//     consecutive d exactly once for both operands.
#include "lbpf_internal.h"

#include <algorithm>

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
                                                int32_t *__restrict__ out,
                                                const int32_t *__restrict__ n_dev) {
    const int lane = threadIdx.x & 63;
    if (n_dev) N = *n_dev;
    const int32_t n = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (n >= N) return;
    const float *row = S + (size_t)n * K;
    float best = -INFINITY;
    int32_t arg = K;  // larger than any valid index
    if ((K & 3) == 0 && ((uintptr_t)S & 15) == 0) {
        // Four consecutive identities a lane per step (16-byte loads), still
        // scanned in increasing order within the lane.
        typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll 4
        for (int32_t k = 4 * lane; k < K; k += 256) {
            const f4 v = *reinterpret_cast<const f4 *>(row + k);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (v[e] > best || arg == K) {
                    best = v[e];
                    arg = k + e;
                }
        }
    } else {
        for (int32_t k = lane; k < K; k += 64) {
            float v = row[k];
            if (v > best || arg == K) {
                best = v;
                arg = k;
            }
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

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void glb_void_t;
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int kVm>
__device__ __forceinline__ void wait_vm() {
    static_assert(kVm >= 0 && kVm < 64, "vmcnt range");
    // gfx9 s_waitcnt: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8], vmcnt[15:14].
    __builtin_amdgcn_s_waitcnt((kVm & 15) | (7 << 4) | (15 << 8) | ((kVm >> 4) << 14));
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

// --- FP32, 128 x 128 tiles, split feature dimension --------------------------------
//
// A workgroup of 4 waves owns a 128 x 128 tile of S over one of `splits`
// equal ranges of the feature dimension; wave w computes the 64 x 64 quarter
// (rows 64 (w & 1), columns 64 (w >> 1)) as 2 x 2 blocks of 32 x 32 (four
// independent accumulator chains). 128-byte slices of the 128 X rows and 128
// W rows stream through a ring of kRingN 32 KB stages (global_load_lds; each
// wave copies 32 rows of each; chunk c of row r at position c ^ (r % 8)), and
// a stage's fragments are read one stage ahead. The barrier per stage orders
// LDS only (barrier_lds), so the copies of later stages stay in flight.
// With splits > 1 every workgroup stores its partial tile and k_reduce_argmax,
// queued after it on the same stream, adds the partials in split order and
// the bias (and takes the argmax in the same pass). (Reducing inside the kernel would need device-scope fences, which
// on this GPU write back and invalidate the XCD's L2 under the tiles still
// streaming through it.)

template <int kRingN, int kTK>
__global__ __launch_bounds__(256) void k_score_f32_split(
    const float *__restrict__ X, int32_t N, const float *__restrict__ W,
    const float *__restrict__ bias, int32_t K, int32_t D, float *__restrict__ S, int32_t splits,
    float *__restrict__ part, const int32_t *__restrict__ n_dev) {
    // Tile: 128 feature rows x kTK identities (kTK = 256, 128 or 64); wave w owns
    // rows 64 (w & 1) .. +64 and identities (kTK / 2) (w >> 1) .. + kTK / 2 as
    // 2 x kJB blocks of 32 x 32.
    constexpr int kSlice = 128, kTM = 128;
    constexpr int kJB = kTK / 64;                          // 32-wide blocks per wave
    constexpr int kWRows = kTK / 4;                        // W rows each wave copies
    constexpr int kCopies = 4 + kWRows / 8;                // 1 KB copies per wave and stage
    constexpr int kStage = (kTM + kTK) * kSlice;
    __shared__ __attribute__((aligned(1024))) uint8_t lds[kRingN * kStage];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int32_t n0 = blockIdx.x * kTM, k0 = blockIdx.y * kTK, sp = blockIdx.z;
    if (n_dev) N = *n_dev;  // the grid covers the most rows; tiles past N leave
    if (n0 >= N) return;    // uniform
    const int32_t dsp = D / splits, d0 = sp * dsp;
    const int nst = dsp / (kSlice / 4);
    auto swz = [](int row, int chunk) { return chunk ^ (row & 7); };

    // Copy role: X rows 32 w .. +31 (4 copies of 8 rows) and W rows
    // kWRows w .. + kWRows; lane i -> row i / 8 of its kilobyte, position i % 8.
    const int rr = lane >> 3, pos = lane & 7;
    const float *src[kCopies];
    int dst[kCopies];
#pragma unroll
    for (int j = 0; j < kCopies; ++j) {
        const bool isx = j < 4;
        const int row = isx ? wave * 32 + j * 8 + rr : wave * kWRows + (j - 4) * 8 + rr;
        const int32_t g = isx ? min(n0 + row, N - 1) : min(k0 + row, K - 1);
        src[j] = (isx ? X : W) + (size_t)g * D + d0 + 4 * swz(row, pos);
        dst[j] = isx ? (wave * 32 + j * 8) * kSlice : kTM * kSlice + (wave * kWRows + (j - 4) * 8) * kSlice;
    }
    // Copy j of stage st into ring slot st % kRingN. Stages past the last one
    // re-read the last stage's slice into a slot nobody reads again, so every
    // step issues the same copies: the loop body has no branch and the copies
    // can be spread between its matrix instructions.
    auto copy1 = [&](int st, int j) {
        uint8_t *stage = lds + (st % kRingN) * kStage;
        const int sg = min(st, nst - 1);
        __builtin_amdgcn_global_load_lds((glb_void_t *)(src[j] + sg * (kSlice / 4)),
                                         (lds_void_t *)(stage + dst[j]), 16, 0, 0);
    };

    const int fr = lane & 31, fq = lane >> 5;
    int oa[2][4], ob[kJB][4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ra = wm * 64 + 32 * i + fr;
            oa[i][p] = ra * kSlice + 16 * swz(ra, 2 * p + fq);
        }
#pragma unroll
        for (int j = 0; j < kJB; ++j) {
            const int rb = wn * (kTK / 2) + 32 * j + fr;
            ob[j][p] = kTM * kSlice + rb * kSlice + 16 * swz(rb, 2 * p + fq);
        }
    }
    struct Frag {
        floatx4 a[2][4], b[kJB][4];
    };
    // Fragments of feature chunk p (4 floats of each lane's row) of stage st.
    auto read_p = [&](int st, Frag &f, int p) {
        const uint8_t *stage = lds + (st % kRingN) * kStage;
#pragma unroll
        for (int i = 0; i < 2; ++i)
            f.a[i][p] = *reinterpret_cast<const floatx4 *>(stage + oa[i][p]);
#pragma unroll
        for (int j = 0; j < kJB; ++j)
            f.b[j][p] = *reinterpret_cast<const floatx4 *>(stage + ob[j][p]);
    };
    floatx16 acc[2][kJB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < kJB; ++j) acc[i][j] = floatx16{};
    auto mma_p = [&](const Frag &f, int p) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < kJB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[i][p][c], f.b[j][p][c],
                                                                      acc[i][j], 0, 0, 0);
    };
    auto mma = [&](const Frag &f) {
#pragma unroll
        for (int p = 0; p < 4; ++p) mma_p(f, p);
    };
    // Stage st's buffer is free once its fragments are in registers (read
    // during the previous step, before this step's barrier), so the copy of
    // stage st + kRingN goes there: kRingN - 1 stages stay in flight. With a
    // single wave per SIMD the matrix core idles whenever this wave stalls on
    // issuing memory instructions, so each step runs as four groups, one per
    // feature chunk p: a share of the copies, the next stage's chunk-p
    // fragments, and the current stage's chunk-p MFMAs. The scheduling
    // barriers keep the groups apart.
    auto step = [&](int st, const Frag &cur, Frag &nxt) {
        wait_vm<(kRingN - 2) * kCopies>();
        barrier_lds();
#pragma unroll
        for (int p = 0; p < 4; ++p) {
#pragma unroll
            for (int j = 0; j < kCopies; ++j)
                if (j % 4 == p) copy1(st + kRingN, j);
            read_p(st + 1, nxt, p);
            mma_p(cur, p);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
#pragma unroll
    for (int st = 0; st < kRingN; ++st)
#pragma unroll
        for (int j = 0; j < kCopies; ++j) copy1(st, j);
    Frag f0, f1;
    wait_vm<(kRingN - 1) * kCopies>();
    barrier_lds();
#pragma unroll
    for (int p = 0; p < 4; ++p) read_p(0, f0, p);
    int st = 0;
    for (; st + 2 < nst; st += 2) {
        step(st, f0, f1);
        step(st + 1, f1, f0);
    }
    if (st + 1 < nst) {
        step(st, f0, f1);
        mma(f1);
    } else {
        mma(f0);
    }
    // The copies past the last stage must land before the workgroup's LDS
    // is released.
    wait_vm<0>();

    // 32 x 32 block layout: register r of lane l is row 8 (r / 4) + 4 (l / 32)
    // + r % 4, column l % 32.
    auto for_each = [&](auto &&f) {
#pragma unroll
        for (int j = 0; j < kJB; ++j) {
            const int32_t k = k0 + wn * (kTK / 2) + 32 * j + (lane & 31);
            if (k >= K) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t n = n0 + wm * 64 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    if (n < N) f(i, j, r, n, k);
                }
        }
    };
    if (splits == 1) {
        for_each([&](int i, int j, int r, int32_t n, int32_t k) {
            S[(size_t)n * K + k] = acc[i][j][r] + bias[k];
        });
        return;
    }
    const size_t plane = (size_t)N * K;
    for_each([&](int i, int j, int r, int32_t n, int32_t k) {
        part[(size_t)sp * plane + (size_t)n * K + k] = acc[i][j][r];
    });
}

// Split-D epilogue, one wave per row: S = (((part_0 + part_1) + ...) + b in
// split order, and (optionally) the row's argmax, ties to the lowest index as
// in k_argmax.
// kVec: K a multiple of 4 and 16-byte aligned rows, so each lane takes four
// consecutive identities per step as float4.
template <bool kVec>
__global__ __launch_bounds__(256) void k_reduce_argmax(const float *__restrict__ part,
                                                       int32_t splits, int32_t N, int32_t K,
                                                       const float *__restrict__ bias,
                                                       float *__restrict__ S,
                                                       int32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int32_t n = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (n >= N) return;
    const size_t plane = (size_t)N * K, row = (size_t)n * K;
    float best = -INFINITY;
    int32_t arg = K;
    if constexpr (kVec) {
        for (int32_t k = 4 * lane; k < K; k += 256) {
            floatx4 v = *reinterpret_cast<const floatx4 *>(part + row + k);
            for (int q = 1; q < splits; ++q)
                v += *reinterpret_cast<const floatx4 *>(part + (size_t)q * plane + row + k);
            v += *reinterpret_cast<const floatx4 *>(bias + k);
            *reinterpret_cast<floatx4 *>(S + row + k) = v;
#pragma unroll
            for (int c = 0; c < 4; ++c)  // k + c ascending: a strict > keeps the first
                if (v[c] > best || arg == K) {
                    best = v[c];
                    arg = k + c;
                }
        }
    } else {
        for (int32_t k = lane; k < K; k += 64) {
            float v = part[row + k];
            for (int q = 1; q < splits; ++q) v += part[(size_t)q * plane + row + k];
            v += bias[k];
            S[row + k] = v;
            if (v > best || arg == K) {
                best = v;
                arg = k;
            }
        }
    }
    if (!out) return;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ob = __shfl_xor(best, off, 64);
        const int32_t oa = __shfl_xor(arg, off, 64);
        if (ob > best || (ob == best && oa < arg)) {
            best = ob;
            arg = oa;
        }
    }
    if (lane == 0) out[n] = arg;
}

}  // namespace

// Identities per tile of the split kernel. On the 4096 x 256 x 7552 product
// 128 (64 tiles, D split in 4) ran in 164 us and 64 (128 tiles, D split in 2)
// in 171-176 us.
constexpr int kSplitTK = 128;

int32_t score_f32_splits(int32_t N, int32_t K, int32_t D, int32_t num_cus, size_t part_elems) {
    const int64_t tiles = (int64_t)((N + 127) / 128) * ((K + kSplitTK - 1) / kSplitTK);
    int32_t best = 1;
    for (int32_t sp = 2; sp <= 4; sp *= 2) {
        if (tiles * best >= num_cus) break;  // enough workgroups already
        if (D % (32 * sp) != 0) break;
        if ((size_t)sp * (size_t)N * (size_t)K > part_elems) break;
        best = sp;
    }
    return best;
}

hipError_t launch_score_f32(const float *X, int32_t N, const float *W, const float *b, int32_t K,
                            int32_t D, float *S, int32_t *argmax, hipStream_t s, int32_t splits,
                            float *part, const int32_t *n_dev) {
    if (N <= 0 || K <= 0) return hipSuccess;
    const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)W % 16 == 0);
    // Unsplit products whose tiles fill the CUs in fewer rounds as 128 x 256:
    // 256 identities per tile (48 KB stages, two-stage ring, one workgroup of
    // 434 registers a lane per CU), 4/3 the matrix work per copied byte of the
    // 128 x 128 tile. A round of 128 x 256 tiles takes about 1.91 rounds of
    // 128 x 128 ones (16384 x 1024 x 7552: 1858 us in 2 rounds against
    // 1941-1947 in 4), so the wide tile is taken when 1.91 r256 < r128 (on
    // 5120 x 5120 x 7552, 4 wide rounds against 7: 3.8 ms against 3.45).
    int cus = 256;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        cus = std::max(cus, 1);
    }
    const size_t nt = (size_t)((N + 127) / 128);
    const size_t r128 = (nt * (size_t)((K + 127) / 128) + cus - 1) / cus;
    const size_t r256 = (nt * (size_t)((K + 255) / 256) + cus - 1) / cus;
    if (aligned && splits == 1 && D % 32 == 0 && K >= 256 && 191 * r256 < 100 * r128) {
        const dim3 g((N + 127) / 128, (K + 255) / 256, 1);
        hipLaunchKernelGGL((k_score_f32_split<2, 256>), g, dim3(256), 0, s, X, N, W, b, K, D, S,
                           1, part, n_dev);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || !argmax) return e;
        return launch_argmax(S, N, K, argmax, s, n_dev);
    }
    if (aligned && splits >= 1 && D % (32 * splits) == 0 && (splits == 1 || part)) {
        dim3 g((N + 127) / 128, (K + kSplitTK - 1) / kSplitTK, splits);
        // 128 x 128 tiles. At least two tiles per CU (512 on the 256-CU
        // MI355X): a two-stage ring (64 KB of LDS; the workgroup's 270
        // registers a lane still leave one workgroup per CU, and a shallower
        // ring measured faster than four stages: 1940-1946 us against
        // 1960-1964 on 16384 x 1024 x 7552). Otherwise (fewer tiles, or D
        // split over workgroups) a four-stage ring.
        if (splits == 1 && (size_t)g.x * g.y >= 512)
            hipLaunchKernelGGL((k_score_f32_split<2, kSplitTK>), g, dim3(256), 0, s, X, N, W, b, K,
                               D, S, splits, part, n_dev);
        else
            hipLaunchKernelGGL((k_score_f32_split<4, kSplitTK>), g, dim3(256), 0, s, X, N, W, b, K,
                               D, S, splits, part, n_dev);
        if (splits > 1) {
            const bool v4 = K % 4 == 0 && ((uintptr_t)S % 16 == 0) && ((uintptr_t)b % 16 == 0);
            if (v4)
                hipLaunchKernelGGL(k_reduce_argmax<true>, dim3((N + 3) / 4), dim3(256), 0, s, part,
                                   splits, N, K, b, S, argmax);
            else
                hipLaunchKernelGGL(k_reduce_argmax<false>, dim3((N + 3) / 4), dim3(256), 0, s,
                                   part, splits, N, K, b, S, argmax);
            return hipGetLastError();
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !argmax) return e;
        return launch_argmax(S, N, K, argmax, s, n_dev);
    }
    if (n_dev) return hipErrorInvalidValue;  // device row counts: the tiled kernel only
    dim3 grid((N + kTile - 1) / kTile, (K + kTile - 1) / kTile);
    const bool vec = (D % 4 == 0) && ((uintptr_t)X % 16 == 0) && ((uintptr_t)W % 16 == 0);
    if (vec)
        hipLaunchKernelGGL(k_score_f32<true>, grid, dim3(512), 0, s, X, N, W, b, K, D, S);
    else
        hipLaunchKernelGGL(k_score_f32<false>, grid, dim3(512), 0, s, X, N, W, b, K, D, S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !argmax) return e;
    return launch_argmax(S, N, K, argmax, s);
}

hipError_t launch_argmax(const float *S, int32_t N, int32_t K, int32_t *argmax, hipStream_t s,
                         const int32_t *n_dev) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_argmax, dim3((N + 3) / 4), dim3(256), 0, s, S, N, K, argmax, n_dev);
    return hipGetLastError();
}

}  // namespace lbpf
