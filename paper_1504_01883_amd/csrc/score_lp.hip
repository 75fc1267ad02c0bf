// Reduced-precision SVM scoring, S = (s_x[n] s_w[k]) (Xq Wq^T)[n][k] + b[k],
// on gfx950 matrix cores with FP32 accumulation (Sec. 2.5 decision values).
//
// Operand formats (rows quantised by k_quant_rows):
//   BF16: round-to-nearest-even, no scale (s = 1);
//   FP16: per-row power-of-two scale s = 2^(e - 14), e = exponent of the row's
//         largest magnitude, so the row's largest value lands in [2^14, 2^15)
//         and the scaling itself is exact;
//   FP8 : OCP e4m3 (bias 7, max 448, no infinities), per-row scale
//         s = amax / 448 and encoding factor r = 448 / amax (each one FP32
//         division per row); x r (FP32 product) rounded to nearest even on
//         the e4m3 grid and saturated. One multiply per element instead of a
//         division; s r differs from 1 by at most 2^-23, far below e4m3's
//         2^-4 step.
// Quantised rows are stored with a row pitch rounded up to 128 bytes, zero
// padded, so every k-stage of the GEMM is a whole 128-byte chunk. Rows of up
// to 8192 values are quantised by k_quant_rows_vec in one read (the row held
// in registers, vector stores), longer ones by k_quant_rows.
//
// Large products (N >= 512, K >= 256) run k_score_lp_big (256 x 256 tiles
// through an LDS ring, described there), whose epilogue also reduces each
// row's best identity over the tile; k_argmax_tiles merges the tiles, so an
// argmax-only call never writes S.
//
// Small products, GEMM: a workgroup of 4 wave64 owns a 256 (n) x 128 (k) tile of S; wave w
// owns rows 128 (w & 1) .. +128 and columns 64 (w >> 1) .. +64 as 4 x 2
// blocks of 32 x 32 (v_mfma_f32_32x32x16_{bf16,f16} or
// v_mfma_f32_32x32x64_f8f6f4). Per k-stage of 128 bytes per row the
// workgroup stages its A (256 x 128 B) and B (128 x 128 B) tiles in LDS (rows
// padded to 144 B so the 16-byte fragment reads of 8 consecutive rows cover
// all 32 banks), and the next stage's tiles are loaded into registers while
// the current one is multiplied.
#include "lbpf_internal.h"

#include <algorithm>

namespace lbpf {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Split FP32 operands (LBPF_F16X3): a row scaled by 2^-sh is stored as an
// FP16 high part h and an FP16 low part l = fp16(x - h), in segments of
// lp_seg(D) bytes: feature rows as [h | l], weight rows as [h | l | h]. The
// GEMM walks three segments of the reduction, reading the feature row's h
// twice (the A operand's segment remap), so one FP16 product sums
// h_x h_w + h_x l_w + l_x h_w.
constexpr int kF16X3W = 5;  // quantiser mode of split weight rows

constexpr int kTM = 256, kTN = 128;  // workgroup tile
constexpr int kRowB = 128;           // bytes of k per stage and row
constexpr int kPitch = 144;          // LDS row pitch (bytes)
constexpr uint32_t kGroupN = 4;      // row tiles per group of the tile order

// --- conversions ------------------------------------------------------------

__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

__device__ __forceinline__ uint16_t to_f16_rne(float f) {
    return __builtin_bit_cast(uint16_t, (_Float16)f);  // IEEE conversion, round to nearest even
}

// OCP e4m3: 1 sign, 4 exponent (bias 7), 3 mantissa bits; finite values
// 2^-9 .. 448; saturating, round to nearest even.
__device__ __forceinline__ uint8_t to_e4m3_rne_sat(float f) {
    const uint32_t sign = (__float_as_uint(f) >> 24) & 0x80u;
    float a = fabsf(f);
    if (!(a < 448.0f)) return (uint8_t)(sign | 0x7Eu);  // saturate (NaN too) to 448
    if (a == 0.0f) return (uint8_t)sign;
    int e;
    frexpf(a, &e);                 // a = m 2^e, m in [0.5, 1)
    int ex = e - 1;                // a in [2^ex, 2^(ex+1))
    if (ex < -6) ex = -6;          // subnormal range: quantum 2^-9
    const float q = ldexpf(1.0f, ex - 3);  // spacing of representable values
    float n = rintf(a / q);        // exact division by a power of two; rint = nearest even
    // n in [8, 16] for normals (16 rounds up into the next binade), [0, 8) subnormal
    uint32_t bits;
    if (n >= 16.0f) {
        ex += 1;
        n = 8.0f;
    }
    if (ex == -6 && n < 8.0f) {
        bits = (uint32_t)n;  // subnormal: exponent field 0
    } else {
        bits = ((uint32_t)(ex + 7) << 3) | ((uint32_t)n - 8u);
    }
    if (bits > 0x7Eu) bits = 0x7Eu;
    return (uint8_t)(sign | bits);
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// One workgroup per row: amax, scale, convert; pads the row to `pitch` bytes.
template <int kMode>
__global__ __launch_bounds__(256) void k_quant_rows(const float *__restrict__ X, int32_t rows,
                                                    int32_t D, int32_t pitch,
                                                    uint8_t *__restrict__ out,
                                                    float *__restrict__ scales,
                                                    const int32_t *__restrict__ n_dev) {
    __shared__ float part[4];
    const int r = blockIdx.x;
    if (n_dev && r >= *n_dev) return;  // uniform: fewer rows than the grid
    const float *x = X + (size_t)r * D;
    float amax = 0.0f;
    for (int i = threadIdx.x; i < D; i += 256) amax = fmaxf(amax, fabsf(x[i]));
    amax = wave_max(amax);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = amax;
    __syncthreads();
    amax = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
    uint8_t *o = out + (size_t)r * pitch;
    if (kMode == LBPF_BF16) {
        if (threadIdx.x == 0) scales[r] = 1.0f;
        uint16_t *o16 = reinterpret_cast<uint16_t *>(o);
        for (int i = threadIdx.x; i < pitch / 2; i += 256) o16[i] = i < D ? to_bf16_rne(x[i]) : 0;
    } else if (kMode == LBPF_FP16) {
        int e = 0;
        if (amax > 0.0f) frexpf(amax, &e);  // amax in [2^(e-1), 2^e)
        const int sh = (amax > 0.0f) ? (e - 1) - 14 : 0;
        if (threadIdx.x == 0) scales[r] = ldexpf(1.0f, sh);
        uint16_t *o16 = reinterpret_cast<uint16_t *>(o);
        for (int i = threadIdx.x; i < pitch / 2; i += 256)
            o16[i] = i < D ? to_f16_rne(ldexpf(x[i], -sh)) : 0;
    } else if (kMode == LBPF_F16X3 || kMode == kF16X3W) {
        int e = 0;
        if (amax > 0.0f) frexpf(amax, &e);
        const int sh = (amax > 0.0f) ? (e - 1) - 14 : 0;
        if (threadIdx.x == 0) scales[r] = ldexpf(1.0f, sh);
        uint16_t *o16 = reinterpret_cast<uint16_t *>(o);
        const int seg = pitch / (kMode == kF16X3W ? 6 : 4);  // elements per segment
        for (int i = threadIdx.x; i < seg; i += 256) {
            const float y = i < D ? ldexpf(x[i], -sh) : 0.0f;
            const _Float16 hv = (_Float16)y;
            const uint16_t hb = __builtin_bit_cast(uint16_t, hv);
            const uint16_t lb = to_f16_rne(y - (float)hv);
            o16[i] = hb;
            o16[seg + i] = lb;
            if (kMode == kF16X3W) o16[2 * seg + i] = hb;
        }
    } else {
        const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        const float f = amax > 0.0f ? 448.0f / amax : 1.0f;
        if (threadIdx.x == 0) scales[r] = s;
        for (int i = threadIdx.x; i < pitch; i += 256) o[i] = i < D ? to_e4m3_rne_sat(x[i] * f) : 0;
    }
}

// One wave per row, four rows per workgroup, for rows of D <= 256 kC values
// with D % 4 == 0 and 16-byte aligned rows: the row is read once into
// registers (float4 per lane and chunk), its amax reduced over the wave, and
// the converted values stored as one 8-byte (BF16, FP16) or 4-byte (FP8)
// vector per float4; the pad up to `pitch` is zeroed. Same values and scales
// as k_quant_rows.
template <int kMode, int kC>
__global__ __launch_bounds__(256) void k_quant_rows_vec(const float *__restrict__ X, int32_t rows,
                                                        int32_t D, int32_t pitch,
                                                        uint8_t *__restrict__ out,
                                                        float *__restrict__ scales,
                                                        const int32_t *__restrict__ n_dev) {
    const int lane = threadIdx.x & 63;
    const int32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= (n_dev ? *n_dev : rows)) return;
    const int nq = D >> 2;
    const f32x4 *x = reinterpret_cast<const f32x4 *>(X + (size_t)r * D);
    f32x4 v[kC];
    float amax = 0.0f;
#pragma unroll
    for (int c = 0; c < kC; ++c) {
        const int q = c * 64 + lane;
        v[c] = q < nq ? __builtin_nontemporal_load(x + q) : f32x4{0.f, 0.f, 0.f, 0.f};
        amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v[c].x), fabsf(v[c].y)),
                                 fmaxf(fabsf(v[c].z), fabsf(v[c].w))));
    }
    amax = wave_max(amax);
    uint8_t *o = out + (size_t)r * pitch;
    constexpr int kEB = kMode == LBPF_FP8_E4M3 ? 1 : 2;
    if constexpr (kMode == LBPF_F16X3 || kMode == kF16X3W) {
        int e = 0;
        if (amax > 0.0f) frexpf(amax, &e);
        const int sh = (amax > 0.0f) ? (e - 1) - 14 : 0;
        if (lane == 0) scales[r] = ldexpf(1.0f, sh);
        const int seg = pitch / (kMode == kF16X3W ? 3 : 2);  // bytes per segment
        // The high part is the scaled value rounded to FP16, the low part
        // the rounded remainder (exact in FP32: h is within an FP16 ulp).
        auto split = [&](float f, uint32_t &hb, uint32_t &lb) {
            const float y = ldexpf(f, -sh);
            const _Float16 hv = (_Float16)y;
            hb = __builtin_bit_cast(uint16_t, hv);
            lb = to_f16_rne(y - (float)hv);
        };
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            const int q = c * 64 + lane;
            if (q < nq) {
                uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
                split(v[c].x, h0, l0);
                split(v[c].y, h1, l1);
                split(v[c].z, h2, l2);
                split(v[c].w, h3, l3);
                const uint2 hw = uint2{h0 | (h1 << 16), h2 | (h3 << 16)};
                *reinterpret_cast<uint2 *>(o + 8 * q) = hw;
                *reinterpret_cast<uint2 *>(o + seg + 8 * q) = uint2{l0 | (l1 << 16), l2 | (l3 << 16)};
                if constexpr (kMode == kF16X3W) *reinterpret_cast<uint2 *>(o + 2 * seg + 8 * q) = hw;
            }
        }
        // Zero pad every segment past D (segments are multiples of 128 bytes).
        for (int q = nq + lane; q < seg / 8; q += 64) {
            *reinterpret_cast<uint2 *>(o + 8 * q) = uint2{0u, 0u};
            *reinterpret_cast<uint2 *>(o + seg + 8 * q) = uint2{0u, 0u};
            if constexpr (kMode == kF16X3W) *reinterpret_cast<uint2 *>(o + 2 * seg + 8 * q) = uint2{0u, 0u};
        }
        return;
    }
    if constexpr (kMode == LBPF_FP8_E4M3) {
        const float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        const float f = amax > 0.0f ? 448.0f / amax : 1.0f;
        if (lane == 0) scales[r] = s;
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            const int q = c * 64 + lane;
            if (q < nq) {
                // The packed hardware conversion (OCP e4m3, round to nearest
                // even). Over every float below 464 in magnitude it gives the
                // same bytes as a saturating round-to-nearest-even encoder
                // (checked exhaustively on gfx950 against an integer one);
                // the scaled values here stay below 448 + 2^-13.
                const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[c].x * f, v[c].y * f, 0, false);
                const uint32_t w =
                    (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(v[c].z * f, v[c].w * f, lo, true);
                *reinterpret_cast<uint32_t *>(o + 4 * q) = w;
            }
        }
    } else {
        int sh = 0;
        if constexpr (kMode == LBPF_FP16) {
            int e = 0;
            if (amax > 0.0f) frexpf(amax, &e);  // amax in [2^(e-1), 2^e)
            sh = (amax > 0.0f) ? (e - 1) - 14 : 0;
            if (lane == 0) scales[r] = ldexpf(1.0f, sh);
        } else {
            if (lane == 0) scales[r] = 1.0f;
        }
        auto cvt = [&](float f) -> uint32_t {
            if constexpr (kMode == LBPF_FP16) return to_f16_rne(ldexpf(f, -sh));
            // The compiler's conversion (v_cvt_pk_bf16_f32, round to nearest
            // even): the same bits as to_bf16_rne on every finite float
            // (checked exhaustively on gfx950).
            else return __builtin_bit_cast(uint16_t, (__bf16)f);
        };
#pragma unroll
        for (int c = 0; c < kC; ++c) {
            const int q = c * 64 + lane;
            if (q < nq) {
                const uint32_t lo = cvt(v[c].x) | (cvt(v[c].y) << 16);
                const uint32_t hi = cvt(v[c].z) | (cvt(v[c].w) << 16);
                *reinterpret_cast<uint2 *>(o + 8 * q) = uint2{lo, hi};
            }
        }
    }
    // Zero pad: elements D .. pitch / kEB - 1, four at a time (pitch is a
    // multiple of 128 bytes and D of 4).
    for (int q = nq + lane; q < pitch / (4 * kEB); q += 64) {
        if constexpr (kEB == 1) *reinterpret_cast<uint32_t *>(o + 4 * q) = 0u;
        else *reinterpret_cast<uint2 *>(o + 8 * q) = uint2{0u, 0u};
    }
}

// --- GEMM ----------------------------------------------------------------------

template <int kMode>
__device__ __forceinline__ f32x16 mfma_step(const u32x4 a[2], const u32x4 b[2], f32x16 acc, int sub) {
    if constexpr (kMode == LBPF_FP8_E4M3) {
        // one 32x32x64 step consumes 32 bytes (two 16-byte fragments) per lane
        const i32x8 av = {(int)a[0].x, (int)a[0].y, (int)a[0].z, (int)a[0].w,
                          (int)a[1].x, (int)a[1].y, (int)a[1].z, (int)a[1].w};
        const i32x8 bv = {(int)b[0].x, (int)b[0].y, (int)b[0].z, (int)b[0].w,
                          (int)b[1].x, (int)b[1].y, (int)b[1].z, (int)b[1].w};
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc, 0, 0, 0, 0, 0, 0);
    } else if constexpr (kMode == LBPF_FP16) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a[sub]),
                                                     __builtin_bit_cast(f16x8, b[sub]), acc, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[sub]),
                                                      __builtin_bit_cast(bf16x8, b[sub]), acc, 0, 0, 0);
    }
}

// Xq: [N][pitch] bytes, Wq: [K][pitch] bytes, pitch a multiple of 128.
// S: [N][K] FP32 (ld = ldS). Rows past N / K read as zero and are not stored.
template <int kMode>
__global__ __launch_bounds__(256) void k_score_lp(const uint8_t *__restrict__ Xq,
                                                  const float *__restrict__ sx, int32_t N,
                                                  const uint8_t *__restrict__ Wq,
                                                  const float *__restrict__ sw,
                                                  const float *__restrict__ bias, int32_t K,
                                                  int32_t pitch, float *__restrict__ S,
                                                  const int32_t *__restrict__ n_dev,
                                                  int32_t a_pitch, int32_t a_seg) {
    __shared__ __attribute__((aligned(16))) uint8_t sA[kTM * kPitch];
    if (n_dev) N = *n_dev;  // the grid covers the most rows; tiles past N leave
    __shared__ __attribute__((aligned(16))) uint8_t sB[kTN * kPitch];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // Tile order. Consecutive workgroups are dealt round-robin to the 8 XCDs;
    // the remap gives each XCD a contiguous range of logical tiles, walked in
    // groups of kGroupN row tiles x all identity tiles, so the ~32 tiles an XCD
    // runs at once share 4 feature-row tiles and 8 weight tiles in its L2.
    const uint32_t nwg = gridDim.x, pid = blockIdx.x;
    const uint32_t xcd = pid & 7u, per = nwg >> 3, rem = nwg & 7u;
    const uint32_t L = xcd * per + min(xcd, rem) + (pid >> 3);
    const uint32_t KT = (uint32_t)(K + kTN - 1) / kTN, NT = (uint32_t)(N + kTM - 1) / kTM;
    if (L >= NT * KT) return;  // uniform
    const uint32_t g = L / (kGroupN * KT), i_g = L - g * (kGroupN * KT);
    const uint32_t gn = min((uint32_t)kGroupN, NT - g * kGroupN);
    const int32_t n0 = (int32_t)(g * kGroupN + i_g % gn) * kTM;
    const int32_t k0 = (int32_t)(i_g / gn) * kTN;

    // Global -> register staging: thread t moves 16-byte chunk (t % 8) of rows
    // t / 8 + 32 j.
    const int ch = tid & 7, r0 = tid >> 3;
    u32x4 ra[8], rb[4];
    auto load_stage = [&](int32_t kb) {
        // The feature row's byte for reduction byte kb (split operands read
        // their first segment twice).
        const int32_t kba = (a_seg && kb >= a_seg) ? kb - a_seg : kb;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int32_t n = n0 + r0 + 32 * j;
            ra[j] = n < N ? *reinterpret_cast<const u32x4 *>(Xq + (size_t)n * a_pitch + kba + 16 * ch)
                          : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t k = k0 + r0 + 32 * j;
            rb[j] = k < K ? *reinterpret_cast<const u32x4 *>(Wq + (size_t)k * pitch + kb + 16 * ch)
                          : u32x4{0u, 0u, 0u, 0u};
        }
    };
    auto store_stage = [&]() {
#pragma unroll
        for (int j = 0; j < 8; ++j)
            *reinterpret_cast<u32x4 *>(sA + (r0 + 32 * j) * kPitch + 16 * ch) = ra[j];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            *reinterpret_cast<u32x4 *>(sB + (r0 + 32 * j) * kPitch + 16 * ch) = rb[j];
    };

    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};

    const int fr = lane & 31, fq = lane >> 5;  // fragment row, 16-byte half of 32 bytes
    load_stage(0);
    for (int32_t kb = 0; kb < pitch; kb += kRowB) {
        __syncthreads();  // the previous stage's fragments have been read
        store_stage();
        __syncthreads();
        if (kb + kRowB < pitch) load_stage(kb + kRowB);
        // 4 sub-steps of 32 bytes per row: lane (fr, fq) supplies bytes
        // 16 fq .. 16 fq + 15 of its row's 32-byte slice; an FP8 step takes
        // both halves of a 64-byte slice.
        constexpr int kSubB = (kMode == LBPF_FP8_E4M3) ? 64 : 32;
#pragma unroll
        for (int sb = 0; sb < kRowB; sb += kSubB) {
            u32x4 a[4][2], b[2][2];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint8_t *p = sA + (wm * 128 + 32 * i + fr) * kPitch + sb;
                if constexpr (kMode == LBPF_FP8_E4M3) {
                    a[i][0] = *reinterpret_cast<const u32x4 *>(p + 32 * fq);
                    a[i][1] = *reinterpret_cast<const u32x4 *>(p + 32 * fq + 16);
                } else {
                    a[i][0] = *reinterpret_cast<const u32x4 *>(p + 16 * fq);
                }
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const uint8_t *p = sB + (wn * 64 + 32 * j + fr) * kPitch + sb;
                if constexpr (kMode == LBPF_FP8_E4M3) {
                    b[j][0] = *reinterpret_cast<const u32x4 *>(p + 32 * fq);
                    b[j][1] = *reinterpret_cast<const u32x4 *>(p + 32 * fq + 16);
                } else {
                    b[j][0] = *reinterpret_cast<const u32x4 *>(p + 16 * fq);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = mfma_step<kMode>(a[i], b[j], acc[i][j], 0);
        }
    }

    // 32 x 32 block layout: lane l, register r holds row 8 (r / 4) + 4 (l / 32)
    // + r % 4 and column l % 32.
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int32_t k = k0 + wn * 64 + 32 * j + (lane & 31);
        if (k >= K) continue;
        const float swk = sw[k], bk = bias[k];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int32_t n = n0 + wm * 128 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (n < N) S[(size_t)n * K + k] = (sx[n] * swk) * acc[i][j][r] + bk;
            }
    }
}

// --- GEMM, large tiles ----------------------------------------------------------
//
// A workgroup of kW waves owns a 256 (n) x 256 (k) tile of S; wave (wm, wn)
// owns rows 128 wm .. +128 and columns (256 / (kW / 2)) wn .. as 4 x (8 / kW * 2)
// blocks of 32 x 32 (4 waves: 4 x 4 blocks; 8 waves: 4 x 2). The reduction dimension advances in stages of 64 bytes per row
// through a ring of kStages LDS buffers (32 KB each: A 256 rows, B 256 rows).
// Stages are copied with global_load_lds_dwordx4 (global -> LDS without
// registers): each wave instruction fills 1 KB = 16 rows of 64 bytes, lane i
// landing at byte 16 i, so lane i fetches the 16-byte chunk that belongs at
// row i / 4, position i % 4. Within a row the four chunks are stored at
// position chunk ^ ((row >> 1) & 3): the 16-byte fragment reads of 8
// consecutive rows then hit 8 different bank groups.
// The fragments of stage s + 1 are read into registers while stage s is
// multiplied, so MFMAs after a barrier never wait for LDS, and the copy of
// stage s + kStages, issued right after that barrier, reuses stage s's buffer.

constexpr int kBigT = 256;      // tile rows and columns
constexpr int kStageB = 64;     // bytes of the reduction per row and stage
constexpr int kStages = 5;  // 5 x 32 KB: all of the 160 KB LDS
// Waves per 256 x 256 workgroup (4 or 8). On 32768 x 8192 x 7552, quantisation
// included: 8 waves BF16 827 TFLOP/s, FP8 1278; 4 waves 784 and 1182.
constexpr int kBigWaves = 8;
constexpr int kStageBytes = 2 * kBigT * kStageB;  // A then B

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void glb_void_t;

template <int kVm>
__device__ __forceinline__ void wait_vm() {
    static_assert(kVm >= 0 && kVm < 64, "vmcnt range");
    // gfx9 s_waitcnt: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8], vmcnt[15:14].
    __builtin_amdgcn_s_waitcnt((kVm & 15) | (7 << 4) | (15 << 8) | ((kVm >> 4) << 14));
}

__device__ __forceinline__ int swz(int row, int chunk) { return chunk ^ ((row >> 1) & 3); }

// Workgroup barrier ordering LDS accesses only. __syncthreads would also
// drain every outstanding global access, including the LDS copies of the
// stages still in flight, which is exactly the overlap this kernel is after;
// each wave waits for its own copies of the current stage (wait_vm) first.
__device__ __forceinline__ void barrier_lds() {
    // lgkmcnt(0): this wave's LDS reads of the previous stage are done.
    __builtin_amdgcn_s_waitcnt((63 & 15) | (7 << 4) | (0 << 8) | ((63 >> 4) << 14));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Copy stage kb (byte offset into every row) into LDS buffer `buf`; with kW
// waves each copies 256 / kW rows of A and of B (1 KB = 16 rows per
// instruction). Rows past the matrix end re-read its last row (their results
// are dropped).
template <int kW>
__device__ __forceinline__ void copy_stage(const uint8_t *__restrict__ Xq, int32_t N, int32_t n0,
                                           const uint8_t *__restrict__ Wq, int32_t K, int32_t k0,
                                           int32_t pitch, int32_t kb, uint8_t *buf, int wave,
                                           int lane, int32_t a_pitch, int32_t a_seg) {
    constexpr int kPer = kBigT / kW / 16;  // instructions per wave and matrix
    const int r_in = lane >> 2, pos = lane & 3;
    // The feature row's byte for reduction byte kb (split operands read their
    // first segment twice; a 64-byte stage never straddles two segments).
    const int32_t kba = (a_seg && kb >= a_seg) ? kb - a_seg : kb;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = (wave * kPer + j) * 16 + r_in;  // 0..255
        const int c = swz(r, pos);
        const int32_t n = min(n0 + r, N - 1);
        const uint8_t *src = Xq + (size_t)n * a_pitch + kba + 16 * c;
        __builtin_amdgcn_global_load_lds((glb_void_t *)src,
                                         (lds_void_t *)(buf + (wave * kPer + j) * 1024), 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int r = (wave * kPer + j) * 16 + r_in;
        const int c = swz(r, pos);
        const int32_t k = min(k0 + r, K - 1);
        const uint8_t *src = Wq + (size_t)k * pitch + kb + 16 * c;
        __builtin_amdgcn_global_load_lds(
            (glb_void_t *)src, (lds_void_t *)(buf + kBigT * kStageB + (wave * kPer + j) * 1024),
            16, 0, 0);
    }
}

// kW waves (4: one per SIMD, each 128 x 128 of the tile; 8: two per SIMD,
// each 128 x 64, so one wave's waits are covered by the other's MFMAs).
// The blocks are multiplied with the weight tile as the MFMA's first operand,
// so each holds a 32 x 32 block of S transposed (identities x feature rows):
// every lane then holds 16 identities of one feature row, and the per-row
// argmax over the tile is mostly in-register work. S may be null (argmax
// only); apart, when not null, receives each row's (best score, identity)
// over the tile's 256 identities: values at apart[n KT + t], identities (as
// int32) at apart[N KT + n KT + t], t = k0 / 256, KT = ceil(K / 256).
template <int kMode, int kW>
__global__ __launch_bounds__(64 * kW) void k_score_lp_big(const uint8_t *__restrict__ Xq,
                                                          const float *__restrict__ sx, int32_t N,
                                                          const uint8_t *__restrict__ Wq,
                                                          const float *__restrict__ sw,
                                                          const float *__restrict__ bias,
                                                          int32_t K, int32_t pitch,
                                                          float *__restrict__ S,
                                                          float *__restrict__ apart,
                                                          const int32_t *__restrict__ n_dev,
                                                          int32_t a_pitch, int32_t a_seg) {
    if (n_dev) N = *n_dev;  // the grid covers the most rows; tiles past N leave
    constexpr int kCW = kBigT / (kW / 2);  // identities per wave
    constexpr int kJB = kCW / 32;          // 32-wide blocks per wave
    constexpr int kCopies = 2 * (kBigT / kW / 16);
    __shared__ __attribute__((aligned(1024))) uint8_t lds[kStages * kStageBytes];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // Tile order as in k_score_lp: XCD-contiguous ranges, groups of row tiles.
    const uint32_t nwg = gridDim.x, pid = blockIdx.x;
    const uint32_t xcd = pid & 7u, per = nwg >> 3, rem = nwg & 7u;
    const uint32_t L = xcd * per + min(xcd, rem) + (pid >> 3);
    const uint32_t KT = (uint32_t)(K + kBigT - 1) / kBigT, NT = (uint32_t)(N + kBigT - 1) / kBigT;
    if (L >= NT * KT) return;  // uniform
    const uint32_t g = L / (kGroupN * KT), i_g = L - g * (kGroupN * KT);
    const uint32_t gn = min((uint32_t)kGroupN, NT - g * kGroupN);
    const int32_t n0 = (int32_t)(g * kGroupN + i_g % gn) * kBigT;
    const int32_t k0 = (int32_t)(i_g / gn) * kBigT;

    f32x16 acc[4][kJB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < kJB; ++j) acc[i][j] = f32x16{};

    const int nst = pitch / kStageB;
    const int fr = lane & 31, fq = lane >> 5;
    // Fragments of one stage: [block][h]. BF16/FP16: h = the 32-byte sub-step
    // (this lane's 16 bytes of it); FP8: the two 16-byte halves of this lane's
    // 32 bytes of the single 64-byte step.
    struct Frag {
        u32x4 a[4][2], b[kJB][2];
    };
    auto read = [&](int st, Frag &f) {
        const uint8_t *bufA = lds + (st % kStages) * kStageBytes;
        const uint8_t *bufB = bufA + kBigT * kStageB;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = (kMode == LBPF_FP8_E4M3) ? 2 * fq + h : 2 * h + fq;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int ra = wm * 128 + 32 * i + fr;
                f.a[i][h] = *reinterpret_cast<const u32x4 *>(bufA + ra * kStageB + 16 * swz(ra, c));
            }
#pragma unroll
            for (int j = 0; j < kJB; ++j) {
                const int rb = wn * kCW + 32 * j + fr;
                f.b[j][h] = *reinterpret_cast<const u32x4 *>(bufB + rb * kStageB + 16 * swz(rb, c));
            }
        }
    };
    auto mma = [&](const Frag &f) {
        constexpr int kSubs = (kMode == LBPF_FP8_E4M3) ? 1 : 2;
#pragma unroll
        for (int sub = 0; sub < kSubs; ++sub)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < kJB; ++j)
                    acc[i][j] = mfma_step<kMode>(f.b[j], f.a[i], acc[i][j], sub);
    };
    // Iteration st: make stage st + 1 visible, start copying stage
    // st + kStages - 1 into the buffer of stage st - 1 (read an iteration
    // ago), read stage st + 1's fragments, multiply stage st's.
    // Called for st + 1 < nst only (the last stage is multiplied on its own,
    // so no path without a barrier joins the steady-state loop). Stage st's
    // buffer is free once its fragments are in registers (read during the
    // previous step, before this step's barrier), so the copy of stage
    // st + kStages goes there: kStages - 1 stages stay in flight.
    auto wait_younger = [](int younger) {
        if (younger >= 4) wait_vm<kCopies * 4>();
        else if (younger == 3) wait_vm<kCopies * 3>();
        else if (younger == 2) wait_vm<kCopies * 2>();
        else if (younger == 1) wait_vm<kCopies>();
        else wait_vm<0>();
    };
    auto step = [&](int st, const Frag &cur, Frag &nxt) {
        wait_younger(min(nst - 2 - st, kStages - 2));
        barrier_lds();
        if (st + kStages < nst)
            copy_stage<kW>(Xq, N, n0, Wq, K, k0, pitch, (st + kStages) * kStageB,
                           lds + (st % kStages) * kStageBytes, wave, lane, a_pitch, a_seg);
        read(st + 1, nxt);
        mma(cur);
    };
#pragma unroll
    for (int st = 0; st < kStages; ++st)
        if (st < nst)
            copy_stage<kW>(Xq, N, n0, Wq, K, k0, pitch, st * kStageB, lds + st * kStageBytes,
                           wave, lane, a_pitch, a_seg);
    if constexpr (kW == 8) {
        // Two waves per SIMD: fragments single-buffered (the registers go to
        // the accumulators), the other wave's MFMAs cover the LDS reads.
        // Stage st's buffer is refilled one step later, after the barrier
        // that follows its reads.
        Frag f;
        for (int st = 0; st < nst; ++st) {
            // Issued so far: stages 0 .. kStages - 1, then one per earlier
            // iteration j >= 1 (stage j - 1 + kStages): younger than st are
            // kStages - 1 stages at st = 0 and kStages - 2 after that.
            wait_younger(min(nst - 1 - st, st == 0 ? kStages - 1 : kStages - 2));
            barrier_lds();
            if (st >= 1 && st - 1 + kStages < nst)
                copy_stage<kW>(Xq, N, n0, Wq, K, k0, pitch, (st - 1 + kStages) * kStageB,
                               lds + ((st - 1) % kStages) * kStageBytes, wave, lane, a_pitch,
                               a_seg);
            read(st, f);
            mma(f);
        }
    } else {
    wait_younger(min(nst - 1, kStages - 1));
    barrier_lds();
    Frag f0, f1;
    read(0, f0);
    int st = 0;
    for (; st + 2 < nst; st += 2) {
        step(st, f0, f1);
        step(st + 1, f1, f0);
    }
    if (st + 1 < nst) {  // two stages left
        step(st, f0, f1);
        mma(f1);
    } else {
        mma(f0);
    }
    }

    // Transposed 32 x 32 block layout: lane l, register r of acc[i][j] holds
    // feature row 32 i + l % 32 of the wave's rows and identity
    // 32 j + 8 (r / 4) + 4 (l / 32) + r % 4 of its identities. Each lane scans
    // its identities in increasing order keeping the first maximum, then
    // meets lane l ^ 32 (the other identities of the same row).
    const int32_t kw = k0 + wn * kCW;
    const bool vec4 = (K & 3) == 0;
    // This lane's identities are the same for every row block: their scales
    // and biases are loaded once.
    float swv[kJB][16], bsv[kJB][16];
#pragma unroll
    for (int j = 0; j < kJB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int32_t k = kw + 32 * j + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            swv[j][r] = k < K ? sw[k] : 0.0f;
            bsv[j][r] = k < K ? bias[k] : 0.0f;
        }
    float best[4];
    int32_t barg[4];
    // Scores of a wave whose identities all lie inside K (K a multiple of 4)
    // leave through LDS: the MFMA layout gives every store instruction 32 B
    // of 32 different rows, so each 32-row block is first written to the
    // wave's own LDS area (rows padded to 68 floats against bank
    // conflicts), then stored 16 lanes to a row, 256 contiguous bytes each.
    // The ring is free once every wave has passed this barrier.
    constexpr int kSRow = kCW + 4;  // padded row of the staging area, floats
    const bool staged = S && vec4 && kw + kCW <= K;
    float *stg = reinterpret_cast<float *>(lds) + wave * 32 * kSRow;
    if (S) __syncthreads();  // uniform: S is a kernel argument
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int32_t n = n0 + wm * 128 + 32 * i + (lane & 31);
        const float sxn = n < N ? sx[n] : 0.0f;
        best[i] = -INFINITY;
        barg[i] = K;  // no identity yet
#pragma unroll
        for (int j = 0; j < kJB; ++j)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int32_t kg = kw + 32 * j + 8 * g + 4 * (lane >> 5);
                f32x4 v;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int32_t k = kg + t;
                    if (k < K) {
                        v[t] = (sxn * swv[j][4 * g + t]) * acc[i][j][4 * g + t] + bsv[j][4 * g + t];
                        if (v[t] > best[i] || barg[i] == K) {
                            best[i] = v[t];
                            barg[i] = k;
                        }
                    }
                }
                if (staged) {
                    *reinterpret_cast<f32x4 *>(stg + (lane & 31) * kSRow + (kg - kw)) = v;
                } else if (S && n < N) {
                    float *row = S + (size_t)n * K;
                    if (vec4 && kg + 3 < K) {
                        *reinterpret_cast<f32x4 *>(row + kg) = v;
                    } else {
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            if (kg + t < K) row[kg + t] = v[t];
                    }
                }
            }
        if (staged) {
            // Row rr of the block: lanes 16 q .. 16 q + 15 store its kCW
            // scores (kCW / 64 passes of 4 floats per lane).
            constexpr int kLanesPerRow = 16, kRowsPer = 64 / kLanesPerRow;
#pragma unroll
            for (int r0 = 0; r0 < 32; r0 += kRowsPer) {
                const int rr = r0 + lane / kLanesPerRow;
                const int32_t nr = n0 + wm * 128 + 32 * i + rr;
#pragma unroll
                for (int c0 = 0; c0 < kCW; c0 += 4 * kLanesPerRow) {
                    const int c = c0 + 4 * (lane % kLanesPerRow);
                    const f32x4 v = *reinterpret_cast<const f32x4 *>(stg + rr * kSRow + c);
                    if (nr < N) *reinterpret_cast<f32x4 *>(S + (size_t)nr * K + kw + c) = v;
                }
            }
        }
        const float ob = __shfl_xor(best[i], 32, 64);
        const int32_t oa = __shfl_xor(barg[i], 32, 64);
        if (ob > best[i] || (ob == best[i] && oa < barg[i])) {
            best[i] = ob;
            barg[i] = oa;
        }
    }
    if (!apart) return;
    // The kW / 2 waves of a row half cover the tile's identities in
    // increasing ranges: merge them through LDS (the ring is no longer read
    // once every wave has passed this barrier).
    __syncthreads();
    float *red_v = reinterpret_cast<float *>(lds);                 // [2][kW / 2][128]
    int32_t *red_i = reinterpret_cast<int32_t *>(lds + 4 * 128 * kW);
    if (lane < 32) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            red_v[(wm * (kW / 2) + wn) * 128 + 32 * i + lane] = best[i];
            red_i[(wm * (kW / 2) + wn) * 128 + 32 * i + lane] = barg[i];
        }
    }
    __syncthreads();
    const int32_t kt_n = (int32_t)KT, kt = k0 / kBigT;
    for (int rr = tid; rr < kBigT; rr += 64 * kW) {
        const int h = rr >> 7, q = rr & 127;
        float bv = -INFINITY;
        int32_t bi = K;
#pragma unroll
        for (int w = 0; w < kW / 2; ++w) {
            const float v = red_v[(h * (kW / 2) + w) * 128 + q];
            const int32_t a = red_i[(h * (kW / 2) + w) * 128 + q];
            if (v > bv || (v == bv && a < bi)) {
                bv = v;
                bi = a;
            }
        }
        const int32_t n = n0 + rr;
        if (n < N) {
            apart[(size_t)n * kt_n + kt] = bv;
            reinterpret_cast<int32_t *>(apart)[(size_t)N * kt_n + (size_t)n * kt_n + kt] = bi;
        }
    }
}

// Merge of the per-tile (best score, identity) pairs of k_score_lp_big, one
// thread per row: tiles in increasing identity order, a strict > keeps the
// lowest identity among equal scores.
__global__ __launch_bounds__(256) void k_argmax_tiles(const float *__restrict__ apart, int32_t N,
                                                      int32_t KT, int32_t *__restrict__ out,
                                                      const int32_t *__restrict__ n_dev) {
    if (n_dev) N = *n_dev;
    const int32_t n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const float *pv = apart + (size_t)n * KT;
    const int32_t *pi = reinterpret_cast<const int32_t *>(apart) + (size_t)N * KT + (size_t)n * KT;
    float bv = pv[0];
    int32_t bi = pi[0];
    for (int32_t t = 1; t < KT; ++t) {
        const float v = pv[t];
        if (v > bv) {
            bv = v;
            bi = pi[t];
        }
    }
    out[n] = bi;
}

}  // namespace

// float4 chunks per lane of the register-resident quantiser: rows up to
// 8192 values.
constexpr int kQuantChunks = 32;

int32_t lp_seg(int32_t D) { return (2 * D + kRowB - 1) / kRowB * kRowB; }

int32_t lp_pitch(int32_t D, int32_t mode) {
    if (mode == LBPF_F16X3) return 3 * lp_seg(D);  // weight rows [h | l | h]
    const int32_t bytes = D * (mode == LBPF_FP8_E4M3 ? 1 : 2);
    return (bytes + kRowB - 1) / kRowB * kRowB;
}

int32_t lp_pitch_features(int32_t D, int32_t mode) {
    return mode == LBPF_F16X3 ? 2 * lp_seg(D) : lp_pitch(D, mode);  // feature rows [h | l]
}

hipError_t launch_quant_rows(const float *X, int32_t rows, int32_t D, int32_t mode, uint8_t *out,
                             float *scales, hipStream_t s, const int32_t *n_dev, bool weights) {
    if (rows <= 0) return hipSuccess;
    // Split rows: weight rows hold three segments, feature rows two.
    const int32_t qmode = (mode == LBPF_F16X3 && weights) ? kF16X3W : mode;
    const int32_t pitch = weights ? lp_pitch(D, mode) : lp_pitch_features(D, mode);
    auto go = [&](auto vec_kernel, auto row_kernel) {
        if (D % 4 == 0 && D <= 256 * kQuantChunks && ((uintptr_t)X & 15) == 0)
            hipLaunchKernelGGL(vec_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, X, rows, D,
                               pitch, out, scales, n_dev);
        else
            hipLaunchKernelGGL(row_kernel, dim3(rows), dim3(256), 0, s, X, rows, D, pitch, out,
                               scales, n_dev);
    };
    switch (qmode) {
        case LBPF_BF16:
            go(k_quant_rows_vec<LBPF_BF16, kQuantChunks>, k_quant_rows<LBPF_BF16>);
            break;
        case LBPF_FP16:
            go(k_quant_rows_vec<LBPF_FP16, kQuantChunks>, k_quant_rows<LBPF_FP16>);
            break;
        case LBPF_FP8_E4M3:
            go(k_quant_rows_vec<LBPF_FP8_E4M3, kQuantChunks>, k_quant_rows<LBPF_FP8_E4M3>);
            break;
        case LBPF_F16X3:
            go(k_quant_rows_vec<LBPF_F16X3, kQuantChunks>, k_quant_rows<LBPF_F16X3>);
            break;
        default:
            go(k_quant_rows_vec<kF16X3W, kQuantChunks>, k_quant_rows<kF16X3W>);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_score_lp(const uint8_t *Xq, const float *sx, int32_t N, const uint8_t *Wq,
                           const float *sw, const float *b, int32_t K, int32_t D, int32_t mode,
                           float *S, int32_t *argmax, float *scratch, size_t scratch_elems,
                           hipStream_t s, const int32_t *n_dev) {
    if (N <= 0 || K <= 0) return hipSuccess;
    const int32_t pitch = lp_pitch(D, mode);  // reduction bytes per row (weights)
    const int32_t a_pitch = lp_pitch_features(D, mode);
    const int32_t a_seg = mode == LBPF_F16X3 ? lp_seg(D) : 0;
    if (N >= 2 * kBigT && K >= kBigT) {
        // Large products: 256 x 256 tiles fed through the LDS ring, the
        // argmax taken in the epilogue (per tile) when its pairs fit the
        // scratch, else by a pass over the scores.
        const int32_t KT = (K + kBigT - 1) / kBigT;
        const bool fuse = argmax && 2 * (size_t)N * KT <= scratch_elems;
        float *Sout = S ? S : (fuse ? nullptr : scratch);
        float *apart = fuse ? scratch : nullptr;
        dim3 grid((uint32_t)KT * ((N + kBigT - 1) / kBigT));
        constexpr int kW = kBigWaves;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(64 * kW), 0, s, Xq, sx, N, Wq, sw, b, K, pitch,
                               Sout, apart, n_dev, a_pitch, a_seg);
        };
        if (mode == LBPF_BF16) go(k_score_lp_big<LBPF_BF16, kW>);
        else if (mode == LBPF_FP8_E4M3) go(k_score_lp_big<LBPF_FP8_E4M3, kW>);
        else go(k_score_lp_big<LBPF_FP16, kW>);  // FP16 and split FP16
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || !argmax) return e;
        if (!fuse) return launch_argmax(Sout, N, K, argmax, s, n_dev);
        hipLaunchKernelGGL(k_argmax_tiles, dim3((N + 255) / 256), dim3(256), 0, s, apart, N, KT,
                           argmax, n_dev);
        return hipGetLastError();
    }
    // Small products. Without S the scores go through the scratch, in row
    // blocks that fit it (one block when the row count is on the device).
    int32_t blk = N;
    if (!S) {
        if (!n_dev) blk = (int32_t)std::min<size_t>((size_t)N, scratch_elems / (size_t)K);
        if (blk < 1 || (size_t)blk * K > scratch_elems) return hipErrorInvalidValue;
    }
    for (int32_t r0 = 0; r0 < N; r0 += blk) {
        const int32_t n = std::min(blk, N - r0);
        float *Sb = S ? S + (size_t)r0 * K : scratch;
        dim3 grid(((K + kTN - 1) / kTN) * ((n + kTM - 1) / kTM));
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, Xq + (size_t)r0 * a_pitch, sx + r0, n,
                               Wq, sw, b, K, pitch, Sb, n_dev, a_pitch, a_seg);
        };
        if (mode == LBPF_BF16) go(k_score_lp<LBPF_BF16>);
        else if (mode == LBPF_FP8_E4M3) go(k_score_lp<LBPF_FP8_E4M3>);
        else go(k_score_lp<LBPF_FP16>);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess && argmax) e = launch_argmax(Sb, n, K, argmax + r0, s, n_dev);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace lbpf
