// On-device SVM training (Sec. 2.5: one max-margin hyperplane per person, that
// person against all others; the paper trains on the CPU, Sec. 3).
//
// Problem per class k: L2-regularised hinge loss with C, the bias as an extra
// constant feature 1, features scaled by sigma = 1 / (lower median of the
// sample norms). Solver: dual coordinate descent (Hsieh et al., ICML 2008),
// in FP64, visiting the samples of every epoch in a seeded random order:
//   G  = y_i w.x_i - 1
//   PG = G, except min(G, 0) at alpha_i = 0 and max(G, 0) at alpha_i = C
//   alpha_i <- clamp(alpha_i - G / Q_ii, 0, C), Q_ii = x_i.x_i (+1 for the bias)
//   w <- w + (alpha_i' - alpha_i) y_i x_i
// until max |PG| over an epoch is below eps, or max_epochs. W = sigma w, b =
// the bias weight.
//
// Order of the samples: epoch e of class k is a Fisher-Yates shuffle of
// 0..N-1 (i from N-1 down to 1 swaps i with r mod (i+1)) drawing r from the
// splitmix64 stream (Steele, Lea and Flood, OOPSLA 2014: state += golden
// gamma, output = the variant-13 mix of the state) seeded with
// seed XOR (k+1) * 0x5851F42D4C957F2D; epoch e uses draws e(N-1) .. e(N-1)+N-2
// (splitmix64 is counter based: draw m is the mix of state0 + (m+1) gamma).
// One thread shuffles while the others wait at the barrier; it costs a few
// percent of an epoch.
//
// Layout: one workgroup per class. Thread t owns coordinates d = t + 256 j
// (j < kJ) of w, held in registers; the sample row is read as FP32 straight
// from the feature matrix (coalesced, one row ahead), scaled in FP64. alpha
// and the epoch's order live in LDS. One barrier per coordinate step (the
// dot product's cross-wave sum, double-buffered).
#include "gram.h"
#include "lbpf_internal.h"

#include <algorithm>

namespace lbpf {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Squared norms of the rows (one wave per row) and, with sigma given, the
// diagonal Q_ii = sum (sigma x)^2 + 1.
__global__ __launch_bounds__(kThreads) void k_row_norms(const float *__restrict__ X, int32_t N,
                                                        int32_t D, const double *__restrict__ sigma,
                                                        double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int32_t i = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (i >= N) return;
    const float *x = X + (size_t)i * D;
    const double s = sigma ? *sigma : 1.0;
    double acc = 0.0;
    for (int d = lane; d < D; d += 64) {
        const double v = s * (double)x[d];
        acc += v * v;
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) out[i] = sigma ? acc + 1.0 : sqrt(acc);
}

// sigma = 1 / (lower median of the norms), 1 when that median is 0: the
// element of rank (N-1)/2, ranks broken by index so exactly one qualifies.
__global__ __launch_bounds__(kThreads) void k_sigma(const double *__restrict__ norms, int32_t N,
                                                    double *__restrict__ sigma) {
    const uint32_t want = (uint32_t)(N - 1) / 2;
    for (int32_t i = threadIdx.x; i < N; i += kThreads) {
        const double v = norms[i];
        uint32_t rank = 0;
        for (int32_t j = 0; j < N; ++j) {
            const double u = norms[j];
            rank += (u < v || (u == v && j < i)) ? 1u : 0u;
        }
        if (rank == want) *sigma = v > 0.0 ? 1.0 / v : 1.0;
    }
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t state0, uint64_t m) {
    // Output of draw m (0-based) of a stream whose state starts at state0.
    uint64_t z = state0 + (m + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct TrainArgs {
    const float *X;
    const int32_t *labels;
    const double *sigma, *qii;
    int32_t N, D, K;
    double C, eps;
    int32_t max_epochs;
    uint64_t seed;
    int32_t warm;
    double *alpha;   // [K][N]: warm start in, final values out (may be null)
    float *W;        // [K][D]
    float *b;        // [K]
    double *W64;     // [K][D] or null
    double *b64;     // [K] or null
    int32_t *epochs; // [K] or null
};

template <int kJ>
__device__ __forceinline__ void load_row(const float *__restrict__ X, int32_t i, int32_t D, int tid,
                                         float (&x)[kJ]) {
    const float *row = X + (size_t)i * D;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const int d = tid + kThreads * j;
        x[j] = d < D ? row[d] : 0.0f;
    }
}

// One workgroup per class. Dynamic LDS: alpha (N doubles), order (N ints).
template <int kJ>
__global__ __launch_bounds__(kThreads) void k_train(TrainArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    double *alpha = reinterpret_cast<double *>(smem);
    int32_t *order = reinterpret_cast<int32_t *>(alpha + a.N);
    __shared__ double red[2][kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t k = blockIdx.x;
    const int32_t N = a.N, D = a.D;
    const double sigma = *a.sigma, C = a.C;
    const bool warm = a.warm && a.alpha;

    // w: coordinates tid + 256 j in registers; the bias weight wb is kept
    // by every thread (its updates are uniform).
    double w[kJ];
#pragma unroll
    for (int j = 0; j < kJ; ++j) w[j] = 0.0;
    double wb = 0.0;
    for (int32_t i = tid; i < N; i += kThreads) alpha[i] = warm ? a.alpha[(size_t)k * N + i] : 0.0;
    __syncthreads();
    if (warm) {
        // w = sum_i alpha_i y_i x_i over the scaled, augmented samples.
        for (int32_t i = 0; i < N; ++i) {
            const double ai = alpha[i];
            if (ai == 0.0) continue;
            const double ay = a.labels[i] == k ? ai : -ai;
            float x[kJ];
            load_row<kJ>(a.X, i, D, tid, x);
#pragma unroll
            for (int j = 0; j < kJ; ++j) w[j] += ay * (sigma * (double)x[j]);
            wb += ay;
        }
    }

    const uint64_t state0 = a.seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(k + 1));
    int32_t epoch = 0;
    while (epoch < a.max_epochs) {
        if (tid == 0) {
            const uint64_t base = (uint64_t)epoch * (uint64_t)(N - 1);
            for (int32_t i = 0; i < N; ++i) order[i] = i;
            for (int32_t i = N - 1; i > 0; --i) {
                const uint64_t r = splitmix64_at(state0, base + (uint64_t)(N - 1 - i));
                const int32_t j = (int32_t)(r % (uint64_t)(i + 1));
                const int32_t t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
        }
        __syncthreads();

        double max_pg = 0.0;
        float xn[kJ];
        load_row<kJ>(a.X, order[0], D, tid, xn);
        for (int32_t s = 0; s < N; ++s) {
            const int32_t i = order[s];
            float xc[kJ];
#pragma unroll
            for (int j = 0; j < kJ; ++j) xc[j] = xn[j];
            if (s + 1 < N) load_row<kJ>(a.X, order[s + 1], D, tid, xn);
            const double a_old = alpha[i];  // read before this step's barrier
            const double y = a.labels[i] == k ? 1.0 : -1.0;
            const double q = a.qii[i];
            double part = 0.0;
#pragma unroll
            for (int j = 0; j < kJ; ++j) part += w[j] * (sigma * (double)xc[j]);
            part = wave_sum_f64(part);
            if (lane == 0) red[s & 1][wave] = part;
            __syncthreads();
            double wx = red[s & 1][0];
#pragma unroll
            for (int v = 1; v < kWaves; ++v) wx += red[s & 1][v];
            wx += wb;
            const double G = y * wx - 1.0;
            double PG = G;
            if (a_old <= 0.0) PG = G < 0.0 ? G : 0.0;
            else if (a_old >= C) PG = G > 0.0 ? G : 0.0;
            max_pg = fmax(max_pg, fabs(PG));
            if (PG != 0.0 && q > 0.0) {
                const double a_new = fmin(fmax(a_old - G / q, 0.0), C);
                if (tid == 0) alpha[i] = a_new;
                const double step = (a_new - a_old) * y;
                if (step != 0.0) {
#pragma unroll
                    for (int j = 0; j < kJ; ++j) w[j] += step * (sigma * (double)xc[j]);
                    wb += step;
                }
            }
        }
        ++epoch;
        __syncthreads();  // order and alpha are rewritten next
        if (max_pg < a.eps) break;  // uniform: every thread holds the same max_pg
    }

#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const int d = tid + kThreads * j;
        if (d < D) {
            const double v = sigma * w[j];
            a.W[(size_t)k * D + d] = (float)v;
            if (a.W64) a.W64[(size_t)k * D + d] = v;
        }
    }
    if (tid == 0) {
        a.b[k] = (float)wb;
        if (a.b64) a.b64[k] = wb;
        if (a.epochs) a.epochs[k] = epoch;
    }
    if (a.alpha)
        for (int32_t i = tid; i < N; i += kThreads) a.alpha[(size_t)k * N + i] = alpha[i];
}

template <int kJ>
hipError_t launch_train_j(const TrainArgs &a, hipStream_t s) {
    const size_t lds = (size_t)a.N * (sizeof(double) + sizeof(int32_t));
    hipError_t e = hipFuncSetAttribute((const void *)k_train<kJ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_train<kJ>, dim3(a.K), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

// --- Gram form (FP32) ----------------------------------------------------------
//
// The same dual coordinate descent, restated on the Gram matrix G = X X^T of
// the unscaled features (one FP32 matrix-core GEMM). With s2 = sigma^2, the
// margin of sample i under the current duals is
//   w.x_i = s2 g_i + c,   g_i = sum_j alpha_j y_j G_ij,   c = sum_j alpha_j y_j
// (c is the bias feature's share), and a step on alpha_i moves g by
// (alpha_i' - alpha_i) y_i times row i of G (N values) and c by the same
// scalar. Most steps change nothing: a sample whose projected gradient is 0
// leaves alpha and g as they are. The solver wave therefore tests the next
// 64 samples of the epoch's order at once (one LDS read of g per lane), takes
// the first whose projected gradient is not 0, updates, and tests again from
// the sample after it: the same steps as visiting the samples one by one.
// A second wave draws the next epoch's order meanwhile. FP32 throughout.

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

typedef float gf4 __attribute__((ext_vector_type(4)));

// Eight 16-byte pieces of LDS at byte offsets 0, 1024, .., 7168 from addr,
// waited for in the same block: the eight results land in distinct registers,
// so the reads go out back to back. The outputs are early-clobber: a read
// that returns while later ones are still being issued must not land in the
// address register.
__device__ __forceinline__ void lds_read8(uint32_t addr, gf4 (&v)[8]) {
    asm volatile(
        "ds_read_b128 %0, %8\n\t"
        "ds_read_b128 %1, %8 offset:1024\n\t"
        "ds_read_b128 %2, %8 offset:2048\n\t"
        "ds_read_b128 %3, %8 offset:3072\n\t"
        "ds_read_b128 %4, %8 offset:4096\n\t"
        "ds_read_b128 %5, %8 offset:5120\n\t"
        "ds_read_b128 %6, %8 offset:6144\n\t"
        "ds_read_b128 %7, %8 offset:7168\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]), "=&v"(v[6]),
          "=&v"(v[7])
        : "v"(addr)
        : "memory");
}

__device__ __forceinline__ float readlane_f(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// The zero bias row of the Gram products.
__global__ __launch_bounds__(256) void k_gram_zero(float *__restrict__ z, int32_t n) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) z[i] = 0.0f;
}

// Row norms sqrt(G_ii).
__global__ __launch_bounds__(256) void k_gram_diag(const float *__restrict__ G, int32_t N,
                                                   float *__restrict__ norms) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < N) norms[i] = sqrtf(G[(size_t)i * N + i]);
}

// sigma = 1 / (lower median of the norms), 1 when that median is 0: the
// element of rank (N-1)/2, ties ranked by index.
__global__ __launch_bounds__(256) void k_gram_sigma(const float *__restrict__ norms, int32_t N,
                                                    float *__restrict__ sigma) {
    const uint32_t want = (uint32_t)(N - 1) / 2;
    for (int32_t i = blockIdx.x * 256 + threadIdx.x; i < N; i += gridDim.x * 256) {
        const float v = norms[i];
        uint32_t rank = 0;
        for (int32_t j = 0; j < N; ++j) {
            const float u = norms[j];
            rank += (u < v || (u == v && j < i)) ? 1u : 0u;
        }
        if (rank == want) *sigma = v > 0.0f ? 1.0f / v : 1.0f;
    }
}

// A[k][i] = alpha[k][i] y_ki, the left operand of a warm start's margins.
__global__ __launch_bounds__(256) void k_gram_alpha_y(const float *__restrict__ alpha,
                                                      const int32_t *__restrict__ labels,
                                                      int32_t N, int32_t K, float *__restrict__ A) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)N * K) return;
    const int32_t k = (int32_t)(e / (size_t)N), i = (int32_t)(e % (size_t)N);
    A[e] = labels[i] == k ? alpha[e] : -alpha[e];
}

constexpr size_t kGramLds = 160 * 1024 - 64;  // dynamic LDS of k_train_gram at most

struct GramArgs {
    const float *G;          // [N][N]
    const int32_t *labels;
    const float *sigma;
    const float *g0;         // [K][N] margins sum_j alpha_j y_j G_ij of a warm start, or null
    int32_t N, K;
    float C, eps;
    int32_t max_epochs;
    uint64_t seed;
    float *alpha;            // [K][N]: warm start in (with g0), final values out
    float *b;                // [K]
    int32_t *epochs;         // [K] or null
};

// Segment `seg` of `nseg` of epoch e's order (N entries): Fisher-Yates from
// the identity, i = N-1 down to 1 swapping i with r mod (i+1), r = draw
// e(N-1) + (N-1-i) of the class's splitmix64 stream; segment s takes the
// steps i in [max(1, N - (s+1) L), N-1 - s L], L = ceil((N-1) / nseg), and
// segment 0 first writes the identity. One wave: the draws of 64 swaps in
// parallel, then the swaps one after another by lane 0 (each needs the
// previous one's result).
__device__ void gram_order(int16_t *ord, int32_t N, uint64_t state0, int32_t e, int seg, int nseg,
                           int lane) {
    if (seg == 0)
        for (int32_t p = lane; p < N; p += 64) ord[p] = (int16_t)p;
    const int32_t L = (N - 1 + nseg - 1) / nseg;
    const int32_t hi = N - 1 - seg * L, lo = max(1, N - (seg + 1) * L);
    const uint64_t base = (uint64_t)e * (uint64_t)(N - 1);
    for (int32_t top = hi; top >= lo; top -= 64) {
        const int32_t i = top - lane;
        int32_t j = 0;
        if (i >= lo) {
            const uint64_t r = splitmix64_at(state0, base + (uint64_t)(N - 1 - i));
            j = (int32_t)(r % (uint64_t)(i + 1));
        }
        const int cnt = min(64, top - lo + 1);
        for (int t = 0; t < cnt; ++t) {
            const int32_t jt = __builtin_amdgcn_readlane(j, t);
            const int32_t it = top - t;
            if (lane == 0) {
                const int16_t u = ord[it], v = ord[jt];
                ord[it] = v;
                ord[jt] = u;
            }
        }
    }
}

// One workgroup per class: wave 0 solves, waves 1..W draw epoch orders
// (W = blockDim / 64 - 1). The order of epoch f is built by wave 1 + f mod W
// in W segments during the W epochs before f, so each wave does 1/W of an
// order per epoch and every epoch ends at one barrier; W + 1 order buffers
// (epoch f in buffer f mod (W + 1)). Dynamic LDS ((15 + 2W) N bytes): g,
// alpha, the diagonal s2 G_ii + 1 (FP32 each), y (int8), the orders (int16).
// kV4: the Gram rows are read as float4 (N % 4 == 0).
template <bool kV4>
__global__ __launch_bounds__(320) void k_train_gram(GramArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    const int32_t N = a.N;
    const int W = (int)(blockDim.x >> 6) - 1, B = W + 1;
    float *g = reinterpret_cast<float *>(smem);
    float *al = g + N;
    float *qd = al + N;
    int16_t *ord = reinterpret_cast<int16_t *>(qd + N);  // [W + 1][N]
    int8_t *ys = reinterpret_cast<int8_t *>(ord + (size_t)B * N);
    __shared__ int32_t done[2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t k = blockIdx.x;
    const float sig = *a.sigma, s2 = sig * sig, C = a.C;
    const bool warm = a.g0 != nullptr;
    for (int32_t i = tid; i < N; i += (int32_t)blockDim.x) {
        ys[i] = a.labels[i] == k ? 1 : -1;
        al[i] = warm ? a.alpha[(size_t)k * N + i] : 0.0f;
        g[i] = warm ? a.g0[(size_t)k * N + i] : 0.0f;
        qd[i] = s2 * a.G[(size_t)i * N + i] + 1.0f;
    }
    const uint64_t state0 = a.seed ^ (0x5851F42D4C957F2Dull * (uint64_t)(k + 1));
    __syncthreads();

    float c = 0.0f;  // solver wave: sum alpha y (the bias weight)
    if (wave == 0 && warm) {
        float part = 0.0f;
        for (int32_t i = lane; i < N; i += 64) part += ys[i] > 0 ? al[i] : -al[i];
        c = wave_sum_f32(part);
    }
    int32_t epoch = a.max_epochs;
    // e < 0: the first orders only.
    for (int32_t e = -W; e < a.max_epochs; ++e) {
        if (wave == 0) {
            if (e >= 0) {
                const int16_t *od = ord + (size_t)(e % B) * N;
                float max_pg = 0.0f;
                int32_t s = 0;
                while (s < N) {  // uniform
                    const int32_t p = s + lane;
                    const bool v = p < N;
                    const int32_t i = v ? od[p] : 0;
                    const float y = ys[i] > 0 ? 1.0f : -1.0f;
                    const float ai = al[i], qi = qd[i];
                    const float G = y * (s2 * g[i] + c) - 1.0f;
                    float PG = G;
                    if (ai <= 0.0f) PG = G < 0.0f ? G : 0.0f;
                    else if (ai >= C) PG = G > 0.0f ? G : 0.0f;
                    const uint64_t m = __ballot(v && PG != 0.0f);
                    if (m == 0) {
                        s += 64;
                        continue;
                    }
                    const int t = __builtin_ctzll(m);
                    const int32_t it = __builtin_amdgcn_readlane(i, t);
                    const float Gt = readlane_f(G, t), at = readlane_f(ai, t);
                    const float yt = readlane_f(y, t), q = readlane_f(qi, t);
                    max_pg = fmaxf(max_pg, fabsf(readlane_f(PG, t)));
                    if (q > 0.0f) {
                        const float an = fminf(fmaxf(at - Gt / q, 0.0f), C);
                        if (lane == 0) al[it] = an;
                        const float d = (an - at) * yt;
                        if (d != 0.0f) {
                            const float *row = a.G + (size_t)it * N;
                            if constexpr (kV4) {
                                // 24 float4 per lane in flight (a row of up
                                // to 6144 values in one round), then the
                                // updates.
                                typedef float f4 __attribute__((ext_vector_type(4)));
                                for (int32_t j0 = 4 * lane; j0 < N; j0 += 256 * 24) {
                                    // Every load unconditional, its address kept
                                    // inside the row (pieces past the end are
                                    // not used): guarded loads would keep the old
                                    // values of r alive across updates.
                                    f4 r[24];
#pragma unroll
                                    for (int u = 0; u < 24; ++u)
                                        r[u] = *reinterpret_cast<const f4 *>(row + min(j0 + 256 * u, N - 4));
                                    // Groups of eight pieces that lie inside g
                                    // for every lane (2048 (q + 1) <= N - j0 +
                                    // 4 lane): one LDS round trip a group; the
                                    // rest piece by piece.
                                    const int32_t nfull = (N - (j0 - 4 * lane)) / 2048;
#pragma unroll
                                    for (int q = 0; q < 3; ++q) {
                                        if (q < nfull) {  // uniform
                                            gf4 gv[8];
                                            lds_read8((uint32_t)(uintptr_t)(g + j0 + 2048 * q), gv);
#pragma unroll
                                            for (int u = 0; u < 8; ++u) {
                                                gf4 v = gv[u];
                                                const f4 ru = r[8 * q + u];
                                                v.x += d * ru.x;
                                                v.y += d * ru.y;
                                                v.z += d * ru.z;
                                                v.w += d * ru.w;
                                                *reinterpret_cast<gf4 *>(g + j0 + 2048 * q + 256 * u) = v;
                                            }
                                        } else {
                                            // Piece u lies inside g for every lane
                                            // when base + 256 (u + 1) <= N, for none
                                            // when base + 256 u >= N (uniform tests).
                                            const int32_t base = j0 - 4 * lane;
#pragma unroll
                                            for (int u = 8 * q; u < 8 * q + 8; ++u) {
                                                const int32_t j = j0 + 256 * u;
                                                if (base + 256 * u >= N) break;
                                                if (base + 256 * (u + 1) <= N || j < N) {
                                                    f4 gv = *reinterpret_cast<const f4 *>(g + j);
                                                    gv.x += d * r[u].x;
                                                    gv.y += d * r[u].y;
                                                    gv.z += d * r[u].z;
                                                    gv.w += d * r[u].w;
                                                    *reinterpret_cast<f4 *>(g + j) = gv;
                                                }
                                            }
                                        }
                                    }
                                }
                            } else {
#pragma unroll 8
                                for (int32_t j = lane; j < N; j += 64) g[j] += d * row[j];
                            }
                            c += d;
                        }
                    }
                    s += t + 1;
                }
                if (lane == 0) done[e & 1] = max_pg < a.eps;
            }
        } else {
            // The epoch f in [e + 1, e + W] with f = wave - 1 (mod W), at
            // its segment e - f + W.
            const int w = wave - 1;
            const int32_t f = e + 1 + (((w - (e + 1)) % W) + W) % W;
            if (f >= 0 && f < a.max_epochs)
                gram_order(ord + (size_t)(f % B) * N, N, state0, f, (int)(e - f + W), W, lane);
        }
        __syncthreads();
        if (e >= 0 && done[e & 1] != 0) {  // uniform
            epoch = e + 1;
            break;
        }
    }
    for (int32_t i = tid; i < N; i += (int32_t)blockDim.x) a.alpha[(size_t)k * N + i] = al[i];
    if (tid == 0) {
        a.b[k] = c;
        if (a.epochs) a.epochs[k] = epoch;
    }
}

// W_k = s2 sum_i alpha_ki y_ki x_i (samples in index order, zero duals
// skipped); thread t owns coordinates t + 256 j.
template <int kJ>
__global__ __launch_bounds__(256) void k_gram_weights(const float *__restrict__ X,
                                                      const int32_t *__restrict__ labels,
                                                      int32_t N, int32_t D,
                                                      const float *__restrict__ alpha,
                                                      const float *__restrict__ sigma,
                                                      float *__restrict__ W) {
    __shared__ float coef[1024];
    const int tid = threadIdx.x;
    const int32_t k = blockIdx.x;
    float acc[kJ];
#pragma unroll
    for (int j = 0; j < kJ; ++j) acc[j] = 0.0f;
    for (int32_t i0 = 0; i0 < N; i0 += 1024) {
        const int32_t n = min(1024, N - i0);
        __syncthreads();
        for (int32_t t = tid; t < n; t += 256) {
            const float av = alpha[(size_t)k * N + i0 + t];
            coef[t] = labels[i0 + t] == k ? av : -av;
        }
        __syncthreads();
        for (int32_t t = 0; t < n; ++t) {
            const float cf = coef[t];
            if (cf == 0.0f) continue;  // uniform
            const float *x = X + (size_t)(i0 + t) * D;
#pragma unroll
            for (int j = 0; j < kJ; ++j) {
                const int d = tid + 256 * j;
                if (d < D) acc[j] += cf * x[d];
            }
        }
    }
    const float sg = *sigma, s2 = sg * sg;
#pragma unroll
    for (int j = 0; j < kJ; ++j) {
        const int d = tid + 256 * j;
        if (d < D) W[(size_t)k * D + d] = s2 * acc[j];
    }
}

}  // namespace

size_t train_gram_workspace_bytes(int32_t N, int32_t K) {
    const size_t n = (size_t)N, kn = (size_t)K * N;
    return sizeof(float) * (n * n + 2 * n + 64 + 3 * kn);
}

hipError_t launch_train_gram(const float *X, const int32_t *labels, int32_t N, int32_t D,
                             int32_t K, float C, float eps, int32_t max_epochs, uint64_t seed,
                             float *alpha, int32_t warm, float *W, float *b, int32_t *epochs,
                             void *workspace, hipStream_t s) {
    const size_t n = (size_t)N, kn = (size_t)K * N;
    float *G = static_cast<float *>(workspace);
    float *norms = G + n * n;
    float *zeros = norms + n;
    float *sigma = zeros + n;
    float *A = sigma + 64;
    float *G0 = A + kn;
    float *al = alpha ? alpha : G0 + kn;
    const dim3 blk(256), rows((N + 255) / 256);
    hipLaunchKernelGGL(k_gram_zero, rows, blk, 0, s, zeros, N);
    hipError_t e = launch_score_f32(X, N, X, zeros, N, D, G, nullptr, s, 1, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_diag, rows, blk, 0, s, G, N, norms);
    hipLaunchKernelGGL(k_gram_sigma, rows, blk, 0, s, norms, N, sigma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const bool w = warm && alpha;
    if (w) {
        hipLaunchKernelGGL(k_gram_alpha_y, dim3((unsigned)((kn + 255) / 256)), blk, 0, s, alpha,
                           labels, N, K, A);
        if ((e = launch_score_f32(A, K, G, zeros, N, N, G0, nullptr, s, 1, nullptr)) != hipSuccess)
            return e;
    }
    GramArgs a{G, labels, sigma, w ? G0 : nullptr, N, K, C, eps, max_epochs, seed, al, b, epochs};
    // As many order waves (at most 4) as the LDS holds buffers for: (15 + 2W) N
    // bytes, W >= 1 for every N up to kGramMaxN.
    const int nw = (int)std::min<size_t>(4, (kGramLds / n - 15) / 2);
    const size_t lds = (15 + 2 * (size_t)nw) * n;
    const bool v4 = N % 4 == 0;
    const void *kern = v4 ? (const void *)k_train_gram<true> : (const void *)k_train_gram<false>;
    if ((e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
        return e;
    if (v4)
        hipLaunchKernelGGL(k_train_gram<true>, dim3(K), dim3(64 * (1 + nw)), lds, s, a);
    else
        hipLaunchKernelGGL(k_train_gram<false>, dim3(K), dim3(64 * (1 + nw)), lds, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    auto wts = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(K), blk, 0, s, X, labels, N, D, al, sigma, W);
    };
    if (D <= 4 * 256) wts(k_gram_weights<4>);
    else if (D <= 8 * 256) wts(k_gram_weights<8>);
    else if (D <= 16 * 256) wts(k_gram_weights<16>);
    else wts(k_gram_weights<32>);
    return hipGetLastError();
}

size_t train_workspace_bytes(int32_t N) { return ((size_t)2 * N + 1) * sizeof(double); }

hipError_t launch_train(const float *X, const int32_t *labels, int32_t N, int32_t D, int32_t K,
                        double C, double eps, int32_t max_epochs, uint64_t seed, double *alpha,
                        int32_t warm, float *W, float *b, double *W64, double *b64,
                        int32_t *epochs, void *workspace, hipStream_t s) {
    double *norms = static_cast<double *>(workspace);
    double *qii = norms + N;
    double *sigma = qii + N;
    const dim3 rows((N + kWaves - 1) / kWaves);
    hipLaunchKernelGGL(k_row_norms, rows, dim3(kThreads), 0, s, X, N, D, nullptr, norms);
    hipLaunchKernelGGL(k_sigma, dim3(1), dim3(kThreads), 0, s, norms, N, sigma);
    hipLaunchKernelGGL(k_row_norms, rows, dim3(kThreads), 0, s, X, N, D, sigma, qii);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TrainArgs a{X, labels, sigma, qii, N, D, K, C, eps, max_epochs, seed, warm, alpha,
                W, b, W64, b64, epochs};
    if (D <= 4 * kThreads) return launch_train_j<4>(a, s);
    if (D <= 8 * kThreads) return launch_train_j<8>(a, s);
    if (D <= 16 * kThreads) return launch_train_j<16>(a, s);
    return launch_train_j<32>(a, s);
}

}  // namespace lbpf
