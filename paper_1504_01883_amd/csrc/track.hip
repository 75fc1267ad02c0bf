// Nearest-centre tracking (Sec. 2.3, Fig. 4): a face is followed into the next
// frame by the detection whose box centre is nearest to the face's centre in
// the previous frame.
//
// Centres are kept doubled, (2x + w, 2y + h), so they are exact integers;
// distances are squared Euclidean distances of doubled centres in int64.
//   match[p] = nearest current box of the same stream for track p (lowest
//              index on ties), -1 if none lies within the gate;
//   owner[c] = among the tracks matched to box c, the nearest (lowest track
//              on ties), -1 if none: box c is a new face.
// Owners are resolved with one 64-bit atomicMin per track on the key
// (distance << 24) | track, which orders by distance and then track index.
#include "lbpf_internal.h"

namespace lbpf {

namespace {

constexpr int kThreads = 256;
constexpr uint64_t kNoKey = ~0ull;

__global__ __launch_bounds__(kThreads) void k_fill_keys(uint64_t *__restrict__ keys, int32_t C) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c < C) keys[c] = kNoKey;
}

// One wave per track.
__global__ __launch_bounds__(kThreads) void k_track(const int32_t *__restrict__ prev,
                                                    const int32_t *__restrict__ ps, int32_t P,
                                                    const int32_t *__restrict__ cur,
                                                    const int32_t *__restrict__ cs, int32_t C,
                                                    int64_t gate4, int32_t *__restrict__ match,
                                                    uint64_t *__restrict__ keys) {
    const int lane = threadIdx.x & 63;
    const int32_t p = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (p >= P) return;  // uniform per wave
    const int64_t px = 2 * (int64_t)prev[4 * p] + prev[4 * p + 2];
    const int64_t py = 2 * (int64_t)prev[4 * p + 1] + prev[4 * p + 3];
    const int32_t sp = ps[p];
    int64_t bd = INT64_MAX;
    int32_t bc = INT32_MAX;
    for (int32_t c = lane; c < C; c += 64) {  // c grows: a strict < keeps the lowest
        if (cs[c] != sp) continue;
        const int64_t dx = 2 * (int64_t)cur[4 * c] + cur[4 * c + 2] - px;
        const int64_t dy = 2 * (int64_t)cur[4 * c + 1] + cur[4 * c + 3] - py;
        const int64_t d = dx * dx + dy * dy;
        if (gate4 >= 0 && d > gate4) continue;
        if (d < bd) {
            bd = d;
            bc = c;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t od = __shfl_xor(bd, off, 64);
        const int32_t oc = __shfl_xor(bc, off, 64);
        if (od < bd || (od == bd && oc < bc)) {
            bd = od;
            bc = oc;
        }
    }
    if (lane == 0) {
        const bool found = bc != INT32_MAX;
        match[p] = found ? bc : -1;
        if (found) atomicMin((unsigned long long *)&keys[bc],
                             (unsigned long long)(((uint64_t)bd << 24) | (uint64_t)p));
    }
}

__global__ __launch_bounds__(kThreads) void k_owner(const uint64_t *__restrict__ keys, int32_t C,
                                                    int32_t *__restrict__ owner) {
    const int32_t c = blockIdx.x * kThreads + threadIdx.x;
    if (c < C) owner[c] = keys[c] == kNoKey ? -1 : (int32_t)(keys[c] & 0xFFFFFFu);
}

}  // namespace

hipError_t launch_track(const int32_t *prev, const int32_t *ps, int32_t P, const int32_t *cur,
                        const int32_t *cs, int32_t C, int64_t gate2, int32_t *match,
                        int32_t *owner, uint64_t *keys, hipStream_t s) {
    const int64_t gate4 = gate2 > 0 ? 4 * gate2 : -1;
    if (C > 0) hipLaunchKernelGGL(k_fill_keys, dim3((C + kThreads - 1) / kThreads), dim3(kThreads), 0, s, keys, C);
    if (P > 0)
        hipLaunchKernelGGL(k_track, dim3((P + 3) / 4), dim3(kThreads), 0, s, prev, ps, P, cur, cs,
                           C, gate4, match, keys);
    if (C > 0) hipLaunchKernelGGL(k_owner, dim3((C + kThreads - 1) / kThreads), dim3(kThreads), 0, s, keys, C, owner);
    return hipGetLastError();
}

}  // namespace lbpf
