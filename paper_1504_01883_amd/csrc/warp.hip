// Warped face crops (Sec. 2.1, Eq. 1: p' = x u + y v + t, the affine frame
// that turns the mapped face region into a rectangle; Sec. 3: the face is
// resized to 200 x 200 before its features are taken).
//
// Crop pixel (x, y) reads the source pixel
//   sx = floor((ux x + vx y + tx) / 2^16),  sy = floor((uy x + vy y + ty) / 2^16)
// (16.16 fixed point, exact in 64-bit integers, nearest sample). The host has
// checked that the four corner samples, and so by linearity every sample,
// lie inside the plane; the kernel clamps anyway so that no frame can send a
// load outside the plane.
//
// One workgroup per crop, one wave per output row at a time: the stores of a
// row are contiguous (64 bytes of grey, 128 of depth per wave instruction);
// the loads follow the frame (contiguous for a resize, strided for a
// rotation).
#include "lbpf_internal.h"

namespace lbpf {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int32_t sample(int64_t a, int32_t lim) {
    const int64_t q = a >> 16;  // arithmetic shift: floor division by 2^16
    return (int32_t)min<int64_t>(max<int64_t>(q, 0), (int64_t)lim - 1);
}

__global__ __launch_bounds__(kThreads) void k_warp(const WarpDesc *__restrict__ descs) {
    const WarpDesc &d = descs[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int w = d.w, h = d.h;
    for (int y = wave; y < h; y += kThreads / 64) {
        const int64_t dgx = (int64_t)d.df[2] * y + d.df[4], dgy = (int64_t)d.df[3] * y + d.df[5];
        const int64_t ggx = (int64_t)d.gf[2] * y + d.gf[4], ggy = (int64_t)d.gf[3] * y + d.gf[5];
        for (int x = lane; x < w; x += 64) {
            const int32_t zx = sample(dgx + (int64_t)d.df[0] * x, d.src_w);
            const int32_t zy = sample(dgy + (int64_t)d.df[1] * x, d.src_h);
            d.d_dst[(size_t)y * w + x] = d.d_src[(size_t)zy * d.d_pitch + zx];
            if (d.g_src) {
                const int32_t gx = sample(ggx + (int64_t)d.gf[0] * x, d.src_w);
                const int32_t gy = sample(ggy + (int64_t)d.gf[1] * x, d.src_h);
                d.g_dst[(size_t)y * w + x] = d.g_src[(size_t)gy * d.g_pitch + gx];
            }
        }
    }
}

}  // namespace

hipError_t launch_warp(const WarpDesc *d, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_warp, dim3(n), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}

}  // namespace lbpf
