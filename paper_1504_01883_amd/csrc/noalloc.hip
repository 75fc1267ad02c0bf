// FP32 scoring for callers that cannot allocate device memory (lbpf.h:
// lbpf_score_noalloc). The same kernels as lbpf_score's FP32 path; the
// scratch they need (the scores of argmax-only passes, the partial tiles of a
// split feature dimension) lives in a static device array of fixed size
// instead of a context's workspace.
#include <algorithm>
#include <mutex>
#include <string>

#include "lbpf_internal.h"

namespace lbpf {

namespace {

constexpr size_t kScratchFloats = LBPF_NOALLOC_SCRATCH_BYTES / sizeof(float);
// Argmax-only calls keep each pass's scores in the first half and the split
// partials in the second; calls with caller scores give all of it to the
// partials.
constexpr size_t kHalf = kScratchFloats / 2;

// One copy per GPU, held until the process ends. Host code never names it
// (in host code the name is a stand-in, not a device address): the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    float *ptr = nullptr;
    int32_t num_cus = 0;
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

// The current device's scratch address and CU count, looked up on the first
// call on that device (with it current).
hipError_t device_scratch(DeviceScratch &out, std::string &what) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        what = "hipGetDevice";
        return e;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        what = "device ordinal above the supported 64";
        return hipErrorInvalidDevice;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            what = "hipGetSymbolAddress(scratch)";
            return e;
        }
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) {
            what = "hipDeviceGetAttribute";
            return e;
        }
        d.num_cus = cus;
        d.ptr = static_cast<float *>(p);
    }
    out = d;
    return hipSuccess;
}

}  // namespace

}  // namespace lbpf

using namespace lbpf;

extern "C" lbpf_status lbpf_score_noalloc(const float *hist, int32_t N, const float *W,
                                          const float *b, int32_t K, int32_t D,
                                          float *scores_opt, int32_t *argmax_opt, void *stream) {
    if (N < 0 || K < 1 || D < 1) return set_last_error(LBPF_E_INVALID, "N < 0, K < 1 or D < 1");
    if (!scores_opt && !argmax_opt) return set_last_error(LBPF_E_INVALID, "no output requested");
    if (N == 0) return LBPF_OK;
    if (!hist || !W || !b) return set_last_error(LBPF_E_INVALID, "hist, W or b is NULL");
    if (!scores_opt && (size_t)K > kHalf)
        return set_last_error(LBPF_E_BUDGET,
                              "argmax-only scoring needs K <= LBPF_NOALLOC_SCRATCH_BYTES / 8 "
                              "(one row of scores in half of the static scratch)");
    DeviceScratch ds;
    std::string what;
    hipError_t e = device_scratch(ds, what);
    if (e != hipSuccess) return set_last_error(LBPF_E_HIP, what + ": " + hipGetErrorString(e));
    hipStream_t s = (hipStream_t)stream;
    const size_t Kz = (size_t)K, Dz = (size_t)D;
    // Rows per pass: all of them into the caller's scores, otherwise as many
    // rows of scores as half of the scratch holds.
    const int32_t rows = scores_opt ? N : (int32_t)std::min<size_t>((size_t)N, kHalf / Kz);
    float *part = scores_opt ? ds.ptr : ds.ptr + kHalf;
    const size_t part_elems = scores_opt ? kScratchFloats : kHalf;
    for (int32_t n0 = 0; n0 < N; n0 += rows) {
        const int32_t n = std::min(rows, N - n0);
        float *S = scores_opt ? scores_opt + (size_t)n0 * Kz : ds.ptr;
        const int32_t sp = score_f32_splits(n, K, D, ds.num_cus, part_elems);
        e = launch_score_f32(hist + (size_t)n0 * Dz, n, W, b, K, D, S,
                             argmax_opt ? argmax_opt + n0 : nullptr, s, sp, part);
        if (e != hipSuccess)
            return set_last_error(LBPF_E_HIP, std::string("score launch: ") + hipGetErrorString(e));
    }
    return LBPF_OK;
}
