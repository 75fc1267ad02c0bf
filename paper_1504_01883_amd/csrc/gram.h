// On-device SVM training in the Gram form (train.hip), used by runtime.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbpf {

// Largest training set of the Gram solver: its per-class state (g, alpha,
// the diagonal, labels and two epoch orders: 17 bytes a sample) lives in LDS.
constexpr int32_t kGramMaxN = 8192;

// Workspace of launch_train_gram: the N x N Gram matrix X X^T, its row
// norms, sigma, a zero bias row, and for warm starts alpha y and its product
// with the Gram matrix ([K][N] each), plus [K][N] duals when the caller keeps
// none.
size_t train_gram_workspace_bytes(int32_t N, int32_t K);

// Gram matrix G = X X^T on the FP32 matrix-core GEMM (launch_score_f32 with
// X as both operands), sigma = 1 / lower median of sqrt(G_ii), then dual
// coordinate descent per class in FP32 (one workgroup per class), then W and
// b from the duals. alpha: [K][N] FP32 (in with warm, out), or null.
hipError_t launch_train_gram(const float *X, const int32_t *labels, int32_t N, int32_t D,
                             int32_t K, float C, float eps, int32_t max_epochs, uint64_t seed,
                             float *alpha, int32_t warm, float *W, float *b, int32_t *epochs,
                             void *workspace, hipStream_t s);

}  // namespace lbpf
