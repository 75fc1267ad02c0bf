"""Scoring calls larger than one pass of the library's scratch (Sec. 2.5 at
the precision workload's scale).

* Reduced precision quantises the feature rows in chunks of 16,384 rows: with
  N = 2 * 16384 + 1 distinct rows every chunk (including a one-row tail) is
  compared row by row with the exact FP64 product of the quantised operands
  at the FP32 accumulation tolerance, and the argmax with the FP64 oracle.
* FP32 products whose tiles fill the GPU (no split of D): on every such
  kernel shape the argmax is the first maximum of the scores, with exact
  ties planted inside a lane's columns, across lanes, wave halves and tiles.
* FP32 argmax-only scoring (no caller score buffer) runs in passes of
  16 M / K rows through the context's score scratch: with N * K above 16 M
  the argmax of every row equals the argmax of the same call with caller
  scores, and sampled rows of every pass (the pass boundaries included)
  match the FP64 oracle at the FP32 tolerance.
"""
import hashlib

import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, score_tolerance, stacked_planes
from tests.lp_ref import lp_tolerance, quantised_reference

pytestmark = pytest.mark.gpu

LP_CHUNK = 16384
N_LP = 2 * LP_CHUNK + 1
K_LP = 264             # >= 256 and off the 256-wide tile grid: the large-tile kernel
SCRATCH_ELEMS = 16 << 20
K_F32 = 2048           # 8192 rows per argmax-only pass
N_F32 = 2 * (SCRATCH_ELEMS // K_F32) + 1


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


def distinct_rows(ctx, n, base=8192):
    """n distinct feature rows: the features of `base` seeded 48x48 crops,
    block j (rows j*base ..) cyclically shifted by j whole 59-bin cells, so
    every row is a valid-looking histogram and no row repeats."""
    g, z, _ = synth.make_crops(base, 48, 48, synth.W_PRECISION, 211)
    planes, boxes = stacked_planes(g, z)
    X0, _ = ctx.features(planes, boxes)
    blocks = [torch.roll(X0, shifts=59 * j, dims=1) for j in range((n + base - 1) // base)]
    X = torch.cat(blocks)[:n].contiguous()
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    digests = {hashlib.blake2b(r.tobytes(), digest_size=16).digest() for r in Xh}
    assert len(digests) == n, "feature rows are not distinct"
    return X, Xh


@pytest.fixture(scope="module")
def lp_data(ctx, ref):
    X, Xh = distinct_rows(ctx, N_LP)
    W, b = synth.synthetic_weights(K_LP, ctx.dim, synth.W_PRECISION)
    S64, A64 = ref.score_f64(Xh, W, b, n_threads=16)
    return X, Xh, W, b, S64, A64


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp8", "f16x3"])
def test_lp_every_chunk_matches_quantised_reference(ctx, lp_data, prec):
    X, Xh, W, b, S64, A64 = lp_data
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda(), precision=prec)
    S, A = ctx.score(X, wts)
    _, A_only = ctx.score(X, wts, want_scores=False)
    torch.cuda.synchronize()
    S = S.cpu().numpy()
    A, A_only = A.cpu().numpy(), A_only.cpu().numpy()
    wts.close()
    ref, scale = quantised_reference(Xh, W, b, prec)
    err = np.abs(S.astype(np.float64) - ref)
    tol = lp_tolerance(prec, ctx.dim)
    bad = np.nonzero((err > tol * scale + 1e-30).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} rows off, first {bad[:5]} (chunk {bad[0] // LP_CHUNK})"
    # The argmax (with and without caller scores) is the first maximum of the
    # scores, in every chunk.
    assert np.array_equal(A, np.argmax(S, axis=1))
    assert np.array_equal(A_only, A)
    # Against the FP64 oracle on the unquantised operands: wherever the
    # oracle's top-2 margin exceeds twice this row's largest score error the
    # identities must agree (lowest index on ties, Sec. 2.5).
    e_row = np.abs(S.astype(np.float64) - S64).max(axis=1)
    top2 = np.sort(S64, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * e_row
    assert np.array_equal(A[clear], A64[clear])
    agree = float((A == A64).mean())
    print(f"{prec}: {N_LP} rows, max |S - S64| {np.abs(S - S64).max():.3e}, "
          f"argmax agreement {agree:.4f} ({clear.mean():.4f} of rows clear of the error)")
    # Each full chunk has rows clear of the error, so the oracle comparison
    # above reaches every chunk (the one-row tail chunk is covered by the
    # exact comparison alone: its row may sit within the error of a tie).
    for c in range(2):
        assert clear[c * LP_CHUNK:(c + 1) * LP_CHUNK].any()


def test_fp32_argmax_only_multipass(ctx, ref):
    X, Xh = distinct_rows(ctx, N_F32)
    W, b = synth.synthetic_weights(K_F32, ctx.dim, synth.W_RAGGED)
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda())
    assert N_F32 * K_F32 > SCRATCH_ELEMS
    S, A = ctx.score(X, wts)
    _, A_only = ctx.score(X, wts, want_scores=False)
    torch.cuda.synchronize()
    S, A, A_only = S.cpu().numpy(), A.cpu().numpy(), A_only.cpu().numpy()
    wts.close()
    assert np.array_equal(A, np.argmax(S, axis=1))
    rows_per_pass = SCRATCH_ELEMS // K_F32
    # Full passes run the same unsplit kernel as the call with scores: the
    # same sums, so the same argmax, bit for bit. The one-row tail pass is too
    # small to fill the GPU and splits D (partials added in order), which may
    # round differently: there the argmax must agree wherever the top-2 margin
    # of the scores exceeds the FP32 tolerance.
    full = 2 * rows_per_pass
    assert np.array_equal(A_only[:full], A[:full]), \
        f"argmax-only differs in rows {np.nonzero(A_only[:full] != A[:full])[0][:8]}"
    tail = Xh[full:]
    tol_tail = score_tolerance(tail, W, b).max(axis=1)
    top2 = np.sort(S[full:], axis=1)[:, -2:]
    margin_ok = (top2[:, 1] - top2[:, 0]) > 2 * tol_tail
    assert np.array_equal(A_only[full:][margin_ok], A[full:][margin_ok])
    rng = np.random.default_rng(21)
    edges = [0, 1, rows_per_pass - 1, rows_per_pass, rows_per_pass + 1, 2 * rows_per_pass - 1,
             2 * rows_per_pass, N_F32 - 1]
    sample = np.unique(np.concatenate([edges, rng.integers(0, N_F32, 56)]))
    S64, A64 = ref.score_f64(Xh[sample], W, b, n_threads=16)
    tol = score_tolerance(Xh[sample], W, b)
    assert (np.abs(S[sample].astype(np.float64) - S64) <= tol).all()
    top2 = np.sort(S64, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * tol.max(axis=1)
    assert np.array_equal(A[sample][clear], A64[clear])


@pytest.mark.parametrize("N,K", [(16384, 1024), (16384, 1000), (8197, 1024), (4096, 1000)])
def test_fp32_unsplit_argmax_first_maximum(ctx, N, K):
    """Unsplit FP32 products and their argmax: 128 x 256 tiles (16384 x
    1024, and 16384 x 1000 with a partial last tile), 128 x 128 tiles on the
    two-stage ring (8197 x 1024, a ragged row tile) and on the four-stage
    ring (4096 x 1000). Two groups of identities share a weight row and bias
    each: group A (3,
    35, 700: one lane's columns j = 0 and 1, another tile) weighs the first
    half of the features, group B (129, 160, 900: two lanes of the upper half
    of a tile, another tile) the second half, and every other identity is
    small, so each row's best score is tied within one group. The scores of
    a group must be equal bit for bit (the same sums), and the argmax must be
    the first maximum of the scores: 3 or 129 (lowest index on ties,
    Sec. 2.5)."""
    D = ctx.dim
    gen = torch.Generator(device="cuda").manual_seed(N + K)
    X = torch.rand((N, D), device="cuda", generator=gen)
    X /= X.sum(dim=1, keepdim=True)
    rng = np.random.default_rng(K)
    W = (0.01 * rng.standard_normal((K, D))).astype(np.float32)
    b = (0.01 * rng.standard_normal(K)).astype(np.float32)
    ga, gb = [3, 35, 700], [129, 160, 900]
    W[ga] = np.concatenate([np.ones(D // 2), np.zeros(D - D // 2)]).astype(np.float32)
    W[gb] = np.concatenate([np.zeros(D // 2), np.ones(D - D // 2)]).astype(np.float32)
    b[ga], b[gb] = 0.25, 0.25
    wts = ctx.weights(torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda())
    S, A = ctx.score(X, wts)
    _, A_only = ctx.score(X, wts, want_scores=False)
    torch.cuda.synchronize()
    S, A, A_only = S.cpu().numpy(), A.cpu().numpy(), A_only.cpu().numpy()
    wts.close()
    for grp in (ga, gb):
        assert all(np.array_equal(S[:, grp[0]], S[:, k]) for k in grp[1:])
    assert np.array_equal(A, np.argmax(S, axis=1))
    assert np.array_equal(A_only, A)
    assert set(np.unique(A).tolist()) == {3, 129}
