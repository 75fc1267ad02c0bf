"""lbpf_score_noalloc (FP32 scoring with the library's static device scratch,
for callers that cannot allocate) against lbpf_score on the same inputs.

Two calls in a row, the second smaller, each with scores + argmax and
argmax only:
  * 5000 rows x 1024 identities: argmax-only runs in three passes of the
    static scratch;
  * 300 rows x 1024 identities: too few tiles to fill the GPU, so the
    feature dimension is split and the partial tiles go to the scratch.
Scores agree with lbpf_score's within the FP32 tolerance (1e-5 of the dot
product's condition scale), argmax equals the first maximum of the call's own
scores and lbpf_score's argmax wherever the top-2 margin exceeds twice the
tolerance; the oversized argmax-only request is refused before any work.
"""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu, score_tolerance, stacked_planes

pytestmark = pytest.mark.gpu

K = 1024


@pytest.fixture(scope="module")
def setup():
    require_gpu()
    ctx = lbpf.Context()
    g, z, _ = synth.make_crops(5000, 48, 48, synth.W_RAGGED, 97)
    planes, boxes = stacked_planes(g, z)
    X, _ = ctx.features(planes, boxes)
    W, b = synth.synthetic_weights(K, ctx.dim, synth.W_RAGGED)
    Wd, bd = torch.from_numpy(W).cuda(), torch.from_numpy(b).cuda()
    wts = ctx.weights(Wd, bd)
    torch.cuda.synchronize()
    yield ctx, X, Wd, bd, wts, W, b
    wts.close()
    ctx.close()


def check_rows(ctx, X, Wd, bd, wts, W, b, n):
    Xn = X[:n].contiguous()
    S_ref, A_ref = ctx.score(Xn, wts)
    S, A = lbpf.score_noalloc(Xn, Wd, bd)
    _, A_only = lbpf.score_noalloc(Xn, Wd, bd, want_scores=False)
    torch.cuda.synchronize()
    S_ref, A_ref = S_ref.cpu().numpy(), A_ref.cpu().numpy()
    S, A, A_only = S.cpu().numpy(), A.cpu().numpy(), A_only.cpu().numpy()
    tol = score_tolerance(Xn.cpu().numpy(), W, b)
    assert (np.abs(S.astype(np.float64) - S_ref) <= tol).all(), f"scores differ ({n} rows)"
    assert np.array_equal(A, np.argmax(S, axis=1))
    top2 = np.sort(S_ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * tol.max(axis=1)
    assert clear.mean() > 0.9
    assert np.array_equal(A[clear], A_ref[clear]), f"argmax differs ({n} rows)"
    assert np.array_equal(A_only[clear], A_ref[clear]), f"argmax-only differs ({n} rows)"


def test_noalloc_matches_score_two_calls(setup):
    ctx, X, Wd, bd, wts, W, b = setup
    half_floats = lbpf.NOALLOC_SCRATCH_BYTES // 8
    assert 5000 * K > half_floats  # argmax-only takes several passes
    check_rows(ctx, X, Wd, bd, wts, W, b, 5000)
    check_rows(ctx, X, Wd, bd, wts, W, b, 300)


def test_noalloc_rejects_oversized_argmax_only(setup):
    big_k = lbpf.NOALLOC_SCRATCH_BYTES // 8 + 1
    Xs = torch.zeros((1, 4), dtype=torch.float32, device="cuda")
    Wb = torch.zeros((big_k, 4), dtype=torch.float32, device="cuda")
    bb = torch.zeros((big_k,), dtype=torch.float32, device="cuda")
    with pytest.raises(lbpf.LbpfError) as ei:
        lbpf.score_noalloc(Xs, Wb, bb, want_scores=False)
    assert ei.value.status == lbpf.LBPF_E_BUDGET
