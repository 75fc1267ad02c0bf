"""GPU parity of the on-device SVM trainers (Sec. 2.5 one-vs-rest max margin)
against the FP64 oracle trainer.

FP64 solver (solver="f64"): the same dual coordinate descent over the same
seeded sample order in FP64; it differs from the oracle only in the summation
order of each D+1-term dot product (and of the row norms behind sigma), a
relative perturbation of about (D+1) * 2^-53 ~ 1e-12 per step. The
trajectories therefore agree far below the tolerance used here, 1e-6 of the
largest weight, while a wrong update (sign, clamp, step, bias, sigma or order)
moves the weights by O(1) of it.

Gram solver (solver="gram", FP32): the same steps in the same order, taken on
the FP32 Gram matrix with FP32 margins, so every margin carries FP32 rounding
(the Gram entries' sums over D products, and one rounding per update of the
margins). Its weights are held to 1e-4 of the largest oracle weight: an FP32
simulation of the solver on the 5,120-sample training set ends within 1e-5,
and a wrong update still moves the weights by O(1).
"""
import numpy as np
import pytest
import torch

from paper_1504_01883_amd import lbpf, synth
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

SEED = 150401883


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = lbpf.Context()
    yield c
    c.close()


def _train_set(ref, n_ident, per, side=64):
    g, z, lab = synth.make_training_set(n_ident, per, side, side, synth.W_TINY)
    n = len(lab)
    planes = [(g.reshape(n * side, side), z.reshape(n * side, side))]
    X, _, _ = ref.features(planes, synth.stacked_boxes(n, side, side), n_threads=8)
    return X, lab


def _close(got, want, rel=1e-6):
    scale = max(np.abs(want).max(), 1e-30)
    err = np.abs(got - want).max()
    assert err <= rel * scale, f"max |diff| {err:.3e} > {rel:g} * {scale:.3e}"


@pytest.mark.parametrize("n_ident,per,eps", [(10, 20, 1e-3), (32, 12, 1e-4)])
def test_cold_training_matches_oracle(ctx, ref, n_ident, per, eps):
    X, lab = _train_set(ref, n_ident, per)
    W_ref, b_ref, ep_ref = ref.train_ovr_f64(X, lab, n_ident, eps=eps, seed=SEED, n_threads=8)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), n_ident, eps=eps,
                    seed=SEED, want_f64=True, solver="f64")
    torch.cuda.synchronize()
    W64, b64 = out["W64"].cpu().numpy(), out["b64"].cpu().numpy()
    _close(W64, W_ref)
    _close(b64, b_ref, rel=1e-6 * max(1.0, np.abs(W_ref).max() / max(np.abs(b_ref).max(), 1e-30)))
    assert int(out["epochs"].max()) == ep_ref
    # FP32 outputs are the FP64 ones rounded to nearest.
    assert np.array_equal(out["W"].cpu().numpy(), W64.astype(np.float32))
    assert np.array_equal(out["b"].cpu().numpy(), b64.astype(np.float32))


def test_trained_weights_recognise(ctx, ref):
    """Weights from the device trainer classify held-out samples like the
    oracle's (the tiny workload's recognition, Sec. 2.5)."""
    X, lab = _train_set(ref, 10, 20)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), 10, seed=SEED,
                    solver="f64")
    g, z, tl = synth.make_crops(100, 64, 64, synth.W_TINY, 10)
    Xt, _, _ = ref.features([(g.reshape(6400, 64), z.reshape(6400, 64))],
                            synth.stacked_boxes(100, 64, 64), n_threads=8)
    W_ref, b_ref, _ = ref.train_ovr_f64(X, lab, 10, seed=SEED, n_threads=8)
    _, a_ref = ref.score_f64(Xt, W_ref.astype(np.float32), b_ref.astype(np.float32),
                             want_scores=False)
    _, a_gpu = ref.score_f64(Xt, out["W"].cpu().numpy(), out["b"].cpu().numpy(),
                             want_scores=False)
    assert np.array_equal(a_gpu, a_ref)
    assert (a_gpu == tl).mean() >= 0.9


def test_warm_start_from_the_solution_stops_after_one_epoch(ctx, ref):
    """Solved to eps = 1e-6, the duals restart a run with eps = 1e-3 that stops
    after its first epoch, with the weights rebuilt from the duals alone."""
    X, lab = _train_set(ref, 10, 20)
    Xd, ld = torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda()
    alpha = torch.zeros((10, len(lab)), dtype=torch.float64, device="cuda")
    cold = ctx.train(Xd, ld, 10, seed=SEED, alpha=alpha, eps=1e-6, max_epochs=5000,
                     want_f64=True, solver="f64")
    a = alpha.cpu().numpy()
    assert a.min() >= 0.0 and a.max() <= 1.0  # box constraints, C = 1
    assert int(cold["epochs"].max()) < 5000
    warm = ctx.train(Xd, ld, 10, seed=SEED, alpha=alpha, warm=True, eps=1e-3, want_f64=True,
                     solver="f64")
    torch.cuda.synchronize()
    assert warm["epochs"].cpu().numpy().tolist() == [1] * 10
    _close(warm["W64"].cpu().numpy(), cold["W64"].cpu().numpy(), rel=1e-3)


def test_incremental_enrolment(ctx, ref):
    """New samples labelled after training (Sec. 2.2-2.3: the database grows
    while faces are tracked): a warm start from the old duals with zeros for
    the new rows reaches a solution that recognises like a cold retrain."""
    X, lab = _train_set(ref, 10, 20)
    first = np.arange(len(lab)) % 20 < 14  # 14 of 20 samples per person first
    Xd = torch.from_numpy(np.ascontiguousarray(X[first])).cuda()
    ld = torch.from_numpy(np.ascontiguousarray(lab[first])).cuda()
    a_old = torch.zeros((10, int(first.sum())), dtype=torch.float64, device="cuda")
    ctx.train(Xd, ld, 10, seed=SEED, alpha=a_old, eps=1e-4, solver="f64")
    order = np.concatenate([np.flatnonzero(first), np.flatnonzero(~first)])
    alpha = torch.zeros((10, len(lab)), dtype=torch.float64, device="cuda")
    alpha[:, : int(first.sum())] = a_old
    Xa = torch.from_numpy(np.ascontiguousarray(X[order])).cuda()
    la = torch.from_numpy(np.ascontiguousarray(lab[order])).cuda()
    inc = ctx.train(Xa, la, 10, seed=SEED, alpha=alpha, warm=True, eps=1e-4, want_f64=True,
                    solver="f64")
    cold = ctx.train(Xa, la, 10, seed=SEED, eps=1e-4, want_f64=True, solver="f64")
    torch.cuda.synchronize()
    _close(inc["W64"].cpu().numpy(), cold["W64"].cpu().numpy(), rel=5e-2)
    g, z, _ = synth.make_crops(100, 64, 64, synth.W_TINY, 10)
    Xt, _, _ = ref.features([(g.reshape(6400, 64), z.reshape(6400, 64))],
                            synth.stacked_boxes(100, 64, 64), n_threads=8)
    _, a_inc = ref.score_f64(Xt, inc["W"].cpu().numpy(), inc["b"].cpu().numpy(), want_scores=False)
    _, a_cold = ref.score_f64(Xt, cold["W"].cpu().numpy(), cold["b"].cpu().numpy(),
                              want_scores=False)
    assert (a_inc == a_cold).mean() >= 0.98


def test_training_limits(ctx):
    X = torch.zeros((4, ctx.dim), dtype=torch.float32, device="cuda")
    lab = torch.zeros(4, dtype=torch.int32, device="cuda")
    for solver in ("f64", "gram"):
        with pytest.raises(lbpf.LbpfError):
            ctx.train(X, lab, 2, warm=True, solver=solver)  # warm start needs alpha
        with pytest.raises(lbpf.LbpfError):
            ctx.train(X, lab, 2, C=0.0, solver=solver)
    with pytest.raises(ValueError):
        ctx.train(X, lab, 2, want_f64=True)  # FP64 outputs only from the FP64 solver
    Xn = torch.zeros((8193, ctx.dim), dtype=torch.float32, device="cuda")
    ln = torch.zeros(8193, dtype=torch.int32, device="cuda")
    with pytest.raises(lbpf.LbpfError) as ei:
        ctx.train(Xn, ln, 2)  # the Gram solver's state lives in LDS: N <= 8192
    assert ei.value.status == lbpf.LBPF_E_UNSUPPORTED
    big = lbpf.Context(mapping=lbpf.MAP_FULL256)  # D = 32768 > 8192
    try:
        Xb = torch.zeros((4, big.dim), dtype=torch.float32, device="cuda")
        for solver in ("f64", "gram"):
            with pytest.raises(lbpf.LbpfError):
                big.train(Xb, lab, 2, solver=solver)
    finally:
        big.close()


@pytest.mark.parametrize("n_ident,per,eps,max_epochs", [(10, 20, 1e-3, 200), (32, 12, 1e-4, 200),
                                                        (16, 16, 1e-6, 40), (10, 19, 1e-4, 200)])
def test_gram_training_matches_oracle(ctx, ref, n_ident, per, eps, max_epochs):
    """The FP32 Gram solver against the FP64 oracle trainer: weights and
    biases within 1e-4 of the largest weight, the same epoch count (40-epoch
    cap at eps = 1e-6, where neither converges). N = 190 is not a multiple of
    4: the solver reads the Gram rows one value per lane."""
    X, lab = _train_set(ref, n_ident, per)
    W_ref, b_ref, ep_ref = ref.train_ovr_f64(X, lab, n_ident, eps=eps, max_epochs=max_epochs,
                                             seed=SEED, n_threads=8)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), n_ident, eps=eps,
                    max_epochs=max_epochs, seed=SEED)
    torch.cuda.synchronize()
    W, b = out["W"].cpu().numpy().astype(np.float64), out["b"].cpu().numpy().astype(np.float64)
    scale = np.abs(W_ref).max()
    assert np.abs(W - W_ref).max() <= 1e-4 * scale
    assert np.abs(b - b_ref).max() <= 1e-4 * max(scale, np.abs(b_ref).max())
    assert int(out["epochs"].max()) == ep_ref


def _histogram_rows(rng, N, D, labels, n_lab):
    """Seeded stand-ins for feature rows: non-negative, unit sum (as the
    normalised histograms are), drawn around one random centre per label."""
    centres = rng.gamma(0.3, size=(max(n_lab, 1), D))
    X = centres[labels] + rng.gamma(0.3, size=(N, D))
    return (X / X.sum(axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("N,K,n_lab,max_epochs", [(8192, 3, 2, 3), (8191, 5, 4, 3), (1, 2, 1, 200),
                                                  (6, 3, 2, 200)])
def test_gram_training_edge_cases(ctx, ref, N, K, n_lab, max_epochs):
    """The Gram solver at its size limit and at the degenerate ends, against
    the FP64 oracle trainer: N = 8192 (the largest N its LDS state allows,
    four-float Gram rows, two order waves), N = 8191 (one value per lane),
    one sample, six samples; the last class of every case has no positive
    sample (labels < n_lab < K). Same bar as the other cases: weights and
    biases within 1e-4 of the largest weight, the same epoch count."""
    rng = np.random.default_rng(N)
    lab = rng.integers(0, n_lab, N).astype(np.int32)
    lab[:n_lab] = np.arange(n_lab)  # every label below n_lab present
    X = _histogram_rows(rng, N, ctx.dim, lab, n_lab)
    W_ref, b_ref, ep_ref = ref.train_ovr_f64(X, lab, K, max_epochs=max_epochs, seed=SEED,
                                             n_threads=8)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), K,
                    max_epochs=max_epochs, seed=SEED)
    torch.cuda.synchronize()
    W, b = out["W"].cpu().numpy().astype(np.float64), out["b"].cpu().numpy().astype(np.float64)
    scale = np.abs(W_ref).max()
    assert scale > 0
    assert np.abs(W - W_ref).max() <= 1e-4 * scale
    assert np.abs(b - b_ref).max() <= 1e-4 * max(scale, np.abs(b_ref).max())
    assert int(out["epochs"].max()) == ep_ref


def test_gram_weights_recognise(ctx, ref):
    """Weights from the Gram solver classify held-out samples like the
    oracle's."""
    X, lab = _train_set(ref, 10, 20)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), 10, seed=SEED)
    g, z, tl = synth.make_crops(100, 64, 64, synth.W_TINY, 10)
    Xt, _, _ = ref.features([(g.reshape(6400, 64), z.reshape(6400, 64))],
                            synth.stacked_boxes(100, 64, 64), n_threads=8)
    W_ref, b_ref, _ = ref.train_ovr_f64(X, lab, 10, seed=SEED, n_threads=8)
    _, a_ref = ref.score_f64(Xt, W_ref.astype(np.float32), b_ref.astype(np.float32),
                             want_scores=False)
    _, a_gpu = ref.score_f64(Xt, out["W"].cpu().numpy(), out["b"].cpu().numpy(),
                             want_scores=False)
    assert np.array_equal(a_gpu, a_ref)
    assert (a_gpu == tl).mean() >= 0.9


def test_gram_warm_start_from_the_solution_stops_after_one_epoch(ctx, ref):
    """Solved to eps = 1e-5, the FP32 duals restart a run with eps = 1e-3 that
    stops after its first epoch, the margins rebuilt from the duals (a Gram
    product) and the weights from the duals alone."""
    X, lab = _train_set(ref, 10, 20)
    Xd, ld = torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda()
    alpha = torch.zeros((10, len(lab)), dtype=torch.float32, device="cuda")
    cold = ctx.train(Xd, ld, 10, seed=SEED, alpha=alpha, eps=1e-5, max_epochs=5000)
    a = alpha.cpu().numpy()
    assert a.min() >= 0.0 and a.max() <= 1.0  # box constraints, C = 1
    assert int(cold["epochs"].max()) < 5000
    warm = ctx.train(Xd, ld, 10, seed=SEED, alpha=alpha, warm=True, eps=1e-3)
    torch.cuda.synchronize()
    assert warm["epochs"].cpu().numpy().tolist() == [1] * 10
    _close(warm["W"].cpu().numpy(), cold["W"].cpu().numpy(), rel=1e-3)


def test_gram_incremental_enrolment(ctx, ref):
    """Incremental enrolment with the Gram solver: a warm start from the old
    duals, zeros for the new rows, recognises like a cold retrain."""
    X, lab = _train_set(ref, 10, 20)
    first = np.arange(len(lab)) % 20 < 14
    Xd = torch.from_numpy(np.ascontiguousarray(X[first])).cuda()
    ld = torch.from_numpy(np.ascontiguousarray(lab[first])).cuda()
    a_old = torch.zeros((10, int(first.sum())), dtype=torch.float32, device="cuda")
    ctx.train(Xd, ld, 10, seed=SEED, alpha=a_old, eps=1e-4)
    order = np.concatenate([np.flatnonzero(first), np.flatnonzero(~first)])
    alpha = torch.zeros((10, len(lab)), dtype=torch.float32, device="cuda")
    alpha[:, : int(first.sum())] = a_old
    Xa = torch.from_numpy(np.ascontiguousarray(X[order])).cuda()
    la = torch.from_numpy(np.ascontiguousarray(lab[order])).cuda()
    inc = ctx.train(Xa, la, 10, seed=SEED, alpha=alpha, warm=True, eps=1e-4)
    cold = ctx.train(Xa, la, 10, seed=SEED, eps=1e-4)
    torch.cuda.synchronize()
    _close(inc["W"].cpu().numpy(), cold["W"].cpu().numpy(), rel=5e-2)
    g, z, _ = synth.make_crops(100, 64, 64, synth.W_TINY, 10)
    Xt, _, _ = ref.features([(g.reshape(6400, 64), z.reshape(6400, 64))],
                            synth.stacked_boxes(100, 64, 64), n_threads=8)
    _, a_inc = ref.score_f64(Xt, inc["W"].cpu().numpy(), inc["b"].cpu().numpy(), want_scores=False)
    _, a_cold = ref.score_f64(Xt, cold["W"].cpu().numpy(), cold["b"].cpu().numpy(),
                              want_scores=False)
    assert (a_inc == a_cold).mean() >= 0.98


def test_gram_training_full_size_matches_oracle(ctx, ref):
    """The enrolment workload at its full size: 256 identities x 20 crops of
    128 x 128 (5,120 samples, D = 7,552), C = 1, eps = 1e-6, the 200-epoch
    cap. All 256 classes train on the device; the oracle trainer recomputes
    four of them (one-vs-rest classes are independent, so the others are
    relabelled as the rest) from its own features."""
    g, z, lab = synth.make_training_set(256, 20, 128, 128, synth.W_UNIFORM)
    n = len(lab)
    X, _, _ = ref.features([(g.reshape(n * 128, 128), z.reshape(n * 128, 128))],
                           synth.stacked_boxes(n, 128, 128), n_threads=16)
    out = ctx.train(torch.from_numpy(X).cuda(), torch.from_numpy(lab).cuda(), 256, seed=SEED)
    torch.cuda.synchronize()
    m = 4
    lab_s = np.where(lab < m, lab, m).astype(np.int32)
    W_ref, b_ref, ep_ref = ref.train_ovr_f64(X, lab_s, m, seed=SEED, n_threads=m)
    W = out["W"].cpu().numpy()[:m].astype(np.float64)
    b = out["b"].cpu().numpy()[:m].astype(np.float64)
    scale = np.abs(W_ref).max()
    assert np.abs(W - W_ref).max() <= 1e-4 * scale
    assert np.abs(b - b_ref).max() <= 1e-4 * max(scale, np.abs(b_ref).max())
    assert ep_ref == 200 and out["epochs"].cpu().numpy().tolist() == [200] * 256
