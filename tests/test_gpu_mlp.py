"""GPU MLP kernels (forward, backward, Adam) against the CPU reference."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_12627_amd import ustat
    ustat.load_library()
    return ustat


def init(F, H1, H2, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.4, size=mlp_ref.num_params(F, H1, H2))
    p[:F] = rng.normal(size=F)
    p[F:2 * F] = rng.uniform(0.5, 2, F)
    return p.astype(np.float32)


@pytest.mark.parametrize("F,H1,H2,N", [(15, 64, 64, 3000), (5, 7, 6, 257)])
def test_gradients_match_cpu_reference(U, F, H1, H2, N):
    print(f"mlp grad F={F} H=({H1},{H2}) N={N}", flush=True)
    assert U.ustat_mlp_num_params(F, H1, H2) == mlp_ref.num_params(F, H1, H2)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(N, F)).astype(np.float32)
    y = rng.normal(size=N).astype(np.float32)
    p = init(F, H1, H2, 5)
    loss, g = U.ustat_mlp_loss_grad(F, H1, H2, p, X, y)
    Lr, gr = mlp_ref.loss_grad(p.astype(np.float64), F, H1, H2, X.astype(np.float64), y)
    assert loss == pytest.approx(Lr, rel=1e-5)
    scale = np.max(np.abs(gr))
    assert np.max(np.abs(g - gr)) <= 1e-4 * scale
    yhat = U.ustat_mlp_predict(F, H1, H2, p, X)
    yr, _ = mlp_ref.forward(p.astype(np.float64), F, H1, H2, X.astype(np.float64))
    assert np.max(np.abs(yhat - yr)) <= 1e-4 * max(1.0, np.max(np.abs(yr)))
    # reproducible
    loss2, g2 = U.ustat_mlp_loss_grad(F, H1, H2, p, X, y)
    assert loss2 == loss and np.array_equal(g2, g)


def test_training_lowers_held_out_loss(U):
    """Fit a teacher network: Adam on the GPU lowers train and held-out MSE."""
    F, H1, H2 = 8, 32, 32
    rng = np.random.default_rng(6)
    teacher = init(F, 16, 16, 7)
    X = rng.normal(size=(4000, F)).astype(np.float32)
    y, _ = mlp_ref.forward(teacher.astype(np.float64), F, 16, 16, X.astype(np.float64))
    y = y.astype(np.float32)
    p0 = init(F, H1, H2, 8)
    p0[:F] = 0.0
    p0[F:2 * F] = 1.0
    Xtr, ytr, Xte, yte = X[:3000], y[:3000], X[3000:], y[3000:]
    print("mlp train", flush=True)
    p, losses = U.ustat_mlp_train(F, H1, H2, p0, Xtr, ytr, steps=800, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0]
    before = mlp_ref.loss(p0.astype(np.float64), F, H1, H2, Xte, yte)
    after = mlp_ref.loss(p.astype(np.float64), F, H1, H2, Xte, yte)
    assert after < 0.3 * before
