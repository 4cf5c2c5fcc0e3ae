"""Pin of the CPU reference MLP (oracle/mlp_ref.py): its chain-rule gradient
equals central finite differences of its loss."""
import numpy as np

from oracle import mlp_ref


def init(F, H1, H2, seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.5, size=mlp_ref.num_params(F, H1, H2))
    p[:F] = rng.normal(size=F)            # mean
    p[F:2 * F] = rng.uniform(0.5, 2, F)   # inv_std
    return p


def test_gradient_matches_finite_differences():
    F, H1, H2, N = 5, 7, 6, 40
    rng = np.random.default_rng(1)
    X = rng.normal(size=(N, F))
    y = rng.normal(size=N)
    p = init(F, H1, H2, 2)
    L0, g = mlp_ref.loss_grad(p, F, H1, H2, X, y)
    assert L0 == mlp_ref.loss(p, F, H1, H2, X, y)
    h = 1e-6
    for i in range(2 * F, p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp_ref.loss(p + e, F, H1, H2, X, y) - mlp_ref.loss(p - e, F, H1, H2, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i
    assert np.all(g[:2 * F] == 0)


def test_forward_special_case_linear():
    """With all hidden pre-activations positive the network is affine:
    yhat = W3 W2 W1 z + W3 W2 b1 + W3 b2 + b3."""
    F, H1, H2 = 3, 4, 2
    rng = np.random.default_rng(3)
    w = {"mean": np.zeros(F), "istd": np.ones(F), "W1": rng.uniform(0, 1, (H1, F)),
         "b1": np.full(H1, 5.0), "W2": rng.uniform(0, 1, (H2, H1)), "b2": np.full(H2, 5.0),
         "W3": rng.normal(size=H2), "b3": np.array([0.3])}
    p = np.concatenate([w["mean"], w["istd"], w["W1"].ravel(), w["b1"], w["W2"].ravel(), w["b2"],
                        w["W3"], w["b3"]])
    X = rng.uniform(0, 1, (10, F))
    yhat, _ = mlp_ref.forward(p, F, H1, H2, X)
    ref = X @ (w["W3"] @ w["W2"] @ w["W1"]).T + w["W3"] @ w["W2"] @ w["b1"] + w["W3"] @ w["b2"] + 0.3
    assert np.allclose(yhat, ref, rtol=1e-13, atol=1e-13)
