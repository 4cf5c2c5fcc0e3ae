"""CPU ORACLE -- test infrastructure only.

Reference forward and backward pass of the cost-model MLP in fp64, written
from the definitions: standardised input z = (x - mean) * inv_std,
h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), yhat = W3 h2 + b3, loss =
mean (yhat - y)^2.  Parameters use the same flat layout as the engine:
mean[F] inv_std[F] W1[H1*F] b1[H1] W2[H2*H1] b2[H2] W3[H2] b3[1].
Pinned in tests/test_oracle_mlp.py by central finite differences.
"""
import numpy as np


def unpack(p, F, H1, H2):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    out = {}
    for name, size, shape in (("mean", F, (F,)), ("istd", F, (F,)), ("W1", H1 * F, (H1, F)),
                              ("b1", H1, (H1,)), ("W2", H2 * H1, (H2, H1)), ("b2", H2, (H2,)),
                              ("W3", H2, (H2,)), ("b3", 1, (1,))):
        out[name] = p[o:o + size].reshape(shape)
        o += size
    assert o == p.size
    return out


def num_params(F, H1, H2):
    return 2 * F + H1 * F + H1 + H2 * H1 + H2 + H2 + 1


def forward(p, F, H1, H2, X):
    w = unpack(p, F, H1, H2)
    z = (np.asarray(X, dtype=np.float64) - w["mean"]) * w["istd"]
    a1 = z @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    yhat = h2 @ w["W3"] + w["b3"][0]
    return yhat, (z, a1, h1, a2, h2)


def loss(p, F, H1, H2, X, y):
    yhat, _ = forward(p, F, H1, H2, X)
    return float(np.mean((yhat - np.asarray(y, dtype=np.float64)) ** 2))


def loss_grad(p, F, H1, H2, X, y):
    """Loss and its gradient by the chain rule (zero for mean, inv_std)."""
    w = unpack(p, F, H1, H2)
    yhat, (z, a1, h1, a2, h2) = forward(p, F, H1, H2, X)
    N = z.shape[0]
    r = yhat - np.asarray(y, dtype=np.float64)
    g = 2.0 * r / N                                # dL/dyhat
    dW3 = h2.T @ g
    db3 = np.array([g.sum()])
    g2 = np.outer(g, w["W3"]) * (a2 > 0)           # dL/da2
    dW2 = g2.T @ h1
    db2 = g2.sum(axis=0)
    g1 = (g2 @ w["W2"]) * (a1 > 0)                 # dL/da1
    dW1 = g1.T @ z
    db1 = g1.sum(axis=0)
    grad = np.concatenate([np.zeros(2 * F), dW1.ravel(), db1, dW2.ravel(), db2, dW3, db3])
    return float(np.mean(r ** 2)), grad
