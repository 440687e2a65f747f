"""FP64 reference of the learned-proposal network -- TEST INFRASTRUCTURE.

A multilayer perceptron 16 -> 64 -> 64 -> 2 with tanh hidden units, written
out in plain NumPy so that the GPU's hand-written FP32 forward, backward and
Adam kernels can be checked against it.  The backward pass is the chain rule
applied layer by layer (checked here against central finite differences).

Parameter layout (one flat vector, row-major matrices, the order the GPU
library uses):  W1 (64 x 16), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).

Inputs are standardised with per-feature mean and standard deviation
(x - mu) / sd; the loss is the mean over samples of the squared error summed
over the two outputs, against targets standardised the same way:
    L = (1/N) sum_n sum_o (y_no - (t_no - tmu_o)/tsd_o)^2.
Initialisation (Glorot and Bengio 2010, uniform): W ~ U(-a, a) with
a = sqrt(6 / (fan_in + fan_out)), drawn as a (2 U - 1) with U the SplitMix64
uniforms of the seed in parameter order; biases zero.
Adam (Kingma and Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

from .splitmix import uniform01

NIN, NH, NOUT = 16, 64, 2
SHAPES = [(NH, NIN), (NH,), (NH, NH), (NH,), (NOUT, NH), (NOUT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)  # 5378


def unpack(theta):
    out, off = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(np.asarray(theta[off:off + k], dtype=np.float64).reshape(s))
        off += k
    return out


def pack(parts) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def init(seed: int) -> np.ndarray:
    u = uniform01(seed, NPARAM)
    theta = np.zeros(NPARAM)
    off = 0
    for s in SHAPES:
        k = int(np.prod(s))
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            theta[off:off + k] = a * (2.0 * u[off:off + k] - 1.0)
        off += k
    return theta


def forward(theta, X, mu, sd):
    """Network outputs (standardised units) and the activations for backward."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Xn = (np.asarray(X, dtype=np.float64) - mu) / sd
    H1 = np.tanh(Xn @ W1.T + b1)
    H2 = np.tanh(H1 @ W2.T + b2)
    Y = H2 @ W3.T + b3
    return Y, (Xn, H1, H2)


def loss(theta, X, T, mu, sd, tmu, tsd) -> float:
    Y, _ = forward(theta, X, mu, sd)
    Tn = (np.asarray(T, dtype=np.float64) - tmu) / tsd
    return float(np.sum((Y - Tn) ** 2) / len(Y))


def grad(theta, X, T, mu, sd, tmu, tsd):
    """(loss, dL/dtheta) by back-propagation."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Y, (Xn, H1, H2) = forward(theta, X, mu, sd)
    Tn = (np.asarray(T, dtype=np.float64) - tmu) / tsd
    N = len(Y)
    dY = 2.0 * (Y - Tn) / N
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * (1.0 - H2 * H2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * (1.0 - H1 * H1)
    dW1 = dZ1.T @ Xn
    db1 = dZ1.sum(axis=0)
    L = float(np.sum((Y - Tn) ** 2) / N)
    return L, pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def predict(theta, X, mu, sd, tmu, tsd) -> np.ndarray:
    """Outputs in target units: y * tsd + tmu."""
    Y, _ = forward(theta, X, mu, sd)
    return Y * tsd + tmu
