"""FP64 multilayer perceptron: the reference for the surrogate's HIP kernels.

TEST INFRASTRUCTURE (see the package docstring).

Network: x in R^6 -> 128 -> 128 -> 128 -> 1.  Each hidden layer is
z = W a + b followed by GELU(z) = z Phi(z) = z/2 (1 + erf(z / sqrt 2)) (the
exact, erf form); the output layer is linear.  Loss: mean squared error over
the batch.  Parameters are one flat vector, in this order: W1 (128 x 6, one
row per output unit), b1 (128), W2 (128 x 128), b2, W3 (128 x 128), b3,
W4 (1 x 128), b4 (1): 34,049 values.  Adam (Kingma & Ba, ICLR 2015, Alg. 1)
with bias-corrected moments.

Everything is written out with numpy matrix products in float64; the
backward pass is the chain rule layer by layer, nothing fused.
"""
import math

import numpy as np
from scipy.special import erf

SIZES = (6, 128, 128, 128, 1)


def n_params(sizes=SIZES):
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    """Views [(W1, b1), ..., (W4, b4)] into the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    out, o = [], 0
    for i in range(len(sizes) - 1):
        n, k = sizes[i + 1], sizes[i]
        W = theta[o:o + n * k].reshape(n, k)
        o += n * k
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    assert o == theta.size
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    """Returns (y [B], cache) for inputs X [B, 6]."""
    layers = unpack(theta)
    a = np.asarray(X, dtype=np.float64)
    zs, acts = [], [a]
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        zs.append(z)
        a = gelu(z) if li < len(layers) - 1 else z
        acts.append(a)
    return a[:, 0], {"zs": zs, "acts": acts}


def loss(theta, X, t):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(theta, X, t):
    """Gradient of the mean squared error with respect to the flat parameters;
    returns (loss, grad)."""
    layers = unpack(theta)
    y, cache = forward(theta, X)
    t = np.asarray(t, dtype=np.float64)
    B = y.size
    delta = (2.0 / B) * (y - t)[:, None]  # dL/dz of the output layer
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_prev = cache["acts"][li]
        grads.append((delta.T @ a_prev, delta.sum(axis=0)))
        if li > 0:
            delta = (delta @ W) * gelu_grad(cache["zs"][li - 1])
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return float(np.mean((y - t) ** 2)), flat


def adam_step(theta, grad, m, v, k, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number k >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** k)
    vhat = v / (1.0 - beta2 ** k)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
