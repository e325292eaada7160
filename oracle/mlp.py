"""FP64 reference of the learned-T0 perceptron (test infrastructure only).

The paper's QPE optimiser picks the clock time T0 from the condition number
(Sec. 3.2, Fig. 4b: the best T0 falls with kappa); the predictor here maps the
spectrum features [log lambda_min, log lambda_max, log kappa, n_c, n_s] of an
instance to log(T0 lambda_max / 2 pi) through a 5 -> 64 -> 64 -> 1 network with
exact GELU activations, x Phi(x), Phi the standard normal CDF.

Everything is plain numpy in float64: the forward pass, the gradient of the
mean squared error written out layer by layer by the chain rule, and the Adam
update (Kingma and Ba, 2015, Algorithm 1).  Parameter vectors use the layout
W1[64][5] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
"""
import math

import numpy as np
from scipy.special import erf

N_IN, N_HID = 5, 64
N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_HID + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    W1 = p[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = p[o:o + N_HID]; o += N_HID
    W2 = p[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = p[o:o + N_HID]; o += N_HID
    W3 = p[o:o + N_HID]; o += N_HID
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def init_params(seed):
    """Glorot-uniform weights, zero biases, from numpy's PCG64 with `seed`."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((N_HID, N_IN), (N_HID, N_HID), (1, N_HID)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    return h2 @ W3 + b3


def loss_and_grad(p, X, t):
    """L = mean_i (net(X_i) - t_i)^2 and dL/dp (same layout as p)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ W3 + b3
    r = y - t
    L = float(np.mean(r * r))
    dy = 2.0 * r / B                      # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * gelu_prime(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_prime(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return L, g


def adam_step(p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (p, m, v).  step is 1-based."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
