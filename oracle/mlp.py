"""Float64 reference of the (p, levels) selector network.

Test infrastructure (see ``oracle/__init__``).  Not from the paper: the paper
studies how the FMM error depends on the particle count, the number of levels
and the expansion order (Sections 4-5); this network predicts that error from
such parameters.  Definitions written out plainly:

features (10), for particles (x, y, Gamma), core size sigma, order p, levels L
and root side S:
    f0 = p
    f1 = L
    f2 = log2 N
    f3 = log2 N - 2 L                      (log2 of the mean particles per leaf)
    f4 = log2(max(w_L, a) / sigma)         (the distance below which every pair is
                                            summed with the regularised kernel, over
                                            the core size: the leaf side w_L = S / 2^L,
                                            or the near radius a of the distance
                                            cut-off, a = min(radius, 4 w_L), if larger;
                                            radius < 0 stands for 6 sigma)
    f5 = log2(sigma / h),  h = S / sqrt(N)
    f6 = mean(Gamma) / rms(Gamma)
    f7 = log10(sum |Gamma| / max |Gamma|)
    f8 = std(x) / S
    f9 = std(y) / S
network: y = W3 . g(W2^T g(W1^T x + b1) + b2) + b3 with 10 -> 64 -> 64 -> 1 and the
tanh form of GELU, g(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)));
loss: mean squared error; optimiser: Adam (Kingma & Ba 2015) with bias
correction.

Parameter vector layout (4929 values): W1[10][64] (row = input), b1[64],
W2[64][64] (row = input), b2[64], W3[64], b3.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 10, 64
SIZES = {"W1": N_IN * N_HID, "b1": N_HID, "W2": N_HID * N_HID, "b2": N_HID, "W3": N_HID, "b3": 1}
N_PARAMS = sum(SIZES.values())
_C = math.sqrt(2.0 / math.pi)


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    out, o = {}, 0
    for k, n in SIZES.items():
        out[k] = theta[o:o + n]
        o += n
    out["W1"] = out["W1"].reshape(N_IN, N_HID)
    out["W2"] = out["W2"].reshape(N_HID, N_HID)
    return out


def pack(d):
    return np.concatenate([np.asarray(d[k], np.float64).ravel() for k in SIZES])


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(_C * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    t = np.tanh(_C * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _C * (1.0 + 3 * 0.044715 * z * z)


def forward(theta, X):
    P = unpack(theta)
    z1 = X @ P["W1"] + P["b1"]
    a1 = gelu(z1)
    z2 = a1 @ P["W2"] + P["b2"]
    a2 = gelu(z2)
    y = a2 @ P["W3"] + P["b3"][0]
    return y, (z1, a1, z2, a2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    return float(np.mean((y - T) ** 2))


def gradient(theta, X, T):
    """d loss / d theta by the chain rule."""
    P = unpack(theta)
    y, (z1, a1, z2, a2) = forward(theta, X)
    B = X.shape[0]
    dy = 2.0 * (y - T) / B
    g = {}
    g["W3"] = a2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, P["W3"]) * gelu_grad(z2)
    g["W2"] = a1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ P["W2"].T) * gelu_grad(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return pack(g)


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation (weights N(0, 2/fan_in), zero biases)."""
    rng = np.random.default_rng(seed)
    d = {"W1": rng.normal(0, math.sqrt(2.0 / N_IN), (N_IN, N_HID)), "b1": np.zeros(N_HID),
         "W2": rng.normal(0, math.sqrt(2.0 / N_HID), (N_HID, N_HID)), "b2": np.zeros(N_HID),
         "W3": rng.normal(0, math.sqrt(1.0 / N_HID), N_HID), "b3": np.zeros(1)}
    return pack(d)


def near_distance(side, levels, sigma, radius=0.0):
    """max(w_L, a): w_L the leaf side, a the near radius clamped to 4 w_L
    (radius < 0: 6 sigma, the distance beyond which the two kernels agree in
    float32; 0: the paper's split, no cut-off)."""
    w = side / 2 ** levels
    if radius == 0.0:
        return w
    a = 6.0 * sigma if radius < 0 else radius
    return max(w, min(a, 4.0 * w))


def features(x, y, gamma, sigma, p, levels, side, radius=0.0):
    """The 10 selector features (see module docstring)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64); g = np.asarray(gamma, np.float64)
    n = len(x)
    h = side / math.sqrt(n)
    rms = math.sqrt(float(np.mean(g * g)))
    amax = float(np.max(np.abs(g)))
    return np.array([
        float(p), float(levels), math.log2(n), math.log2(n) - 2 * levels,
        math.log2(near_distance(side, levels, sigma, radius) / sigma), math.log2(sigma / h),
        float(np.mean(g)) / rms if rms > 0 else 0.0,
        math.log10(float(np.sum(np.abs(g))) / amax) if amax > 0 else 0.0,
        float(np.std(x)) / side, float(np.std(y)) / side,
    ])
