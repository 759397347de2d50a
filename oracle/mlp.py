"""FP64 multilayer perceptron for the tuning emulator (oracle).

Not part of the paper: the emulator maps FGPA parameters and redshift,
(a, b, c, z), to the statistics the plain tuning loop matches (mean flux and
the binned 1D power).  This module is the FP64 reference of the HIP
training and inference kernels:

* layers 4 -> 256 -> 256 -> 256 -> 33, GELU on the hidden layers with the exact
  form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 (Hendrycks & Gimpel 2016),
  linear output;
* row-vector convention: h = gelu(x W + b), W of shape [in, out];
* loss: mean squared error over the batch and the outputs;
* optimiser: Adam (Kingma & Ba 2014) with bias correction.

Pins: central finite differences of the loss for every parameter tensor, the
GELU against scipy's normal CDF, and the first Adam step (exactly lr times the
sign of the gradient for eps -> 0).
"""
import numpy as np
from scipy import special

SIZES = (4, 256, 256, 256, 33)


def gelu(x):
    # Phi(x) = erfc(-x / sqrt 2) / 2 keeps full precision for negative x
    return 0.5 * x * special.erfc(-x / np.sqrt(2.0))


def gelu_grad(x):
    return 0.5 * special.erfc(-x / np.sqrt(2.0)) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def init_params(seed=0, sizes=SIZES):
    """He-style normal initialisation (std sqrt(2/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        params.append(rng.normal(0.0, np.sqrt(2.0 / sizes[i]), (sizes[i], sizes[i + 1])))
        params.append(np.zeros(sizes[i + 1]))
    return params


def forward(params, x):
    """Returns (output, cache) for backward."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        z = h @ W + b
        cache.append((h, z))
        h = gelu(z) if l < nl - 1 else z
    return h, cache


def loss(params, x, t):
    y, _ = forward(params, x)
    return float(np.mean((y - t) ** 2))


def backward(params, x, t):
    """(loss, gradients in the order of params)."""
    y, cache = forward(params, x)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    dy = 2.0 * (y - t) / n
    grads = [None] * len(params)
    nl = len(params) // 2
    d = dy
    for l in range(nl - 1, -1, -1):
        h, z = cache[l]
        if l < nl - 1:
            d = d * gelu_grad(z)
        grads[2 * l] = h.T @ d
        grads[2 * l + 1] = d.sum(axis=0)
        d = d @ params[2 * l].T
    return float(np.mean((y - t) ** 2)), grads


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            p -= self.lr * mh / (np.sqrt(vh) + self.eps)
        return params
