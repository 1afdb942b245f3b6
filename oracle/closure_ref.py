"""FP64 reference (the oracle) for the learned closure of the exact stress.

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU baseline, never by the library.

The paper computes the exact stress from DNS data (Sec. 2.1) and names
machine learning as one way to turn such data into a model of the stress
(Sec. 2.1, last paragraph; Sec. 5). The closure here is such a
model: a multilayer perceptron that maps, at every grid point, the nine
components of the filtered velocity gradient and the distance to the
nearest wall to the six components of tau_ij. Nothing of its form is taken
from the paper; the definitions below are the reference the GPU kernels are
checked against.

* Features: d ubar_i / d x_k for i, k = 1..3 (row-major in (i, k)) and
  1 - |y|. x and z derivatives are spectral (the DFT multiplied by i k, the
  Nyquist mode of an even length set to zero); the y derivative is the
  three-point Lagrange derivative on the non-uniform nodes, and at a wall it
  uses the mirror node of the extension of eq. (7): the neighbour across the
  wall carries s f(y_1) at the same distance, s being the field's parity.
* Network: h_l = GELU(W_l h_{l-1} + b_l) for the hidden layers, a linear
  output layer. GELU(x) = x Phi(x) with Phi the standard normal CDF,
  evaluated through the error function: Phi(x) = (1 + erf(x / sqrt 2)) / 2;
  its derivative is Phi(x) + x phi(x), phi the normal density. Inputs and
  targets are standardised with training-set means and standard
  deviations.
* Physics term: the closure adds the gradient model, the leading term of
  the small-width expansion of the stress of a filter with second moments
  sigma_k^2 (cf. the invertible-filter discussion of Sec. 2.1),
  G_ij = sum_k c_k (d ubar_i / d x_k) (d ubar_j / d x_k), c_k = sigma_k^2 =
  Delta_k^2 / 12. The prediction is tau = G + mu + sd * N((x - m) / s), N
  the network, (m, s) and (mu, sd) the feature and stress moments; the
  network learns the standardised remainder (tau - G - mu) / sd. With
  c = 0 it is the plain network.
* Loss: mean over the batch and the six outputs of the squared error.
* Adam (Kingma & Ba 2015) with bias correction, no weight decay.
* Minibatch sampler: SplitMix64 (Steele, Lea & Flood 2014), output n of a
  stream with seed k is mix(k + (n + 1) * 0x9E3779B97F4A7C15); a draw maps
  to an index by ((r >> 32) * count) >> 32.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np
from scipy.special import erf

PARITY = (1, -1, 1)
LAYERS = (10, 64, 64, 64, 6)
_M64 = (1 << 64) - 1


# ------------------------------------------------------------------ features

def spectral_derivative(f: np.ndarray, length: float, axis: int) -> np.ndarray:
    n = f.shape[axis]
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=length / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def dy_matrix(y: np.ndarray, parity: int) -> np.ndarray:
    """Three-point Lagrange derivative on the nodes y, walls through the mirror node."""
    ny = len(y)
    D = np.zeros((ny, ny))
    for j in range(1, ny - 1):
        h1 = y[j] - y[j - 1]
        h2 = y[j + 1] - y[j]
        D[j, j - 1] = -h2 / (h1 * (h1 + h2))
        D[j, j] = (h2 - h1) / (h1 * h2)
        D[j, j + 1] = h1 / (h2 * (h1 + h2))
    # wall rows: neighbours at -h (value parity * f_1) and +h (value f_1)
    h = y[1] - y[0]
    D[0, 1] = (1.0 - parity) / (2.0 * h)
    h = y[-1] - y[-2]
    D[-1, -2] = -(1.0 - parity) / (2.0 * h)
    return D


def features(ubar: np.ndarray, y: np.ndarray, lx: float, lz: float) -> np.ndarray:
    """[10, nx, ny, nz]: grad(ubar) in (i, k) row-major order, then 1 - |y|."""
    ubar = np.asarray(ubar, dtype=np.float64)
    nx, ny, nz = ubar.shape[1:]
    out = np.empty((10, nx, ny, nz))
    for i in range(3):
        out[3 * i + 0] = spectral_derivative(ubar[i], lx, 0)
        out[3 * i + 1] = np.matmul(dy_matrix(y, PARITY[i])[None], ubar[i])
        out[3 * i + 2] = spectral_derivative(ubar[i], lz, 2)
    out[9] = (1.0 - np.abs(y))[None, :, None] * np.ones((nx, 1, nz))
    return out


# ------------------------------------------------------------ physics term

PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def gradient_model(feat: np.ndarray, coef) -> np.ndarray:
    """G_ij = sum_k coef[k] g_ik g_jk with g_ik = feat[3 i + k], over the
    leading axis of feat [10, ...]; returns [6, ...] in the order 11, 12,
    13, 22, 23, 33."""
    feat = np.asarray(feat, dtype=np.float64)
    out = np.zeros((6,) + feat.shape[1:])
    for q, (i, j) in enumerate(PAIRS):
        for k in range(3):
            out[q] += coef[k] * feat[3 * i + k] * feat[3 * j + k]
    return out


def widths_coef(delta_x: float, delta_y: float, delta_z: float):
    """c_k = Delta_k^2 / 12, the second moment of the filter in direction k."""
    return (delta_x ** 2 / 12.0, delta_y ** 2 / 12.0, delta_z ** 2 / 12.0)


def predict(theta, feat: np.ndarray, norms: np.ndarray, coef=(0.0, 0.0, 0.0)) -> np.ndarray:
    """The closure's stress [6, ...] from features [10, ...]: G + mu + sd N(x')."""
    feat = np.asarray(feat, dtype=np.float64)
    shape = feat.shape[1:]
    x = (feat.reshape(10, -1).T - norms[:10]) / norms[10:20]
    y = forward(theta, x) * norms[26:32] + norms[20:26]
    return y.T.reshape((6,) + shape) + gradient_model(feat, coef)


def standard_targets(tau: np.ndarray, feat: np.ndarray, norms: np.ndarray, coef=(0.0, 0.0, 0.0)) -> np.ndarray:
    """[N, 6] training targets (tau - G - mu) / sd of fields tau [6, ...]."""
    r = np.asarray(tau, dtype=np.float64) - gradient_model(feat, coef)
    return (r.reshape(6, -1).T - norms[20:26]) / norms[26:32]


# --------------------------------------------------------------------- MLP

def gelu(x):
    """x Phi(x), Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx x Phi(x) = Phi(x) + x phi(x), phi(x) = exp(-x^2 / 2) / sqrt(2 pi)."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def param_shapes(layers: Sequence[int] = LAYERS) -> List[Tuple[int, ...]]:
    shapes = []
    for a, b in zip(layers[:-1], layers[1:]):
        shapes += [(b, a), (b,)]
    return shapes


def n_params(layers: Sequence[int] = LAYERS) -> int:
    return sum(int(np.prod(s)) for s in param_shapes(layers))


def unpack(theta: np.ndarray, layers: Sequence[int] = LAYERS):
    out, o = [], 0
    for s in param_shapes(layers):
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def init_params(seed: int, layers: Sequence[int] = LAYERS) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias, PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for a, b in zip(layers[:-1], layers[1:]):
        lim = 1.0 / math.sqrt(a)
        parts.append(rng.uniform(-lim, lim, size=(b, a)).ravel())
        parts.append(rng.uniform(-lim, lim, size=(b,)))
    return np.concatenate(parts)


def forward(theta: np.ndarray, x: np.ndarray, layers: Sequence[int] = LAYERS, keep=False):
    """x: [batch, in]; returns the output [batch, out] (and the cache)."""
    p = unpack(theta, layers)
    h = np.asarray(x, dtype=np.float64)
    cache = [h]
    L = len(layers) - 1
    for l in range(L):
        W, b = p[2 * l], p[2 * l + 1]
        z = h @ W.T + b
        if l < L - 1:
            cache.append(z)
            h = gelu(z)
            cache.append(h)
        else:
            h = z
    return (h, cache) if keep else h


def loss_and_grad(theta: np.ndarray, x: np.ndarray, t: np.ndarray, layers: Sequence[int] = LAYERS):
    """Mean squared error and its gradient by reverse-mode differentiation."""
    p = unpack(theta, layers)
    y, cache = forward(theta, x, layers, keep=True)
    B, nout = y.shape
    loss = float(np.mean((y - t) ** 2))
    d = 2.0 * (y - t) / (B * nout)
    grads = [None] * len(p)
    L = len(layers) - 1
    for l in reversed(range(L)):
        W = p[2 * l]
        h_in = cache[0] if l == 0 else cache[2 * l]
        grads[2 * l] = d.T @ h_in
        grads[2 * l + 1] = d.sum(axis=0)
        if l > 0:
            z_prev = cache[2 * l - 1]
            d = (d @ W) * gelu_grad(z_prev)
    return loss, np.concatenate([g.ravel() for g in grads])


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ sampler

def splitmix64(seed: int, n: np.ndarray) -> np.ndarray:
    """Outputs n (uint64 array) of the SplitMix64 stream started at seed."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + (np.asarray(n, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sample_indices(seed: int, step: int, batch: int, count: int) -> np.ndarray:
    """Indices of minibatch `step` (from 0): draws step*batch .. step*batch+batch-1."""
    r = splitmix64(seed, np.arange(step * batch, (step + 1) * batch, dtype=np.uint64))
    return ((r >> np.uint64(32)) * np.uint64(count)) >> np.uint64(32)


# ------------------------------------------------------------ standardising

def moments(a: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Per-channel mean and standard deviation over all points of [C, ...]."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    mu = a.mean(axis=1)
    sd = np.sqrt(np.mean((a - mu[:, None]) ** 2, axis=1))
    return mu, sd


def train(theta0, xs, ts, steps, batch, seed, lr=1e-3, layers: Sequence[int] = LAYERS):
    """Reference training loop on standardised samples xs [N, in], ts [N, out]."""
    theta = theta0.copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for s in range(steps):
        idx = sample_indices(seed, s, batch, len(xs)).astype(np.int64)
        loss, g = loss_and_grad(theta, xs[idx], ts[idx], layers)
        theta, m, v = adam_step(theta, g, m, v, s + 1, lr)
        losses.append(loss)
    return theta, m, v, np.array(losses)
