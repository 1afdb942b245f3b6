"""The GELU approximations the perceptron kernels evaluate, for the tests.

The kernels replace x Phi(x) by max(x, 0) - h(min(|x|, 4)) with h fitted to
s Phi(-s): for training a degree-7 polynomial in s evaluated in FP32, for
inference a degree-7 polynomial in u = s/2 - 1 evaluated in packed FP16.
The coefficients are read from the kernel source so that the tests bound
the approximations that actually run. This is a description of the
kernels' arithmetic, not part of the oracle: the oracle's GELU is x Phi(x)
through the error function.
"""
import os
import re

import numpy as np

_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1902_02508_amd", "csrc",
                    "k_mlp.hip")


def coefficients():
    """c_1..c_7 of h(s) = sum_k c_k s^k (the source holds them in Horner order)."""
    text = open(_SRC).read()
    body = text[text.index("float gelu_h(float s)"):]
    body = body[:body.index("return")]
    nums = [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    if len(nums) != 7:
        raise ValueError(f"unexpected GELU polynomial in {_SRC}: {nums}")
    return nums[::-1]


def gelu(x):
    c = coefficients()
    x = np.asarray(x, dtype=np.float64)
    s = np.minimum(np.abs(x), 4.0)
    return np.maximum(x, 0.0) - sum(ck * s ** (k + 1) for k, ck in enumerate(c))


def gelu_grad(x):
    c = coefficients()
    x = np.asarray(x, dtype=np.float64)
    s = np.minimum(np.abs(x), 4.0)
    dh = np.where(np.abs(x) < 4.0, sum((k + 1) * ck * s ** k for k, ck in enumerate(c)), 0.0)
    return np.where(x >= 0.0, 1.0 - dh, dh)


def forward(unpack, theta, xs):
    """The network of the oracle with this GELU in FP64 (no roundings)."""
    p = unpack(theta)
    h = np.asarray(xs, dtype=np.float64)
    for l in range(4):
        z = h @ p[2 * l].T + p[2 * l + 1]
        h = gelu(z) if l < 3 else z
    return h


# ---- inference: FP16 polynomial in u = s/2 - 1

def coefficients16():
    """e_0..e_7 of h(s) = sum_k e_k u^k, u = s/2 - 1 (Horner order in the source)."""
    text = open(_SRC).read()
    body = text[text.index("gh2 gelu16_h(gh2 u)"):]
    body = body[:body.index("return")]
    nums = [float(v) for v in re.findall(r"(-?\d+\.\d+(?:e-?\d+)?)f", body)]
    if len(nums) != 8:
        raise ValueError(f"unexpected FP16 GELU polynomial in {_SRC}: {nums}")
    return nums[::-1]


def gelu16(x):
    """The inference GELU in exact arithmetic (FP64)."""
    e = coefficients16()
    x = np.asarray(x, dtype=np.float64)
    u = np.minimum(np.abs(x), 4.0) / 2.0 - 1.0
    return np.maximum(x, 0.0) - sum(ek * u ** k for k, ek in enumerate(e))


def _f16(a):
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def gelu16_rounded(z):
    """The inference GELU as the kernel rounds it: the FP32 input rounded
    to FP16, each step of the Horner recurrence a fused FP16 multiply-add
    (exact in FP64, then rounded once), the result rounded to FP16."""
    e = coefficients16()
    x = _f16(z)
    u = _f16(np.minimum(np.abs(x), 4.0) * 0.5 - 1.0)
    h = np.full_like(u, e[-1])
    for ek in e[-2::-1]:
        h = _f16(h * u + ek)
    return _f16(np.maximum(x, 0.0) - h)


def forward16(unpack, theta, xs):
    """The oracle's network with the inference GELU in FP64 (no roundings)."""
    p = unpack(theta)
    h = np.asarray(xs, dtype=np.float64)
    for l in range(4):
        z = h @ p[2 * l].T + p[2 * l + 1]
        h = gelu16(z) if l < 3 else z
    return h


def forward16_rounded(unpack, theta, xs):
    """The network with the inference kernel's roundings: FP16 weights,
    inputs and activations, FP32 biases, the rounded FP16 GELU (the
    products accumulate in FP64 here, in FP32 on the matrix cores)."""
    p = unpack(theta)
    h = _f16(xs)
    for l in range(4):
        z = h @ _f16(p[2 * l]).T + np.asarray(p[2 * l + 1], dtype=np.float32).astype(np.float64)
        h = gelu16_rounded(z) if l < 3 else z
    return h
