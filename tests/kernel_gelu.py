"""The GELU approximation the perceptron kernels evaluate, for the tests.

The kernels replace x Phi(x) by max(x, 0) - h(min(|x|, 4)), h a degree-7
polynomial fitted to s Phi(-s); its coefficients are read from the kernel
source so that the tests bound the approximation that actually runs. This
is a description of the kernels' arithmetic, not part of the oracle: the
oracle's GELU is x Phi(x) through the error function.
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
