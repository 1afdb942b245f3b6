"""FP64 reference (the oracle) for the error measures of Sec. 4.

TEST INFRASTRUCTURE ONLY. Only the test suite may import this module; the
library never does. It shares no code with the HIP path.

The paper compares an LES velocity u^LES with the DNS velocity u^DNS, each
scaled by its own friction velocity u_tau (the LES velocity being the
explicitly filtered one passed through the inverse filter):

* eq. (13), instantaneous field: the volume L2 norm of
  u1^LES/u_tau^LES - u1^DNS/u_tau^DNS over the volume L2 norm of
  u1^DNS/u_tau^DNS;
* eq. (14), mean profile: the same ratio for the profiles <u1>(y), <.> the
  average over the homogeneous directions x and z, integrated in the
  wall-normal coordinate from the wall to the channel centre (0 .. delta);
* eq. (15), turbulence intensities: the same for the rms profiles
  u_i,rms(y) = sqrt(<u_i^2> - <u_i>^2) of each component.

Readings (the paper names the integrals, not their quadrature): the volume
integral is uniform in the periodic x and z and uses the bounded trapezoid
rule on the y nodes; the profile integrals take the nodes from the lower
wall (y = -1) to the centreline (nodes with y <= 0) with the bounded
trapezoid rule on those nodes; the rms is the population rms over x and z.
"""
from __future__ import annotations

import math

import numpy as np


def trapezoid_weights(y: np.ndarray) -> np.ndarray:
    """w_j with sum_j w_j f(y_j) the trapezoid rule over [y_0, y_last]."""
    y = np.asarray(y, dtype=np.float64)
    w = np.zeros(len(y))
    for j in range(len(y) - 1):
        h = y[j + 1] - y[j]
        w[j] += 0.5 * h
        w[j + 1] += 0.5 * h
    return w


def volume_error(les1: np.ndarray, dns1: np.ndarray, utau_les: float, utau_dns: float, y: np.ndarray) -> float:
    """Eq. (13) for fields [nx, ny, nz]."""
    a = np.asarray(les1, np.float64) / utau_les
    b = np.asarray(dns1, np.float64) / utau_dns
    w = trapezoid_weights(y)
    num = sum(w[j] * np.sum((a[:, j, :] - b[:, j, :]) ** 2) for j in range(len(y)))
    den = sum(w[j] * np.sum(b[:, j, :] ** 2) for j in range(len(y)))
    return math.sqrt(num / den)


def lower_half(y: np.ndarray) -> np.ndarray:
    """Indices of the nodes from the lower wall to the centreline."""
    return np.nonzero(np.asarray(y) <= 0.0)[0]


def half_profile_error(pa: np.ndarray, pb: np.ndarray, y: np.ndarray) -> float:
    """[int_0^delta (pa - pb)^2]^(1/2) / [int_0^delta pb^2]^(1/2), trapezoid rule."""
    k = lower_half(y)
    w = trapezoid_weights(np.asarray(y)[k])
    d = np.asarray(pa, np.float64)[k] - np.asarray(pb, np.float64)[k]
    return math.sqrt(np.sum(w * d * d) / np.sum(w * np.asarray(pb, np.float64)[k] ** 2))


def plane_mean(f: np.ndarray) -> np.ndarray:
    return np.asarray(f, np.float64).mean(axis=(0, 2))


def plane_rms(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f, np.float64)
    m = plane_mean(f)
    return np.sqrt(np.maximum((f ** 2).mean(axis=(0, 2)) - m ** 2, 0.0))


def errors(les: np.ndarray, dns: np.ndarray, utau_les: float, utau_dns: float, y: np.ndarray) -> np.ndarray:
    """[eq. (13), eq. (14), eq. (15) for u1, u2, u3] for velocities [3][nx][ny][nz]."""
    out = [volume_error(les[0], dns[0], utau_les, utau_dns, y),
           half_profile_error(plane_mean(les[0]) / utau_les, plane_mean(dns[0]) / utau_dns, y)]
    for i in range(3):
        out.append(half_profile_error(plane_rms(les[i]) / utau_les, plane_rms(dns[i]) / utau_dns, y))
    return np.array(out)
