"""FP64 reference (the oracle) for the stress on an LES grid and the
commutation error of the discretization operator.

TEST INFRASTRUCTURE ONLY. Only the test suite may import this module; the
library never does. It shares no code with the HIP path.

Sec. 2 (the discrete filtered equations): the LES solves for the
discretized filtered velocity tilde(bar u); its stress is
    T_ij = I(F(u_i u_j)) - I(F(u_i)) I(F(u_j)),
with I the discretization operator. Sec. 4 takes I to be second-order
linear interpolation from the DNS grid to the LES grid (LES2, LES4: grids
coarser by 2 and 4), and notes that on a stretched mesh it does not commute
with second-order finite differences.

Readings:
* I is separable linear interpolation: periodic in x and z (LES nodes
  k L / n_les, DNS nodes i L / n), in y between the bracketing DNS nodes of
  each LES node (the LES y nodes lie in [-1, 1], walls included);
* the commutation error of a field g is
    || d_y^LES(I g) - I(d_y^DNS g) || / || I(d_y^DNS g) ||
  over the LES volume (trapezoid weights in y), with d_y the second-order
  three-point first derivative on each mesh (central on the interior
  nodes, one-sided at the walls).
"""
from __future__ import annotations

import math

import numpy as np


def periodic_weights(n_les: int, n: int):
    """For LES node k at k/n_les of the period: the DNS node i below it and
    the weight w of node i+1 (mod n): I g = (1 - w) g_i + w g_{i+1}."""
    i0 = np.zeros(n_les, dtype=np.int64)
    w = np.zeros(n_les)
    for k in range(n_les):
        pos = k * n / n_les          # position in DNS node units
        i = int(math.floor(pos + 1e-12))
        i0[k] = i % n
        w[k] = pos - i if pos - i > 1e-12 else 0.0
    return i0, w


def wall_weights(y_les: np.ndarray, y: np.ndarray):
    """For each LES y node: the DNS node j below it (j <= ny-2) and the
    weight of node j+1."""
    y_les = np.asarray(y_les, np.float64)
    y = np.asarray(y, np.float64)
    j0 = np.zeros(len(y_les), dtype=np.int64)
    w = np.zeros(len(y_les))
    for k, t in enumerate(y_les):
        j = 0
        while j < len(y) - 2 and y[j + 1] <= t:
            j += 1
        j0[k] = j
        w[k] = (t - y[j]) / (y[j + 1] - y[j])
    return j0, w


class Interp:
    """The discretization operator between a DNS and an LES grid."""

    def __init__(self, nx, ny, nz, y, nx_les, nz_les, y_les):
        self.shape = (nx, ny, nz)
        self.les_shape = (nx_les, len(y_les), nz_les)
        self.y = np.asarray(y, np.float64)
        self.y_les = np.asarray(y_les, np.float64)
        self.ix, self.wx = periodic_weights(nx_les, nx)
        self.iy, self.wy = wall_weights(y_les, y)
        self.iz, self.wz = periodic_weights(nz_les, nz)

    def __call__(self, g: np.ndarray) -> np.ndarray:
        """I g for a DNS field [nx, ny, nz] (one direction at a time)."""
        g = np.asarray(g, np.float64)
        nx, ny, nz = self.shape
        gx = (1 - self.wx)[:, None, None] * g[self.ix] + self.wx[:, None, None] * g[(self.ix + 1) % nx]
        gy = (1 - self.wy)[None, :, None] * gx[:, self.iy] + self.wy[None, :, None] * gx[:, self.iy + 1]
        return (1 - self.wz)[None, None, :] * gy[:, :, self.iz] + self.wz[None, None, :] * gy[:, :, (self.iz + 1) % nz]


PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def les_stress(ubar: np.ndarray, fuu: np.ndarray, I: Interp):
    """(tilde(bar u) [3], T [6]) on the LES grid from the DNS-grid filtered
    velocity ubar [3] and filtered products fuu [6] = F(u_i u_j) in the
    order 11, 12, 13, 22, 23, 33: T_ij = I(F(u_i u_j)) - I(ubar_i) I(ubar_j)."""
    ul = np.stack([I(ubar[i]) for i in range(3)])
    T = np.stack([I(fuu[k]) - ul[i] * ul[j] for k, (i, j) in enumerate(PAIRS)])
    return ul, T


def d_dy(g: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Second-order first derivative in y of [.., ny, ..] fields (axis 1):
    three-point central on the interior, one-sided three-point at the walls."""
    g = np.asarray(g, np.float64)
    y = np.asarray(y, np.float64)
    ny = len(y)
    out = np.empty_like(g)
    for j in range(ny):
        if j == 0:
            h1, h2 = y[1] - y[0], y[2] - y[1]
            c = (-(2 * h1 + h2) / (h1 * (h1 + h2)), (h1 + h2) / (h1 * h2), -h1 / (h2 * (h1 + h2)))
            idx = (0, 1, 2)
        elif j == ny - 1:
            h1, h2 = y[j] - y[j - 1], y[j - 1] - y[j - 2]
            c = ((2 * h1 + h2) / (h1 * (h1 + h2)), -(h1 + h2) / (h1 * h2), h1 / (h2 * (h1 + h2)))
            idx = (j, j - 1, j - 2)
        else:
            hm, hp = y[j] - y[j - 1], y[j + 1] - y[j]
            c = (-hp / (hm * (hm + hp)), (hp - hm) / (hm * hp), hm / (hp * (hm + hp)))
            idx = (j - 1, j, j + 1)
        out[:, j] = sum(ck * g[:, k] for ck, k in zip(c, idx))
    return out


def trapezoid_weights(y: np.ndarray) -> np.ndarray:
    y = np.asarray(y, np.float64)
    w = np.zeros(len(y))
    for j in range(len(y) - 1):
        w[j] += 0.5 * (y[j + 1] - y[j])
        w[j + 1] += 0.5 * (y[j + 1] - y[j])
    return w


def commutation_error(g: np.ndarray, I: Interp) -> float:
    a = d_dy(I(g), I.y_les)
    b = I(d_dy(g, I.y))
    w = trapezoid_weights(I.y_les)[None, :, None]
    return math.sqrt(np.sum(w * (a - b) ** 2) / np.sum(w * b * b))
