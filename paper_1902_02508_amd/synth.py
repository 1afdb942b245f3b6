"""Seeded synthetic channel-flow inputs.

This module only manufactures inputs: the wall-normal grid, the five
channel configurations and divergence-free, no-slip velocity snapshots.
It holds none of the filtering arithmetic, so both the FP64 oracle and the
HIP path may import it.

Geometry follows the channel of the paper's numerical experiment
(Sec. 3): streamwise x and spanwise z are periodic and uniformly sampled,
the wall-normal direction y in [-1, 1] is bounded by two walls and
stretched towards them with a hyperbolic tangent. The paper's DNS fields
are not available; a random solenoidal field stands in for them:

    u = U(y) e_x + curl A,   A_c = e(y) sum_n |k_n|^-p cos(k_n . (x, z) + phi_{c,n})

with e(y) = (1 - y^2)^2, so u vanishes at both walls (no slip) and
div u = 0 holds analytically. Every velocity component is a short sum of
separable terms g(y) f(x, z); the factors are returned as well, which lets
a reference evaluate large volumes term by term.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Tuple

import numpy as np

__all__ = [
    "ChannelConfig", "CONFIGS", "config", "ygrid", "mean_profile",
    "snapshot_factors", "make_snapshot", "assemble", "assemble_on_device", "SEEDS",
]


@dataclasses.dataclass(frozen=True)
class ChannelConfig:
    """One channel workload: grid, box, filter widths and generator law."""
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    lz: float
    ykind: str            # "cgl", "tanh" or "uniform"
    stretch: float        # tanh stretching factor gamma (unused otherwise)
    delta_x: float        # filter widths (second moment of a top hat)
    delta_y: float
    delta_z: float
    kmax: int             # Fourier modes |n_x|, |n_z| <= kmax
    slope: float          # amplitude law |k|^-slope
    mean: str             # "quartic" (1 - y^4) or "reichardt"
    rms: float            # target sqrt(<u'.u'>/3); 0 keeps the raw amplitude

    @property
    def points(self) -> int:
        return self.nx * self.ny * self.nz


_PI = math.pi

CONFIGS: Dict[str, ChannelConfig] = {
    # tiny Chebyshev grid, seconds for a direct quadrature
    "tiny": ChannelConfig("tiny", 32, 33, 32, 2 * _PI, _PI, "cgl", 0.0,
                          2 * _PI / 16, 0.1, _PI / 16, 8, 11.0 / 6.0,
                          "quartic", 0.0),
    # DNS-like shape; widths are twice the spacing of a 48x33x48 LES grid
    "dns192": ChannelConfig("dns192", 192, 129, 192, 4 * _PI, 2 * _PI, "tanh", 2.0,
                            _PI / 6, 0.05, _PI / 12, 48, 5.0 / 3.0,
                            "reichardt", 0.1),
    # precision study; widths are eight grid spacings
    "dns512": ChannelConfig("dns512", 512, 257, 512, 2 * _PI, _PI, "tanh", 2.0,
                            _PI / 32, 0.05, _PI / 64, 128, 5.0 / 3.0,
                            "reichardt", 0.1),
    # production shape at the physical widths of the 192^2 training set
    "dns1024": ChannelConfig("dns1024", 1024, 385, 768, 8 * _PI, 3 * _PI, "tanh", 2.0,
                             _PI / 6, 0.05, _PI / 12, 256, 5.0 / 3.0,
                             "reichardt", 0.1),
}

# seeds per use; training and held-out sets never overlap
SEEDS = {
    "tiny": [0],
    "dns192": [0, 1, 2, 3],
    "dns512": [0],
    "train": list(range(1000, 1032)),
    "heldout": [2000, 2001, 2002, 2003],
    "dns1024": list(range(3000, 3008)),
}


def config(name: str, **over) -> ChannelConfig:
    """Named configuration, optionally with fields replaced."""
    return dataclasses.replace(CONFIGS[name], **over)


def ygrid(ny: int, kind: str = "tanh", stretch: float = 2.0) -> np.ndarray:
    """Wall-normal nodes, strictly increasing, y[0] = -1 and y[-1] = +1 exactly."""
    if ny < 3:
        raise ValueError("ny must be >= 3")
    j = np.arange(ny, dtype=np.float64)
    if kind == "cgl":
        y = -np.cos(np.pi * j / (ny - 1))
    elif kind == "tanh":
        xi = -1.0 + 2.0 * j / (ny - 1)
        y = np.tanh(stretch * xi) / np.tanh(stretch)
    elif kind == "uniform":
        y = -1.0 + 2.0 * j / (ny - 1)
    else:
        raise ValueError(f"unknown y grid {kind!r}")
    y[0], y[-1] = -1.0, 1.0
    if (ny - 1) % 2 == 0:
        y[(ny - 1) // 2] = 0.0
    return y


def mean_profile(y: np.ndarray, kind: str) -> np.ndarray:
    """Streamwise mean U(y) with U(0) = 1 and U(+-1) = 0."""
    if kind == "quartic":
        return 1.0 - y ** 4
    if kind == "reichardt":
        # Reichardt's composite law of the wall at Re_tau = 180, kappa = 0.41
        re_tau, kappa = 180.0, 0.41

        def uplus(yp):
            return (np.log1p(kappa * yp) / kappa
                    + 7.8 * (1.0 - np.exp(-yp / 11.0) - (yp / 11.0) * np.exp(-yp / 3.0)))
        yp = (1.0 - np.abs(y)) * re_tau
        return uplus(yp) / uplus(np.array(re_tau))
    raise ValueError(f"unknown mean profile {kind!r}")


def _plane_sums(cfg: ChannelConfig, coef: np.ndarray) -> np.ndarray:
    """Re sum_n coef[nx, nz] exp(i (kx x + kz z)) on the (x, z) grid, coef indexed from -K."""
    K = cfg.kmax
    n = np.arange(-K, K + 1)
    ex = np.exp(2j * np.pi * np.outer(np.arange(cfg.nx), n) / cfg.nx)   # [nx, 2K+1]
    ez = np.exp(2j * np.pi * np.outer(n, np.arange(cfg.nz)) / cfg.nz)   # [2K+1, nz]
    return np.real(ex @ coef @ ez)


def snapshot_factors(cfg: ChannelConfig, seed: int):
    """Separable form of one snapshot.

    Returns (y, terms) where terms[c] is a list of (g_y [ny], f_xz [nx, nz])
    pairs with u_c = sum_t g_t(y) f_t(x, z), all in FP64.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    y = ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    K = cfg.kmax
    n = np.arange(-K, K + 1)
    kx = 2.0 * np.pi * n[:, None] / cfg.lx * np.ones((1, 2 * K + 1))
    kz = 2.0 * np.pi * n[None, :] / cfg.lz * np.ones((2 * K + 1, 1))
    kk = np.sqrt(kx ** 2 + kz ** 2)
    amp = np.zeros_like(kk)
    nz_mask = kk > 0
    amp[nz_mask] = kk[nz_mask] ** (-cfg.slope)
    # one random phase per potential component and mode
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(3, 2 * K + 1, 2 * K + 1))
    c = amp[None] * np.exp(1j * phase)                     # A_c coefficients
    # phi_c = Re sum c e^{i theta};  d/dx phi_c = Re sum (i kx) c e^{i theta}
    phi = [_plane_sums(cfg, c[i]) for i in range(3)]
    dxphi = [_plane_sums(cfg, 1j * kx * c[i]) for i in range(3)]
    dzphi = [_plane_sums(cfg, 1j * kz * c[i]) for i in range(3)]
    e = (1.0 - y ** 2) ** 2
    de = -4.0 * y * (1.0 - y ** 2)
    # u' = curl A with A_c = e(y) phi_c(x, z)
    fl = [
        [(de, phi[2]), (-e, dzphi[1])],
        [(e, dzphi[0] - dxphi[2])],
        [(e, dxphi[1]), (-de, phi[0])],
    ]
    if cfg.rms > 0:
        ms = 0.0
        for terms in fl:
            for (ga, fa) in terms:
                for (gb, fb) in terms:
                    ms += np.mean(ga * gb) * np.mean(fa * fb)
        scale = cfg.rms / math.sqrt(ms / 3.0)
        fl = [[(g * scale, f) for (g, f) in terms] for terms in fl]
    U = mean_profile(y, cfg.mean)
    ones = np.ones((cfg.nx, cfg.nz))
    terms = [[(U, ones)] + fl[0], fl[1], fl[2]]
    return y, terms


def assemble(cfg: ChannelConfig, terms, dtype=np.float32, x_chunk: int = 64) -> np.ndarray:
    """Evaluate separable terms into a dense [3, nx, ny, nz] array (layout z fastest)."""
    u = np.empty((3, cfg.nx, cfg.ny, cfg.nz), dtype=dtype)
    for c in range(3):
        for x0 in range(0, cfg.nx, x_chunk):
            x1 = min(cfg.nx, x0 + x_chunk)
            acc = np.zeros((x1 - x0, cfg.ny, cfg.nz), dtype=np.float64)
            for (g, f) in terms[c]:
                acc += g[None, :, None] * f[x0:x1, None, :]
            u[c, x0:x1] = acc.astype(dtype)
    return u


def assemble_on_device(cfg: ChannelConfig, terms, device):
    """assemble() into a torch FP32 tensor on `device`: the same FP64 sums in
    the same order (one multiply and one add per term), rounded to FP32,
    so the values equal assemble()'s. For the large grids, whose host
    assembly takes seconds."""
    import torch
    u = torch.empty((3, cfg.nx, cfg.ny, cfg.nz), dtype=torch.float32, device=device)
    for c in range(3):
        gs = [torch.from_numpy(np.ascontiguousarray(g)).to(device) for g, _ in terms[c]]
        fs = [torch.from_numpy(np.ascontiguousarray(f)).to(device) for _, f in terms[c]]
        for x0 in range(0, cfg.nx, 64):
            x1 = min(cfg.nx, x0 + 64)
            acc = torch.zeros((x1 - x0, cfg.ny, cfg.nz), dtype=torch.float64, device=device)
            for g, f in zip(gs, fs):
                acc += g[None, :, None] * f[x0:x1, None, :]
            u[c, x0:x1] = acc.to(torch.float32)
    return u


def make_snapshot(cfg: ChannelConfig, seed: int, dtype=np.float32) -> Tuple[np.ndarray, np.ndarray]:
    """(y, u) with u[3, nx, ny, nz] of the given dtype."""
    y, terms = snapshot_factors(cfg, seed)
    return y, assemble(cfg, terms, dtype)
