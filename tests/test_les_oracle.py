"""Pins of the FP64 oracle of the LES-grid stress and the commutation error
(oracle.les_ref).

Each test checks the oracle against something other than itself: numpy's
linear interpolation, exactness on linear functions, injection when the LES
nodes are DNS nodes, the identity grid, the derivative of polynomials, and
the second-order convergence of the commutation error.
"""
import math

import numpy as np
import pytest

from oracle import filter_ref as R
from oracle import les_ref as L
from paper_1902_02508_amd import synth


def _grids(nx=16, ny=17, nz=12, ratio=2, kind="tanh", stretch=2.0):
    y = synth.ygrid(ny, kind, stretch)
    y_les = synth.ygrid((ny - 1) // ratio + 1, kind, stretch)
    return y, y_les, L.Interp(nx, ny, nz, y, nx // ratio, nz // ratio, y_les)


def test_y_interpolation_equals_numpy():
    y = synth.ygrid(21, "tanh", 2.0)
    y_les = np.linspace(-1, 1, 8)
    I = L.Interp(4, 21, 4, y, 4, 4, y_les)
    g = np.random.default_rng(0).standard_normal((4, 21, 4))
    out = I(g)
    for i in range(4):
        for k in range(4):
            assert np.max(np.abs(out[i, :, k] - np.interp(y_les, y, g[i, :, k]))) < 1e-14


def test_linear_functions_are_reproduced():
    """Separable linear interpolation is exact for a + b y (any LES y nodes)
    and, in x, for a field linear between the bracketing DNS nodes."""
    y = synth.ygrid(25, "tanh", 2.0)
    y_les = np.sort(np.concatenate([[-1.0, 1.0], np.random.default_rng(1).uniform(-1, 1, 7)]))
    I = L.Interp(10, 25, 6, y, 7, 5, y_les)
    g = np.broadcast_to((0.3 + 1.7 * y)[None, :, None], (10, 25, 6))
    assert np.max(np.abs(I(g) - (0.3 + 1.7 * y_les)[None, :, None])) < 1e-14


def test_coinciding_nodes_inject():
    y, y_les, I = _grids(ratio=2, kind="cgl")
    g = np.random.default_rng(2).standard_normal((16, 17, 12))
    assert np.max(np.abs(I(g) - g[::2, ::2, ::2])) < 1e-15


def test_identity_grid_gives_tau():
    """LES grid = DNS grid: T_ij is the DNS-grid stress (the LES1 case)."""
    cfg = synth.config("tiny", nx=16, nz=12, ny=17)
    ops = R.Operators.from_config(cfg)
    y, u = synth.make_snapshot(cfg, 1)
    u = u.astype(np.float64)
    ub, tau = R.sgs_stress(u, ops)
    fuu = np.stack([tau[k] + ub[i] * ub[j] for k, (i, j) in enumerate(L.PAIRS)])
    I = L.Interp(16, 17, 12, y, 16, 12, y)
    ul, T = L.les_stress(ub, fuu, I)
    assert np.max(np.abs(ul - ub)) < 1e-14
    assert np.max(np.abs(T - tau)) < 1e-12


def test_constant_velocity_leaves_interpolated_tau():
    """Spatially constant ubar: I(ubar_i ubar_j) = I(ubar_i) I(ubar_j), so T = I(tau)."""
    y, y_les, I = _grids(ratio=2)
    rng = np.random.default_rng(3)
    ub = np.ones((3, 16, 17, 12)) * np.array([1.3, -0.2, 0.7])[:, None, None, None]
    tau = rng.standard_normal((6, 16, 17, 12))
    fuu = np.stack([tau[k] + ub[i] * ub[j] for k, (i, j) in enumerate(L.PAIRS)])
    _, T = L.les_stress(ub, fuu, I)
    assert np.max(np.abs(T - np.stack([I(t) for t in tau]))) < 1e-13


@pytest.mark.parametrize("deg", [1, 2])
def test_derivative_exact_on_polynomials(deg):
    """The second-order three-point derivatives are exact up to degree 2."""
    y = synth.ygrid(13, "tanh", 2.5)
    g = np.broadcast_to((0.5 + y + (0.8 * y ** 2 if deg == 2 else 0.0 * y))[None, :, None], (3, 13, 2))
    ref = (1.0 + (1.6 * y if deg == 2 else 0.0 * y))[None, :, None]
    assert np.max(np.abs(L.d_dy(g, y) - ref)) < 1e-12


def test_commutation_error_zero_on_linear_and_second_order():
    """Zero for fields linear in y. Not zero on the stretched mesh with the
    LES nodes every other DNS node (the paper's remark). On a uniform mesh
    with coinciding nodes it is the difference of the three-point stencils
    of spacing 2h and h, so it falls by four per refinement (second order)."""
    y, y_les, I = _grids(nx=8, ny=33, nz=4, ratio=2)
    lin = np.broadcast_to((2.0 - 0.5 * y)[None, :, None], (8, 33, 4))
    assert L.commutation_error(lin, I) < 1e-13
    g = np.broadcast_to(np.sin(2.0 * y + 0.3)[None, :, None], (8, 33, 4))
    assert L.commutation_error(g, I) > 1e-4
    errs = []
    for ny in (33, 65, 129):
        y = np.linspace(-1, 1, ny)
        y_les = np.linspace(-1, 1, (ny - 1) // 2 + 1)
        I = L.Interp(4, ny, 4, y, 4, 4, y_les)
        g = np.broadcast_to(np.sin(2.0 * y + 0.3)[None, :, None], (4, ny, 4))
        errs.append(L.commutation_error(g, I))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.7 < errs[1] / errs[2] < 4.3, errs


def test_periodic_interpolation_equals_numpy_with_period():
    """x and z interpolation against numpy's interp with the period given
    (LES nodes between DNS nodes, including the wrap past the last one)."""
    nx, nz, lx, lz = 10, 9, 3.0, 2.0
    y = np.linspace(-1, 1, 5)
    I = L.Interp(nx, 5, nz, y, 7, 4, y)
    g = np.random.default_rng(4).standard_normal((nx, 5, nz))
    out = I(g)
    x, xl = np.arange(nx) * lx / nx, np.arange(7) * lx / 7
    z, zl = np.arange(nz) * lz / nz, np.arange(4) * lz / 4
    ref = np.empty((7, 5, 4))
    for j in range(5):
        gx = np.stack([np.interp(xl, x, g[:, j, k], period=lx) for k in range(nz)], axis=1)   # [7, nz]
        ref[:, j, :] = np.stack([np.interp(zl, z, gx[i], period=lz) for i in range(7)])
    assert np.max(np.abs(out - ref)) < 1e-14
