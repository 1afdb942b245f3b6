"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these retypes the oracle's formulas: every expected value comes
from a closed form (Poisson summation of a sampled Gaussian, eigenfunctions
of the reflected line, the filter of a single Fourier mode), from a brute
force evaluation of eq. (2) on an explicitly extended grid built node by
node, or from an invariant the paper states (constants preserved, odd
fields vanish at the wall after filtering, commutation with derivatives,
the stress is a covariance under a positive kernel).
"""
import math

import numpy as np
import pytest

from oracle import filter_ref as R
from paper_1902_02508_amd import synth


def theta_ratio(k, h, delta, pmax=60):
    """Transfer function of a normalised sampled Gaussian (Poisson summation)."""
    s2 = delta * delta / 12.0
    p = np.arange(-pmax, pmax + 1)
    num = np.exp(-0.5 * s2 * (k + 2 * np.pi * p / h) ** 2).sum()
    den = np.exp(-0.5 * s2 * (2 * np.pi * p / h) ** 2).sum()
    return num / den


# ------------------------------------------------------------ P1 constants

@pytest.mark.parametrize("kind", ["cgl", "tanh", "uniform"])
def test_constants_preserved(kind):
    y = synth.ygrid(17, kind)
    ops = R.Operators(8, 17, 6, 2.0, 1.5, y, 0.7, 0.2, 0.4)
    f = np.full((8, 17, 6), 3.25)
    assert np.max(np.abs(R.filt(f, 1, ops) - 3.25)) < 1e-14
    assert abs(ops.wx.sum() - 1) < 1e-15 and abs(ops.wz.sum() - 1) < 1e-15
    assert np.all(ops.wx >= 0) and np.all(ops.wp >= 0)


# --------------------------------------------- P2 periodic transfer function

@pytest.mark.parametrize("n,length,delta", [(32, 2 * math.pi, 2 * math.pi / 16),
                                            (48, 3.0, 0.9), (10, 1.0, 0.7), (64, 1.0, 0.02)])
def test_periodic_mode_theta_series(n, length, delta):
    w = R.periodic_weights(n, length, delta)
    c = R.circulant(w)
    h = length / n
    x = np.arange(n) * h
    for q in [0, 1, 3, n // 4, n // 2 - 1]:
        k = 2 * np.pi * q / length
        f = np.cos(k * x + 0.3)
        lam = theta_ratio(k, h, delta)
        assert np.max(np.abs(c @ f - lam * f)) < 1e-14


def test_periodic_mode_continuous_limit():
    # well-resolved kernel: the discrete transfer equals the analytic Gaussian's
    n, length, delta = 192, 4 * math.pi, math.pi / 6
    c = R.circulant(R.periodic_weights(n, length, delta))
    x = np.arange(n) * length / n
    for q in [1, 5, 12]:
        k = 2 * np.pi * q / length
        lam = math.exp(-k * k * delta * delta / 24.0)
        assert np.max(np.abs(c @ np.sin(k * x) - lam * np.sin(k * x))) < 1e-11


# ------------------------------ P3 eigenfunctions of the reflected channel

@pytest.mark.parametrize("ny", [9, 17, 33])
@pytest.mark.parametrize("dy", [0.05, 0.3, 1.0, 3.0])
def test_uniform_y_eigenfunctions(ny, dy):
    """On a uniform grid the two-wall extension is a uniform periodic lattice
    of period 4; cos(n pi (y+1)/2) is even and sin(n pi (y+1)/2) odd about
    both walls, so they are eigenvectors of W^+ and W^- with the theta-series
    eigenvalue at wavenumber n pi/2."""
    y = synth.ygrid(ny, "uniform")
    h = 2.0 / (ny - 1)
    wp, wm = R.y_operators(y, dy)
    for n in [0, 1, 2, 5, ny - 2]:
        kap = n * np.pi / 2
        lam = theta_ratio(kap, h, dy)
        c = np.cos(kap * (y + 1))
        s = np.sin(kap * (y + 1))
        assert np.max(np.abs(wp @ c - lam * c)) < 1e-14
        assert np.max(np.abs(wm @ s - lam * s)) < 1e-14


# ------------------------------------- P4/P5 brute force on extended grids

def _periodic_nodes(n, length, delta):
    h = length / n
    reach = 6 * delta + length
    P = int(math.ceil(reach / length)) + 1
    pos, idx = [], []
    for p in range(-P, P + 1):
        for i in range(n):
            pos.append((i + p * n) * h)
            idx.append(i)
    return np.array(pos), np.array(idx), np.full(len(pos), h)


def _extended_y_nodes(y, parity, delta):
    """Explicit node list of the reflected channel: every node with its
    value index, sign and a trapezoid weight taken from its sorted neighbours."""
    ny = len(y)
    N = int(math.ceil((6 * delta + 4) / 4)) + 2
    pos, idx, sgn = [], [], []
    for n in range(-N, N + 1):
        for j in range(ny):
            pos.append(y[j] + 4 * n); idx.append(j); sgn.append(1.0)
        for j in range(1, ny - 1):
            pos.append(4 * n + 2 - y[j]); idx.append(j); sgn.append(float(parity))
    pos, idx, sgn = map(np.array, (pos, idx, sgn))
    order = np.argsort(pos)
    pos, idx, sgn = pos[order], idx[order], sgn[order]
    assert np.all(np.diff(pos) > 0)          # no node appears twice
    w = np.empty(len(pos))
    w[1:-1] = 0.5 * (pos[2:] - pos[:-2])
    w[0] = pos[1] - pos[0]
    w[-1] = pos[-1] - pos[-2]
    if parity < 0:                           # an odd extension is zero at the walls
        sgn = np.where((idx == 0) | (idx == ny - 1), 0.0, sgn)
    return pos, idx, sgn, w


def brute_force_filter(f, parity, nx, nz, lx, lz, y, dx_, dy_, dz_):
    """eq. (2) as one triple sum over the explicitly extended 3-D grid."""
    ny = len(y)
    xp, xi, xw = _periodic_nodes(nx, lx, dx_)
    zp, zi, zw = _periodic_nodes(nz, lz, dz_)
    yp, yi, ys, yw = _extended_y_nodes(y, parity, dy_)
    vext = f[np.ix_(xi, yi, zi)] * ys[None, :, None]
    out = np.empty((nx, ny, nz))
    for i in range(nx):
        gx = xw * R.gauss(i * lx / nx - xp, dx_)
        for j in range(ny):
            gy = yw * R.gauss(y[j] - yp, dy_)
            for k in range(nz):
                gz = zw * R.gauss(k * lz / nz - zp, dz_)
                kern = gx[:, None, None] * gy[None, :, None] * gz[None, None, :]
                out[i, j, k] = np.sum(kern * vext) / np.sum(kern)
    return out


@pytest.mark.parametrize("kind,dy", [("tanh", 0.3), ("cgl", 0.5), ("uniform", 1.2)])
def test_brute_force_3d(kind, dy):
    rng = np.random.default_rng(7)
    nx, ny, nz, lx, lz = 6, 9, 5, 2.0, 1.3
    y = synth.ygrid(ny, kind)
    ops = R.Operators(nx, ny, nz, lx, lz, y, 0.8, dy, 0.5)
    f = rng.standard_normal((nx, ny, nz))
    for parity in (1, -1):
        g = f.copy()
        if parity < 0:
            g[:, [0, -1], :] = 0.0
        ref = brute_force_filter(g, parity, nx, nz, lx, lz, y, 0.8, dy, 0.5)
        assert np.max(np.abs(R.filt(g, parity, ops) - ref)) < 1e-13


@pytest.mark.parametrize("kind", ["tanh", "cgl"])
@pytest.mark.parametrize("ny,dy", [(17, 0.05), (33, 0.1), (12, 0.8), (5, 2.5)])
def test_brute_force_y_fold(kind, ny, dy):
    """W^s equals the plain quadrature over the explicit reflected line."""
    y = synth.ygrid(ny, kind)
    rng = np.random.default_rng(ny)
    f = rng.standard_normal(ny)
    wp, wm = R.y_operators(y, dy)
    for parity, W in ((1, wp), (-1, wm)):
        pos, idx, sgn, w = _extended_y_nodes(y, parity, dy)
        ref = np.array([np.sum(w * R.gauss(yi - pos, dy) * sgn * f[idx]) / np.sum(w * R.gauss(yi - pos, dy))
                        for yi in y])
        assert np.max(np.abs(W @ f - ref)) < 1e-14


# ------------------------------------------------------ P6 wall conditions

def test_wall_values_vanish():
    cfg = synth.config("tiny")
    y, u = synth.make_snapshot(cfg, 0, np.float64)
    ops = R.Operators.from_config(cfg)
    ub, tau = R.sgs_stress(u, ops)
    scale = np.abs(u).max() ** 2
    assert np.max(np.abs(ub[1][:, [0, -1], :])) < 1e-15 * np.abs(u).max()
    assert np.max(np.abs(tau[1][:, [0, -1], :])) < 1e-15 * scale   # tau_12
    assert np.max(np.abs(tau[4][:, [0, -1], :])) < 1e-15 * scale   # tau_23
    # the even components do not vanish there
    assert np.max(np.abs(tau[0][:, [0, -1], :])) > 1e-8


# ----------------------------------------------- P7 commutation, divergence

def _dspec(f, length, axis):
    n = f.shape[axis]
    k = 2 * np.pi * np.fft.fftfreq(n, d=length / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    shape = [1] * f.ndim
    shape[axis] = n
    return np.real(np.fft.ifft(1j * k.reshape(shape) * np.fft.fft(f, axis=axis), axis=axis))


def _dy_uniform(f, parity):
    """Central difference on the reflected uniform line."""
    ny = f.shape[1]
    h = 2.0 / (ny - 1)
    ext = np.concatenate([parity * f[:, 1:2], f, parity * f[:, -2:-1]], axis=1)
    return (ext[:, 2:] - ext[:, :-2]) / (2 * h)


def test_divergence_commutes_uniform_y():
    """div F(u) = F(div u): translation invariance (commutation) plus the
    parity-consistent extension, which keeps the extended field solenoidal."""
    cfg = synth.config("tiny", ykind="uniform")
    y, u = synth.make_snapshot(cfg, 3, np.float64)
    ops = R.Operators.from_config(cfg)

    def div(v):
        return (_dspec(v[0], cfg.lx, 0) + _dy_uniform(v[1], -1) + _dspec(v[2], cfg.lz, 2))

    ub = np.stack([R.filt(u[i], R.PARITY[i], ops) for i in range(3)])
    lhs = div(ub)
    rhs = R.filt(div(u), 1, ops)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.abs(div(u)).max() + 1e-13


def _dy_stretched(y, parity):
    """Three-point second-order derivative on non-uniform nodes for a field of
    the given parity; at a wall the neighbour across it is the mirror of the
    first interior node, carrying parity * f_1 (the eq. (7) reflection)."""
    ny = len(y)
    D = np.zeros((ny, ny))
    for j in range(1, ny - 1):
        hm, hp = y[j] - y[j - 1], y[j + 1] - y[j]
        D[j, j - 1] = -hp / (hm * (hm + hp))
        D[j, j] = (hp - hm) / (hm * hp)
        D[j, j + 1] = hm / (hp * (hm + hp))
    D[0, 1] = (1 - parity) / (2 * (y[1] - y[0]))
    D[-1, -2] = -(1 - parity) / (2 * (y[-1] - y[-2]))
    return D


@pytest.mark.parametrize("kind", ["tanh", "cgl"])
def test_divergence_stretched_y_equals_commutator(kind):
    """On a stretched y grid the filtered divergence differs from the filtered
    divergence by exactly F_xz (D_y W^- - W^+ D_y) u2: x and z are periodic
    and spectral, so they commute with the translation-invariant x/z filter
    (Sec. 2.1), and what is left is the y commutator of the discrete
    derivative with the wall-extended y filter."""
    cfg = synth.config("tiny", ykind=kind, stretch=2.0, ny=33)
    y, u = synth.make_snapshot(cfg, 3, np.float64)
    ops = R.Operators.from_config(cfg)
    Dodd = _dy_stretched(y, -1)

    def div(v):
        return (_dspec(v[0], cfg.lx, 0) + np.einsum("ij,xjz->xiz", Dodd, v[1]) + _dspec(v[2], cfg.lz, 2))

    ub = np.stack([R.filt(u[i], R.PARITY[i], ops) for i in range(3)])
    comm = Dodd @ ops.wm - ops.wp @ Dodd
    rhs = R.filt(div(u), 1, ops) + R.filt_xz(np.einsum("ij,xjz->xiz", comm, u[1]), ops)
    scale = np.abs(np.einsum("ij,xjz->xiz", Dodd, u[1])).max()
    assert np.max(np.abs(div(ub) - rhs)) < 1e-12 * scale


@pytest.mark.parametrize("kind", ["tanh", "cgl"])
def test_divergence_commutator_second_order(kind):
    """The commutator D_y W^- - W^+ D_y applied to an admissible u2 (odd
    about both walls, zero there) is the discretisation commutation error of
    Sec. 3: the continuous filter of constant width commutes with d/dy on
    the reflected line (Sec. 2.1, eq. (7)), the trapezoid quadrature and the
    three-point difference are second order, so it must vanish like h^2.
    Observed order >= 1.8 on every refinement Ny 33 -> 65 -> 129 -> 257."""
    errs = []
    for ny in (33, 65, 129, 257):
        y = synth.ygrid(ny, kind, 2.0)
        wp, wm = R.y_operators(y, 0.1)
        u2 = (1 - y ** 2) ** 2 * np.sin(3 * y + 0.2)
        D = _dy_stretched(y, -1)
        errs.append(np.max(np.abs((D @ wm - wp @ D) @ u2)) / np.max(np.abs(D @ u2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    print(kind, " ".join(f"{e:.2e}" for e in errs), " orders", " ".join(f"{o:.2f}" for o in orders))
    assert min(orders) >= 1.8, (errs, orders)
    assert errs[-1] < 5e-5


def test_divergence_commutator_catches_planted_mistakes(monkeypatch):
    """Swapped parities or a half wall cell break the second-order decay."""
    def orders(make):
        errs = []
        for ny in (33, 65, 129, 257):
            y = synth.ygrid(ny, "tanh", 2.0)
            wp, wm = make(y)
            u2 = (1 - y ** 2) ** 2 * np.sin(3 * y + 0.2)
            D = _dy_stretched(y, -1)
            errs.append(np.max(np.abs((D @ wm - wp @ D) @ u2)) / np.max(np.abs(D @ u2)))
        return [math.log2(errs[i] / errs[i + 1]) for i in range(3)]

    assert min(orders(lambda y: R.y_operators(y, 0.1)[::-1])) < 0.0
    orig = R.wall_weights

    def half_wall(yy):
        om = orig(yy)
        om[0] *= 0.5
        om[-1] *= 0.5
        return om
    monkeypatch.setattr(R, "wall_weights", half_wall)
    assert min(orders(lambda y: R.y_operators(y, 0.1))) < 1.5


def test_generator_is_solenoidal_and_no_slip():
    """The synthetic input is divergence-free and vanishes at both walls."""
    for name in ("tiny", "dns192"):
        cfg = synth.config(name, nx=48, nz=40, kmax=8) if name == "dns192" else synth.config(name)
        y, terms = synth.snapshot_factors(cfg, 1)
        u = synth.assemble(cfg, terms, np.float64)
        assert np.max(np.abs(u[:, :, [0, -1], :])) < 1e-14
        e = (1 - y ** 2) ** 2
        de = -4 * y * (1 - y ** 2)
        (g2, f2), = terms[1]                 # u2 = s e(y) f2(x, z)
        mid = len(y) // 2
        s = g2[mid] / e[mid]
        assert np.allclose(g2, s * e, rtol=1e-14, atol=1e-15)
        dy_u2 = (s * de)[None, :, None] * f2[:, None, :]
        d = _dspec(u[0], cfg.lx, 0) + dy_u2 + _dspec(u[2], cfg.lz, 2)
        assert np.max(np.abs(d)) < 1e-11 * np.abs(dy_u2).max()


# ------------------------------------------------------ P8-P11 the stress

@pytest.fixture(scope="module")
def tiny_case():
    cfg = synth.config("tiny")
    y, u = synth.make_snapshot(cfg, 0, np.float64)
    ops = R.Operators.from_config(cfg)
    return cfg, y, u, ops


def test_stress_symmetric_and_realizable(tiny_case):
    cfg, y, u, ops = tiny_case
    ub, tau = R.sgs_stress(u, ops, full=True)
    assert np.array_equal(tau, np.swapaxes(tau, 0, 1))
    t = np.moveaxis(tau, (0, 1), (-2, -1))
    ev = np.linalg.eigvalsh(t)
    scale = np.max(np.abs(u)) ** 2
    assert ev.min() > -1e-13 * scale
    tr = np.trace(t, axis1=-2, axis2=-1)
    assert tr.min() > -1e-13 * scale


def test_single_mode_stress():
    """u1 = A cos(kx + phi), u3 = B cos(qz + chi): closed forms of tau_11 and tau_13."""
    nx, ny, nz, lx, lz = 24, 9, 20, 2 * np.pi, np.pi
    y = synth.ygrid(ny, "tanh")
    dx_, dz_ = 0.9, 0.5
    ops = R.Operators(nx, ny, nz, lx, lz, y, dx_, 0.3, dz_)
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    k, q, A, B = 3.0, 4.0, 1.7, 0.6
    th = k * x + 0.4
    u = np.zeros((3, nx, ny, nz))
    u[0] = A * np.cos(th)[:, None, None]
    u[2] = B * np.cos(q * z * 1.0 + 1.1)[None, None, :] * np.ones((nx, ny, 1))
    ub, tau = R.sgs_stress(u, ops)
    lk = theta_ratio(k, lx / nx, dx_)
    l2k = theta_ratio(2 * k, lx / nx, dx_)
    t11 = A * A / 2 * (1 + l2k * np.cos(2 * th)) - lk ** 2 * A * A * np.cos(th) ** 2
    assert np.max(np.abs(tau[0] - t11[:, None, None])) < 1e-14
    assert np.max(np.abs(tau[2])) < 1e-15
    assert np.max(np.abs(tau[1])) < 1e-15


def test_mean_shift_identity(tiny_case):
    cfg, y, u, ops = tiny_case
    ub, tau = R.sgs_stress(u, ops)
    rng = np.random.default_rng(1)
    for m in (R.plane_mean(u[0]), rng.standard_normal(cfg.ny), np.full(cfg.ny, 5.0)):
        ub2, tau2 = R.sgs_stress_shifted(u, ops, m)
        assert np.max(np.abs(ub2 - ub)) < 1e-13
        assert np.max(np.abs(tau2 - tau)) < 1e-12 * np.abs(u).max() ** 2


def test_galilean_invariance(tiny_case):
    cfg, y, u, ops = tiny_case
    _, tau = R.sgs_stress(u, ops)
    v = u.copy()
    v[0] += 2.5
    _, tau2 = R.sgs_stress(v, ops)
    assert np.max(np.abs(tau2 - tau)) < 1e-12 * np.abs(v).max() ** 2


# ------------------------------------------------------- P12 small widths

def test_small_width_gradient_limit():
    """tau_11 -> sigma^2 (du/dx)^2 as the width shrinks (leading term of the
    expansion of a filtered product in powers of the width)."""
    n, L = 512, 2 * np.pi
    h = L / n
    x = np.arange(n) * h
    errs = []
    for sig in (4 * h, 8 * h):
        delta = sig * math.sqrt(12.0)
        c = R.circulant(R.periodic_weights(n, L, delta))
        u = np.sin(x)
        tau = c @ (u * u) - (c @ u) ** 2
        lead = sig ** 2 * np.cos(x) ** 2
        errs.append(np.linalg.norm(tau - lead) / np.linalg.norm(lead))
        assert errs[-1] < 2 * sig ** 2
    assert 3.0 < errs[1] / errs[0] < 5.0


# ------------------------------------------------------------- norms

def test_norm_closed_forms():
    y = synth.ygrid(2001, "uniform")
    b = np.ones_like(y)
    a = 1 + 1e-3 * y
    assert abs(R.profile_error(a, b, y) - 1e-3 / math.sqrt(3)) < 1e-9
    assert abs(R.profile_error(a, b, y, half=True) - 1e-3 / math.sqrt(3)) < 1e-9
    f = np.random.default_rng(0).standard_normal((4, len(y), 3)) + 2
    assert abs(R.rel_l2(1.01 * f, f, y) - 0.01) < 1e-14
    assert np.allclose(R.plane_mean(f), f.mean(axis=(0, 2)))


# ------------------------------------------------ sampled-point evaluation

def test_points_match_dense(tiny_case):
    cfg, y, u, ops = tiny_case
    ub, tau = R.sgs_stress(u, ops)
    rng = np.random.default_rng(3)
    pts = np.stack([rng.integers(0, cfg.nx, 40), rng.integers(0, cfg.ny, 40),
                    rng.integers(0, cfg.nz, 40)], axis=1)
    pts[:3, 1] = [0, cfg.ny - 1, cfg.ny // 2]
    ubp, taup = R.sgs_points(u, ops, pts)
    ix, iy, iz = pts.T
    assert np.max(np.abs(ubp - ub[:, ix, iy, iz])) < 1e-13
    assert np.max(np.abs(taup - tau[:, ix, iy, iz])) < 1e-12


# ----------------------------------------------- planted mistakes are caught

def test_pins_catch_planted_mistakes(monkeypatch):
    """Each plausible slip in the operator build fails one of the pins above."""
    y = synth.ygrid(17, "tanh")
    rng = np.random.default_rng(5)
    f = rng.standard_normal(17)
    good = R.y_operators(y, 0.3)

    def fold_error(ops_pair):
        worst = 0.0
        for parity, W in ((1, ops_pair[0]), (-1, ops_pair[1])):
            pos, idx, sgn, w = _extended_y_nodes(y, parity, 0.3)
            ref = np.array([np.sum(w * R.gauss(yi - pos, 0.3) * sgn * f[idx]) /
                            np.sum(w * R.gauss(yi - pos, 0.3)) for yi in y])
            worst = max(worst, np.max(np.abs(W @ f - ref)))
        return worst

    assert fold_error(good) < 1e-14
    # half a cell at the walls instead of the full cell of the extended line
    orig = R.wall_weights

    def half_wall(yy):
        om = orig(yy)
        om[0] *= 0.5
        om[-1] *= 0.5
        return om
    monkeypatch.setattr(R, "wall_weights", half_wall)
    assert fold_error(R.y_operators(y, 0.3)) > 1e-6
    monkeypatch.setattr(R, "wall_weights", orig)
    # transposed operator
    assert fold_error((good[0].T, good[1].T)) > 1e-6
    # swapped parities
    assert fold_error((good[1], good[0])) > 1e-6


def test_row_restricted_outputs_equal_full_oracle():
    """sgs_rows (the y operator's selected rows over the nodes they reach)
    agrees with the full oracle restricted to those rows, walls included."""
    for base, over in (("tiny", {}), ("dns192", dict(nx=24, nz=20, ny=37))):
        cfg = synth.config(base, **over)
        y, u = synth.make_snapshot(cfg, 3)
        ops = R.Operators.from_config(cfg)
        ub, tau = R.sgs_stress(u.astype(np.float64), ops)
        rows = [0, 1, cfg.ny // 2, cfg.ny - 2, cfg.ny - 1]
        rub, rtau = R.sgs_rows(u, ops, rows)
        scale_u = np.abs(ub).max()
        scale_t = np.abs(tau).max()
        assert np.max(np.abs(rub - ub[:, :, rows, :])) < 1e-13 * scale_u
        assert np.max(np.abs(rtau - tau[:, :, rows, :])) < 1e-12 * scale_t
