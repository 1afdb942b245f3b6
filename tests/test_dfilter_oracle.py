"""Pins of the FP64 oracle of the differential filter (Sec. 3, eq. (12)).

The oracle solves (1 - a^2 lap) ubar = u with spectral x/z derivatives and
the three-point wall-normal difference on the reflected channel of eq. (7).
Each test checks it against something other than itself: closed-form
eigenpairs, a dense brute-force solve of the full 3-D operator assembled
from its explicit definition, the forward operator applied node by node,
and single-mode closed forms of tau.
"""
import math

import numpy as np
import pytest

from oracle import dfilter_ref as D
from paper_1902_02508_amd import synth


def _ops(nx, ny, nz, lx, lz, y, a=0.1):
    return D.DOperators(nx, ny, nz, lx, lz, y, a)


def _uniform_y(ny):
    return np.linspace(-1.0, 1.0, ny)


@pytest.mark.parametrize("n,kxi,kzi", [(1, 0, 0), (3, 2, 1), (6, 5, 3), (11, 0, 5), (4, 8, 6)])
def test_eigenfunctions_uniform_y(n, kxi, kzi):
    """On a uniform y grid cos(n pi (y+1)/2) (even) and sin(n pi (y+1)/2)
    (odd) are eigenvectors of the reflected three-point difference with
    eigenvalue -(2/h^2)(1 - cos(n pi h / 2)); with an x/z Fourier mode the
    filter divides by 1 + a^2 (kx^2 + kz^2) + a^2 (2/h^2)(1 - cos(n pi h/2))."""
    nx, ny, nz, lx, lz, a = 16, 25, 12, 2 * math.pi, math.pi, 0.13
    y = _uniform_y(ny)
    h = y[1] - y[0]
    ops = _ops(nx, ny, nz, lx, lz, y, a)
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    kx, kz = 2 * math.pi * kxi / lx, 2 * math.pi * kzi / lz
    kap = n * math.pi / 2
    lam = 1.0 / (1.0 + a * a * (kx * kx + kz * kz) + a * a * (2.0 / h ** 2) * (1.0 - math.cos(kap * h)))
    xz = np.cos(kx * x[:, None, None] + kz * z[None, None, :] + 0.3)
    for parity, prof in ((1, np.cos(kap * (y + 1))), (-1, np.sin(kap * (y + 1)))):
        f = xz * prof[None, :, None]
        if parity < 0:
            f[:, [0, -1], :] = 0.0
        g = D.dfilt(f, parity, ops)
        assert np.max(np.abs(g - lam * f)) < 1e-13, parity


def _spectral_d2(n, length):
    """Dense periodic second-derivative matrix from its definition,
    (1/n) sum_k (-k^2) exp(i k (x_p - x_q)), the grid wavenumbers listed by
    explicit integer loops (the Nyquist mode with k = pi n / L)."""
    x = np.arange(n) * length / n
    m = np.zeros((n, n))
    for s in range(-(n // 2), (n + 1) // 2):
        k = 2 * math.pi * s / length
        m += np.real(-k * k * np.exp(1j * k * (x[:, None] - x[None, :]))) / n
    return m


def _fd_matrix(y, parity):
    """The reflected three-point difference written out row by row on all ny
    nodes (odd rows at the walls left empty: those values are zero)."""
    ny = len(y)
    d = np.zeros((ny, ny))
    ext = np.concatenate([[-2.0 - y[1]], y, [2.0 - y[-2]]])   # mirror nodes of eq. (7)
    for j in range(ny):
        if parity < 0 and j in (0, ny - 1):
            continue
        hm = ext[j + 1] - ext[j]
        hp = ext[j + 2] - ext[j + 1]
        s = 2.0 / (hm + hp)
        for off, w in ((-1, s / hm), (0, -s / hm - s / hp), (1, s / hp)):
            q = j + off
            sign = 1.0
            if q < 0:
                q, sign = 1, parity            # reflected neighbour
            elif q >= ny:
                q, sign = ny - 2, parity
            d[j, q] += sign * w
    if parity < 0:
        d[:, 0] = 0.0
        d[:, -1] = 0.0
    return d


@pytest.mark.parametrize("parity", [1, -1])
def test_brute_force_dense_solve(parity):
    """The FFT + tridiagonal oracle equals a dense solve of the whole 3-D
    operator I - a^2 (Lx + Dy + Lz) assembled by Kronecker products."""
    nx, ny, nz, lx, lz, a = 6, 9, 5, 2.0, 1.3, 0.21
    y = synth.ygrid(ny, "tanh", 2.0)
    ops = _ops(nx, ny, nz, lx, lz, y, a)
    lxm, lzm, dy = _spectral_d2(nx, lx), _spectral_d2(nz, lz), _fd_matrix(y, parity)
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    lap = np.kron(np.kron(lxm, iy), iz) + np.kron(np.kron(ix, dy), iz) + np.kron(np.kron(ix, iy), lzm)
    A = np.eye(nx * ny * nz) - a * a * lap
    rng = np.random.default_rng(3)
    f = rng.standard_normal((nx, ny, nz))
    if parity < 0:
        f[:, [0, -1], :] = 0.0
        keep = np.ones((nx, ny, nz), bool)
        keep[:, [0, -1], :] = False
        k = keep.ravel()
        sol = np.zeros(nx * ny * nz)
        sol[k] = np.linalg.solve(A[np.ix_(k, k)], f.ravel()[k])
    else:
        sol = np.linalg.solve(A, f.ravel())
    g = D.dfilt(f, parity, ops)
    assert np.max(np.abs(g.ravel() - sol)) < 1e-12


@pytest.mark.parametrize("parity", [1, -1])
def test_forward_operator_recovers_input(parity):
    cfg = synth.config("tiny")
    ops = D.DOperators.from_config(cfg)
    f = np.random.default_rng(5).standard_normal((cfg.nx, cfg.ny, cfg.nz))
    if parity < 0:
        f[:, [0, -1], :] = 0.0
    g = D.dfilt(f, parity, ops)
    assert np.max(np.abs(D.laplacian_apply(g, parity, ops) - f)) < 1e-11


def test_constant_preserved_and_odd_walls_zero():
    cfg = synth.config("tiny")
    ops = D.DOperators.from_config(cfg)
    one = np.ones((cfg.nx, cfg.ny, cfg.nz))
    assert np.max(np.abs(D.dfilt(one, 1, ops) - 1.0)) < 1e-14
    f = np.random.default_rng(7).standard_normal(one.shape)
    g = D.dfilt(f, -1, ops)
    assert np.all(g[:, [0, -1], :] == 0.0)


def test_single_mode_tau_closed_form():
    """u1 = A cos(k x), u2 = u3 = 0 (constant in y and z): F(u1) = A cos(kx)/(1 + a^2 k^2),
    F(u1^2) = A^2/2 (1 + cos(2kx)/(1 + 4 a^2 k^2)), and tau_11 their difference;
    the other components vanish."""
    nx, ny, nz, lx, lz, a, A = 32, 17, 8, 2 * math.pi, 1.0, 0.17, 1.7
    y = synth.ygrid(ny, "tanh", 2.0)
    ops = _ops(nx, ny, nz, lx, lz, y, a)
    x = np.arange(nx) * lx / nx
    k = 2 * math.pi * 5 / lx
    u = np.zeros((3, nx, ny, nz))
    u[0] = A * np.cos(k * x)[:, None, None]
    ub, tau = D.sgs_stress(u, ops)
    c = np.cos(k * x)
    ref11 = A * A / 2 * (1 + np.cos(2 * k * x) / (1 + 4 * a * a * k * k)) - (A * c / (1 + a * a * k * k)) ** 2
    assert np.max(np.abs(tau[0] - ref11[:, None, None])) < 1e-13
    assert np.max(np.abs(tau[1:])) < 1e-13


def test_tau_symmetric_galilean_and_shift_identity():
    cfg = synth.config("tiny", nx=16, nz=12, ny=17)
    ops = D.DOperators.from_config(cfg)
    y, u = synth.make_snapshot(cfg, 2)
    u = u.astype(np.float64)
    ub, tau = D.sgs_stress(u, ops)
    # tau_ij from the products in either order
    for k, (i, j) in enumerate(D.PAIRS):
        alt = D.dfilt(u[j] * u[i], D.PARITY[i] * D.PARITY[j], ops) - ub[j] * ub[i]
        assert np.max(np.abs(alt - tau[k])) < 1e-13
    # u1 + c leaves tau unchanged (constants are preserved)
    v = u.copy()
    v[0] += 3.7
    _, tau2 = D.sgs_stress(v, ops)
    assert np.max(np.abs(tau2 - tau)) < 1e-11
    # the mean-shift form equals the plain one for any profile
    m = np.sin(3 * y) + 0.4
    ub3, tau3 = D.sgs_stress_shifted(u, ops, m)
    assert np.max(np.abs(ub3 - ub)) < 1e-13
    assert np.max(np.abs(tau3 - tau)) < 1e-12


def test_planted_parity_mistake_is_caught():
    """Treating an odd field as even changes the output near the walls by
    far more than the pins' tolerance (the eigenfunction pin would fail)."""
    ny = 25
    y = _uniform_y(ny)
    ops = _ops(8, ny, 4, 1.0, 1.0, y, 0.13)
    prof = np.sin(3 * math.pi / 2 * (y + 1))
    f = np.ones((8, ny, 4)) * prof[None, :, None]
    f[:, [0, -1], :] = 0.0
    assert np.max(np.abs(D.dfilt(f, 1, ops) - D.dfilt(f, -1, ops))) > 1e-3


@pytest.mark.parametrize("parity", [1, -1])
def test_inverse_operator_eigenvalues(parity):
    """The inverse filter (1 - a^2 lap), applied forward, multiplies the
    eigenfunctions of the reflected difference by 1 + a^2 (kx^2 + kz^2)
    + a^2 (2/h^2)(1 - cos(n pi h / 2)) on a uniform y grid."""
    nx, ny, nz, lx, lz, a = 12, 21, 10, 2.0, 1.5, 0.17
    y = _uniform_y(ny)
    h = y[1] - y[0]
    ops = _ops(nx, ny, nz, lx, lz, y, a)
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    kx, kz = 2 * math.pi * 3 / lx, 2 * math.pi * 2 / lz
    kap = 5 * math.pi / 2
    lam = 1.0 + a * a * (kx * kx + kz * kz) + a * a * (2.0 / h ** 2) * (1.0 - math.cos(kap * h))
    xz = np.sin(kx * x[:, None, None] + kz * z[None, None, :] - 0.4)
    prof = np.cos(kap * (y + 1)) if parity > 0 else np.sin(kap * (y + 1))
    f = xz * prof[None, :, None]
    if parity < 0:
        f[:, [0, -1], :] = 0.0
    assert np.max(np.abs(D.laplacian_apply(f, parity, ops) - lam * f)) < 1e-12


@pytest.mark.parametrize("parity", [1, -1])
def test_inverse_operator_dense(parity):
    """laplacian_apply equals the dense 3-D operator I - a^2 (Lx + Dy + Lz)
    of explicit matrix definitions (odd fields: zero rows on the walls)."""
    nx, ny, nz, lx, lz, a = 6, 9, 5, 2.0, 1.3, 0.21
    y = synth.ygrid(ny, "tanh", 2.0)
    ops = _ops(nx, ny, nz, lx, lz, y, a)
    lxm, lzm, dy = _spectral_d2(nx, lx), _spectral_d2(nz, lz), _fd_matrix(y, parity)
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    lap = np.kron(np.kron(lxm, iy), iz) + np.kron(np.kron(ix, dy), iz) + np.kron(np.kron(ix, iy), lzm)
    A = np.eye(nx * ny * nz) - a * a * lap
    f = np.random.default_rng(8).standard_normal((nx, ny, nz))
    if parity < 0:
        f[:, [0, -1], :] = 0.0
    ref = (A @ f.ravel()).reshape(nx, ny, nz)
    if parity < 0:
        ref[:, [0, -1], :] = 0.0
    assert np.max(np.abs(D.laplacian_apply(f, parity, ops) - ref)) < 1e-11


# ---- eq. (11) and the eq. (9) extension (a negative test)

def _rms(a):
    return float(np.sqrt(np.mean(np.asarray(a) ** 2)))


def test_eq7_extension_meets_eq11_and_eq9_does_not():
    """With the eq. (7) parities (u2 odd) the filtered wall-normal velocity
    vanishes on the walls and the inverse filter returns the no-slip wall
    values of u1 and u3 (eq. (11)); with the eq. (9) parities (u2 even,
    u1 and u3 odd) ubar_2 is not zero on the walls, so eq. (11) fails."""
    cfg = synth.config("tiny", nx=16, nz=12, ny=17)
    ops = D.DOperators.from_config(cfg)
    y, u = synth.make_snapshot(cfg, 6)
    u = u.astype(np.float64)
    assert np.all(u[:, :, [0, -1], :] == 0.0)          # no-slip input
    good = [D.dfilt(u[i], p, ops) for i, p in enumerate((1, -1, 1))]
    assert np.all(good[1][:, [0, -1], :] == 0.0)
    for i in (0, 2):
        back = D.laplacian_apply(good[i], 1, ops)
        assert np.max(np.abs(back[:, [0, -1], :])) < 1e-12
    bad2 = D.dfilt(u[1], +1, ops)                        # eq. (9): u2 even
    # the wall value is of the size of the next row's, not zero
    assert _rms(bad2[:, 0, :]) > 0.1 * _rms(bad2[:, 1, :])


def test_eq9_extension_violates_eq11_for_the_gaussian_too():
    from oracle import filter_ref as R
    cfg = synth.config("tiny", nx=16, nz=12, ny=17)
    ops = R.Operators.from_config(cfg)
    y, u = synth.make_snapshot(cfg, 6)
    u = u.astype(np.float64)
    good = R.filt(u[1], -1, ops)
    bad = R.filt(u[1], +1, ops)
    assert np.max(np.abs(good[:, [0, -1], :])) < 1e-14
    assert _rms(bad[:, 0, :]) > 0.1 * _rms(bad[:, 1, :])


@pytest.mark.parametrize("parity,nth,sx,sz", [(1, 3, 5, 2), (-1, 2, 3, 4)])
def test_eigenmode_on_stretched_y(parity, nth, sx, sz):
    """On a stretched y grid: phi with D phi = lam phi (numpy's eigen-solver on
    the tridiagonal written from its definition) times a Fourier mode is
    divided by 1 + a^2 (kx^2 + kz^2) - a^2 lam by the filter and multiplied by
    it by the operator."""
    cfg = synth.config("tiny", nx=16, nz=12, ny=33)
    ops = D.DOperators.from_config(cfg)
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    A = _fd_matrix(y, parity)
    if parity < 0:
        A = A[1:-1, 1:-1]
    lam, vec = np.linalg.eig(A)
    k = np.argsort(-lam.real)[nth]
    phi = np.real(vec[:, k])
    if parity < 0:
        phi = np.concatenate([[0.0], phi, [0.0]])
    a = 0.1
    kx, kz = 2 * math.pi * sx / cfg.lx, 2 * math.pi * sz / cfg.lz
    g = 1.0 + a * a * (kx * kx + kz * kz) - a * a * lam[k].real
    x = np.arange(cfg.nx) * cfg.lx / cfg.nx
    z = np.arange(cfg.nz) * cfg.lz / cfg.nz
    u = np.cos(kx * x[:, None, None] + kz * z[None, None, :] + 0.25) * phi[None, :, None]
    assert np.max(np.abs(D.dfilt(u, parity, ops) - u / g)) < 1e-13
    assert np.max(np.abs(D.laplacian_apply(u, parity, ops) - u * g)) < 1e-11
