"""Pins of the FP64 closure reference: derivatives, network gradients, Adam,
the counter-based sampler and the standardisation."""
import math

import numpy as np
import pytest

from oracle import closure_ref as C
from paper_1902_02508_amd import synth


def test_spectral_derivative_exact_on_modes():
    n, L = 24, 3.0
    x = np.arange(n) * L / n
    for q in (0, 1, 5, 11):
        k = 2 * np.pi * q / L
        f = np.sin(k * x + 0.7)[:, None]
        d = C.spectral_derivative(f, L, 0)
        assert np.max(np.abs(d[:, 0] - k * np.cos(k * x + 0.7))) < 1e-12 * max(1, k)
    # the Nyquist mode of an even length has no derivative
    f = np.cos(np.pi * np.arange(n))[:, None]
    assert np.max(np.abs(C.spectral_derivative(f, L, 0))) < 1e-12


def test_dy_interior_exact_on_quadratics():
    y = synth.ygrid(17, "tanh", 2.0)
    f = 3.0 - 2.0 * y + 5.0 * y ** 2
    for par in (1, -1):
        D = C.dy_matrix(y, par)
        assert np.max(np.abs((D @ f)[1:-1] - (-2.0 + 10.0 * y[1:-1]))) < 1e-12


def test_dy_wall_rows_follow_the_extension():
    # even about both walls: zero slope at the walls
    for ny in (17, 33, 65):
        y = synth.ygrid(ny, "cgl")
        D = C.dy_matrix(y, 1)
        f = np.cos(np.pi * (y + 1))
        assert abs((D @ f)[0]) < 1e-14 and abs((D @ f)[-1]) < 1e-14
    # odd about both walls: mirror-symmetric difference, second-order accurate
    errs = []
    for ny in (17, 33, 65):
        y = synth.ygrid(ny, "uniform")
        D = C.dy_matrix(y, -1)
        f = np.sin(np.pi * (y + 1))
        d = D @ f
        errs.append(abs(d[0] - np.pi))
        assert abs(d[0] - f[1] / (y[1] + 1)) < 1e-14
    assert errs[1] / errs[2] > 3.5 and errs[0] / errs[1] > 3.5


def test_features_of_an_analytic_field():
    nx, ny, nz, lx, lz = 16, 21, 12, 2.0, 1.5
    y = synth.ygrid(ny, "uniform")
    x = np.arange(nx) * lx / nx
    z = np.arange(nz) * lz / nz
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    kx, kz = 2 * np.pi * 2 / lx, 2 * np.pi / lz
    ub = np.stack([np.sin(kx * X) * np.ones_like(Y), np.zeros_like(X), np.cos(kz * Z) * (1 + 0 * Y)])
    f = C.features(ub, y, lx, lz)
    assert np.max(np.abs(f[0] - kx * np.cos(kx * X))) < 1e-12
    assert np.max(np.abs(f[8] + kz * np.sin(kz * Z))) < 1e-12
    assert np.max(np.abs(f[[1, 2, 3, 4, 5, 6, 7]])) < 1e-12
    assert np.allclose(f[9], 1 - np.abs(Y))


def test_gelu_special_values():
    """x Phi(x): zero at 0 with slope 1/2; gelu(x) - gelu(-x) = x (Phi(-x) =
    1 - Phi(x)); tabulated normal-CDF values; the identity and zero limits."""
    assert C.gelu(0.0) == 0.0
    assert abs(C.gelu_grad(0.0) - 0.5) < 1e-15
    # Phi(1) and Phi(1.96) from standard normal tables (Abramowitz & Stegun 26.2)
    assert abs(C.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(C.gelu(-1.96) + 1.96 * (1.0 - 0.9750021048517795)) < 1e-15
    x = np.linspace(-8, 8, 161)
    assert np.max(np.abs(C.gelu(x) - C.gelu(-x) - x)) < 1e-14
    assert abs(C.gelu(40.0) - 40.0) < 1e-12 and abs(C.gelu(-40.0)) < 1e-300
    h = 1e-6
    fd = (C.gelu(x + h) - C.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - C.gelu_grad(x))) < 1e-8


def test_gelu_is_x_times_the_integrated_normal_density():
    """Phi by quadrature of the normal density, independent of erf."""
    from scipy.integrate import quad
    dens = lambda t: math.exp(-0.5 * t * t) / math.sqrt(2 * math.pi)  # noqa: E731
    for x in (-5.5, -2.3, -0.4, 0.25, 1.7, 3.9):
        half, _ = quad(dens, 0.0, x, epsabs=1e-15, epsrel=1e-13)
        phi = 0.5 + half
        assert abs(C.gelu(x) - x * phi) < 1e-13, x
        assert abs(C.gelu_grad(x) - (phi + x * dens(x))) < 1e-13, x


def test_kernel_gelu_approximation_bound():
    """The GPU kernels approximate x Phi(x) by max(x, 0) - h(min(|x|, 4)) with
    h a degree-7 polynomial; this bounds that approximation against the
    definition: 2.4e-4 on the value, 5e-3 on the derivative (its worst point
    is the clamp at |x| = 4). The GPU parity tolerances carry its effect."""
    import kernel_gelu as K
    assert all(float(np.float32(v)) == v for v in K.coefficients())
    assert K.coefficients()[0] == 0.5          # slope 1/2 at 0, as x Phi(x)
    x = np.linspace(-30, 30, 600001)
    assert np.max(np.abs(K.gelu(x) - C.gelu(x))) < 2.4e-4
    assert np.max(np.abs(K.gelu_grad(x) - C.gelu_grad(x))) < 5e-3


def test_kernel_gelu16_approximation_bound():
    """Inference evaluates the GELU in packed FP16: max(x, 0) - h(min(|x|,
    4)) with h a degree-7 polynomial in u = s/2 - 1 whose coefficients are
    FP16 numbers. In exact arithmetic it is within 2.4e-4 of x Phi(x); as
    the kernel rounds it (FP16 input, fused FP16 Horner steps, FP16 result)
    within 1.3e-3 absolute over |x| <= 10, and within 7.5e-4 for |x| <= 2,
    where the activations are small. The GPU parity tolerances carry the
    effect on the network."""
    import kernel_gelu as K
    e = K.coefficients16()
    assert all(float(np.float16(v)) == v for v in e)
    x = np.linspace(-30, 30, 600001)
    assert np.max(np.abs(K.gelu16(x) - C.gelu(x))) < 2.4e-4
    x = np.linspace(-10, 10, 400001)
    x16 = x.astype(np.float16).astype(np.float64)
    err = np.abs(K.gelu16_rounded(x16) - C.gelu(x16))
    assert err.max() < 1.3e-3
    assert err[np.abs(x16) <= 2].max() < 7.5e-4


def test_fp16_inference_rounding():
    """The inference kernel's roundings (FP16 weights, inputs and
    activations, the FP16 GELU) keep the network within 3e-3 relative L2 of
    the FP64 network with x Phi(x), for the initial weights and for weights
    twice as large, on standard-normal standardised inputs."""
    import kernel_gelu as K
    rng = np.random.default_rng(0)
    xs = rng.standard_normal((20000, 10))
    for scale in (1.0, 2.0):
        th = C.init_params(11) * scale
        ref = C.forward(th, xs)
        got = K.forward16_rounded(C.unpack, th, xs)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err < 3e-3, (scale, err)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    layers = (10, 8, 7, 6, 6)
    th = C.init_params(3, layers) * 3
    x = rng.standard_normal((5, 10))
    t = rng.standard_normal((5, 6))
    loss, g = C.loss_and_grad(th, x, t, layers)
    h = 1e-6
    idx = rng.choice(len(th), 60, replace=False)
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (C.loss_and_grad(th + e, x, t, layers)[0] - C.loss_and_grad(th - e, x, t, layers)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_full_network_shape_and_count():
    th = C.init_params(0)
    assert len(th) == C.n_params() == 9414
    y = C.forward(th, np.zeros((3, 10)))
    assert y.shape == (3, 6)
    lim = [1 / math.sqrt(a) for a in C.LAYERS[:-1]]
    parts = C.unpack(th)
    for l in range(4):
        assert np.all(np.abs(parts[2 * l]) <= lim[l]) and np.all(np.abs(parts[2 * l + 1]) <= lim[l])


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.02, 1e-3, -40.0])
    th, m, v = C.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-4)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_linear_network_reaches_least_squares():
    rng = np.random.default_rng(4)
    n, a, b = 512, 5, 3
    X = rng.standard_normal((n, a))
    Wt = rng.standard_normal((a, b))
    T = X @ Wt + 0.3 + 0.05 * rng.standard_normal((n, b))
    layers = (a, b)
    th0 = C.init_params(1, layers)
    th, m, v, losses = C.train(th0, X, T, steps=4000, batch=256, seed=9, lr=1e-2, layers=layers)
    A = np.hstack([X, np.ones((n, 1))])
    sol, *_ = np.linalg.lstsq(A, T, rcond=None)
    W, bias = C.unpack(th, layers)
    assert np.max(np.abs(W.T - sol[:a])) < 2e-2
    assert np.max(np.abs(bias - sol[a])) < 2e-2


def test_splitmix64_published_outputs():
    # first outputs of the reference generator seeded with 1234567
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [int(v) for v in C.splitmix64(1234567, np.arange(5, dtype=np.uint64))] == ref


def test_sampler_indices_in_range_and_spread():
    idx = C.sample_indices(7, 3, 65536, 1000)
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx.astype(np.int64), minlength=1000)
    assert counts.min() > 30 and counts.max() < 110
    assert not np.array_equal(idx, C.sample_indices(7, 4, 65536, 1000))


def test_moments():
    a = np.random.default_rng(0).standard_normal((2, 50, 4)) * np.array([1.0, 3.0])[:, None, None] + 2
    mu, sd = C.moments(a)
    assert np.allclose(mu, a.reshape(2, -1).mean(1)) and np.allclose(sd, a.reshape(2, -1).std(1))


def test_gradient_model_small_width_limit():
    """G is the leading term of the filtered stress: for a single smooth x
    mode and a narrow Gaussian, tau_11 / G_11 -> 1 (the oracle filter's
    exact stress, independent of the closure code)."""
    from oracle import filter_ref as R
    nx, ny, nz, lx, lz = 256, 9, 8, 2 * np.pi, 1.0
    y = synth.ygrid(ny, "uniform")
    x = np.arange(nx) * lx / nx
    u = np.zeros((3, nx, ny, nz))
    u[0] = np.sin(x)[:, None, None] * np.ones((1, ny, nz))
    ratios = []
    for d in (0.8, 0.4):
        ops = R.Operators(nx, ny, nz, lx, lz, y, d, 1e-3, 1e-3)
        ub, tau = R.sgs_stress(u, ops)
        feat = C.features(ub, y, lx, lz)
        g = C.gradient_model(feat, C.widths_coef(d, 1e-3, 1e-3))
        ratios.append(np.max(np.abs(tau[0] - g[0])) / np.max(np.abs(tau[0])))
    # relative remainder O(Delta^2): halves the width, quarters the remainder
    assert ratios[1] < 0.3 * ratios[0] and ratios[1] < 1e-2, ratios


def test_gradient_model_pairs_and_symmetry():
    rng = np.random.default_rng(2)
    feat = rng.standard_normal((10, 7))
    c = (0.3, 0.02, 0.1)
    g = C.gradient_model(feat, c)
    grad = feat[:9].reshape(3, 3, 7)            # [i][k][point]
    full = np.einsum("k,ikp,jkp->ijp", np.array(c), grad, grad)
    for q, (i, j) in enumerate(C.PAIRS):
        assert np.allclose(g[q], full[i, j]) and np.allclose(g[q], full[j, i])
    assert np.all(g[[0, 3, 5]] >= 0)            # positive semidefinite diagonal


def test_predict_and_targets_invert_each_other():
    rng = np.random.default_rng(3)
    feat = rng.standard_normal((10, 4, 5, 3))
    th = C.init_params(4)
    norms = np.concatenate([rng.standard_normal(10), rng.uniform(0.5, 2, 10),
                            rng.standard_normal(6), rng.uniform(0.5, 2, 6)])
    c = (0.1, 0.2, 0.05)
    tau = C.predict(th, feat, norms, c)
    t = C.standard_targets(tau, feat, norms, c)
    x = (feat.reshape(10, -1).T - norms[:10]) / norms[10:20]
    assert np.allclose(t, C.forward(th, x), atol=1e-12)
