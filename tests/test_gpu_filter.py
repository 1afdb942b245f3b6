"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are the seeded synthetic channel fields rounded to FP32; the oracle
evaluates the same rounded values in FP64. The tolerance of the FP32 path is
a relative volume-weighted L2 error of 1e-5 on every output; the operators
built on the device in FP64 must match the oracle's to 1e-14.
"""
import math

import numpy as np
import pytest

from oracle import filter_ref as R
from paper_1902_02508_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_02508_amd import eles
    return eles


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def fold(taps, n):
    m = (len(taps) - 1) // 2
    w = np.zeros(n)
    for t, v in enumerate(taps):
        w[(t - m) % n] += v
    return w


GRIDS = [
    # (name, cfg overrides / explicit geometry)
    ("tiny", dict()),
    ("dns192_small", dict(nx=40, nz=36)),
    ("odd", dict(nx=10, nz=13, ny=21, ykind="tanh", stretch=2.0)),
    ("cgl_wide", dict(nx=24, nz=40, ny=9, ykind="cgl", delta_y=0.6)),
]


def _cfg(name, over):
    base = "tiny" if name in ("tiny", "odd", "cgl_wide") else "dns192"
    return synth.config(base, **over)


@pytest.mark.parametrize("name,over", GRIDS)
@pytest.mark.parametrize("tail", [0.0, 1e-8])
def test_operators_match_oracle(E, name, over, tail):
    cfg = _cfg(name, over)
    f = E.Filter.from_config(cfg, tail_tol=tail)
    import torch
    torch.cuda.synchronize()
    ops = f.operators()
    ref = R.Operators.from_config(cfg, tail_tol=tail)
    assert np.max(np.abs(ops["wp"] - ref.wp)) < 1e-14
    assert np.max(np.abs(ops["wm"] - ref.wm)) < 1e-14
    assert np.max(np.abs(fold(ops["wx"], cfg.nx) - ref.wx)) < 1e-15
    assert np.max(np.abs(fold(ops["wz"], cfg.nz) - ref.wz)) < 1e-15
    assert np.array_equal(ops["y"], ref.y)


def _rel(a, b, y):
    return R.rel_l2(a, b, y)


@pytest.mark.parametrize("name,over", GRIDS)
@pytest.mark.parametrize("mode,tol", [("fp32", 2e-6), ("bf16x3", 2e-5), ("bf16", 2e-2)])
def test_filter_fields_match_oracle(E, name, over, mode, tol):
    cfg = _cfg(name, over)
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    rng = np.random.default_rng(11)
    nf = 5
    v = rng.standard_normal((nf, cfg.nx, cfg.ny, cfg.nz)).astype(np.float32) + 1.5
    par = [1, -1, -1, 1, -1]
    f = E.Filter.from_config(cfg, ygemm=mode)
    out = _host(f.filter_fields(_dev(v), par))
    ops = R.Operators.from_config(cfg)
    for k in range(nf):
        ref = R.filt(v[k].astype(np.float64), par[k], ops)
        err = _rel(out[k], ref, y)
        assert err < tol, (k, err)


def _sgs_case(E, cfg, seed, tail=0.0, mode="fp32", xz=None):
    y, u = synth.make_snapshot(cfg, seed)
    f = E.Filter.from_config(cfg, tail_tol=tail, ygemm=mode)
    if xz is not None:
        f.set_xz(xz == "matrix")
    ub, tau, st = f.sgs_stress(_dev(u))
    return y, u, _host(ub), _host(tau), _host(st), f


# (label, base config, overrides, seed, y-pass route): "staged" is the
# LDS-staged persistent kernel, "direct" the one it falls back to when a
# row group does not fit in LDS (here: a y filter as wide as the channel).
SGS_CASES = [
    ("tiny", "tiny", dict(), 0, "staged"),
    ("odd", "tiny", dict(nx=10, nz=13, ny=21, ykind="tanh", stretch=2.0), 1, "staged"),
    ("ragged192", "dns192", dict(nx=27, nz=70, ny=37), 2, "staged"),
    ("strip36", "dns192", dict(nx=20, nz=36, ny=65), 3, "staged"),
    ("wide_y", "tiny", dict(nx=12, nz=16, ny=193, delta_y=1.0), 4, "direct"),
]


def fp32_tolerances(u, ops, y):
    """Per-component tolerance of an FP32 evaluation of tau_ij.

    tau_ij is the difference of F(u_i' u_j') and F(u_i') F(u_j') (u1 shifted
    by its plane mean); each of the few FP32 roundings on the way perturbs
    the larger term by about 2^-24 of its size, so the relative error of
    tau_ij is bounded by a small multiple of kappa_ij 2^-24 with
    kappa_ij = |F(u_i' u_j')| / |tau_ij|. The bound used is
    max(1e-5, 8 kappa_ij 2^-24).
    """
    u = u.astype(np.float64)
    v = u.copy()
    v[0] -= R.plane_mean(u[0])[None, :, None]
    _, tau = R.sgs_stress(u, ops)
    tol = []
    for k, (i, j) in enumerate(R.PAIRS):
        big = R.filt(v[i] * v[j], R.PARITY[i] * R.PARITY[j], ops)
        kappa = math.sqrt(np.sum(big ** 2) / np.sum(tau[k] ** 2))
        tol.append(max(1e-5, 8 * kappa * 2.0 ** -24))
    return tol


@pytest.mark.parametrize("label,base,over,seed,route", SGS_CASES)
@pytest.mark.parametrize("xz", ["matrix", "vector"])
def test_sgs_stress_matches_oracle(E, label, base, over, seed, route, xz):
    """Both x/z routes: the matrix-core kernel (run with the 1e-8 tail cut,
    which brings every case's stencils within its half-width limit) and the
    vector-unit kernel (full kernel)."""
    cfg = synth.config(base, **over)
    tail = 1e-8 if xz == "matrix" else 0.0
    y, u, ub, tau, st, f = _sgs_case(E, cfg, seed, tail, xz=xz)
    groups = f.layout.y_groups
    assert (groups > 0) == (route == "staged"), (label, groups)
    if groups:
        assert f.layout.y_blocks % groups == 0 and f.layout.y_blocks >= groups
    if xz == "matrix":
        assert f.layout.xz_waves > 0, label
    ops = R.Operators.from_config(cfg, tail_tol=tail)
    rub, rtau = R.sgs_stress(u.astype(np.float64), ops)
    tol = fp32_tolerances(u, ops, y)
    for k in range(3):
        assert _rel(ub[k], rub[k], y) < 1e-5, ("ubar", k)
    for k in range(6):
        err = _rel(tau[k], rtau[k], y)
        print(label, "tau", R.PAIRS[k], f"{err:.2e} (tol {tol[k]:.1e})", flush=True)
        assert err < tol[k], ("tau", k, err)
    # plane statistics: the library's FP64 sums of its own outputs ...
    mine = np.concatenate([R.plane_mean(ub), R.plane_mean(tau)])
    assert np.max(np.abs(st - mine)) < 1e-12 * (1 + np.abs(mine).max())
    # ... and the profiles against the oracle's
    check_profiles(u, ops, y, st, rub, rtau)


def profile_tolerances(u, ops, y):
    """Tolerance of the eq. (14)-form error of each <tau_ij>(y). The rounding
    argument of fp32_tolerances applied to plane means: every output point
    carries an error of about 2^-24 |F(u_i' u_j')|, and its plane mean is at
    most the plane's rms of that, so the bound is max(1e-5, 8 kp_ij 2^-24)
    with kp_ij = |rms_xz F(u_i' u_j')| / |<tau_ij>| (profile norms)."""
    u = u.astype(np.float64)
    v = u.copy()
    v[0] -= R.plane_mean(u[0])[None, :, None]
    _, tau = R.sgs_stress(u, ops)
    tol = []
    w = R.trapezoid(y)
    for k, (i, j) in enumerate(R.PAIRS):
        big = R.filt(v[i] * v[j], R.PARITY[i] * R.PARITY[j], ops)
        big_rms = np.sqrt(R.plane_mean(big ** 2))
        ref = R.plane_mean(tau[k])
        kp = math.sqrt(np.sum(w * big_rms ** 2) / np.sum(w * ref ** 2))
        tol.append(max(1e-5, 8 * kp * 2.0 ** -24))
    return tol


def check_profiles(u, ops, y, st, rub, rtau):
    """Every plane-mean profile of the library against the oracle's. <ubar_1>
    and the six <tau_ij> in the eq. (14) form (Sec. 4.1) within
    profile_tolerances; <ubar_2> and <ubar_3> vanish for the generator's
    fields (zero-mean modes), so they are compared absolutely, within 1e-6
    of the field's rms."""
    ptol = profile_tolerances(u, ops, y)
    e = R.profile_error(st[0], R.plane_mean(rub[0]), y)
    assert e < 1e-5, ("<ubar_1>", e)
    for k in (1, 2):
        rms = math.sqrt(np.mean(rub[k] ** 2))
        assert np.max(np.abs(st[k] - R.plane_mean(rub[k]))) < 1e-6 * rms, ("<ubar>", k)
    for k in range(6):
        e = R.profile_error(st[3 + k], R.plane_mean(rtau[k]), y)
        print("profile tau", R.PAIRS[k], f"{e:.2e} (tol {ptol[k]:.1e})", flush=True)
        assert e < ptol[k], ("<tau>", R.PAIRS[k], e, ptol[k])


# Wide stencils (x/z half-widths above 16): the matrix-core wide kernel
# (three of the nine fields per wave, z windows of up to seven 16-column
# chunks) and the vector-unit x/z pass.
# Boxes shrunk with the grid so that the widths keep their size in grid
# steps: sigma/dx = 2.31 as at 192 x 129 x 192 (half-widths 20, z window of
# five chunks), and 6.2 as at 1024 x 385 x 768 (half-widths 37, seven chunks).
WIDE_CASES = [
    # label, base, overrides, seed, tail
    ("h2", "dns192", dict(nx=40, nz=48, ny=33, lx=4 * math.pi * 40 / 192, lz=2 * math.pi * 48 / 192), 5, 0.0),
    ("h3", "dns192", dict(nx=40, nz=64, ny=17, lx=40 * 0.151 / 6.2, lz=64 * 0.0756 / 6.2), 6, 1e-8),
    ("ragged_x", "dns192", dict(nx=27, nz=36, ny=21, lx=4 * math.pi * 27 / 192, lz=2 * math.pi * 36 / 192), 7,
     0.0),
]


@pytest.mark.parametrize("label,base,over,seed,tail", WIDE_CASES)
@pytest.mark.parametrize("xz", ["matrix", "vector"])
def test_sgs_wide_stencils(E, label, base, over, seed, tail, xz):
    cfg = synth.config(base, **over)
    y, u, ub, tau, st, f = _sgs_case(E, cfg, seed, tail, xz=xz)
    assert min(f.layout.mx, f.layout.mz) > 16, (label, f.layout.mx, f.layout.mz)
    assert f.layout.xz_waves > 0 and f.layout.xz_wide == 1, label
    ops = R.Operators.from_config(cfg, tail_tol=tail)
    rub, rtau = R.sgs_stress(u.astype(np.float64), ops)
    tol = fp32_tolerances(u, ops, y)
    for k in range(3):
        assert _rel(ub[k], rub[k], y) < 1e-5, ("ubar", k)
    for k in range(6):
        err = _rel(tau[k], rtau[k], y)
        print(label, f"m=({f.layout.mx},{f.layout.mz})", "tau", R.PAIRS[k], f"{err:.2e} (tol {tol[k]:.1e})",
              flush=True)
        assert err < tol[k], ("tau", k, err)
    check_profiles(u, ops, y, st, rub, rtau)


def test_sgs_dns192_full_size(E):
    """The 192 x 129 x 192 channel at its own widths, FP32 path, seeds 0-1,
    with the full kernel and with the 1e-8 tail cut the benchmark uses (both
    x/z routes)."""
    cfg = synth.config("dns192")
    ops = R.Operators.from_config(cfg)
    for seed, tail, xz in ((0, 0.0, None), (1, 1e-8, "matrix"), (1, 1e-8, "vector")):
        y, u, ub, tau, st, f = _sgs_case(E, cfg, seed, tail, xz=xz)
        if xz == "matrix":
            assert f.layout.xz_waves > 0
        rub, rtau = R.sgs_stress(u.astype(np.float64), ops)
        errs = [_rel(ub[k], rub[k], y) for k in range(3)] + [_rel(tau[k], rtau[k], y) for k in range(6)]
        print(f"seed {seed} tail {tail} x/z {xz}: max rel L2 {max(errs):.2e}", flush=True)
        assert max(errs) < 1e-5, errs
        ref12 = R.plane_mean(rtau[1])
        assert R.profile_error(st[4], ref12, y) < 1e-5
        if seed == 0:
            check_profiles(u, ops, y, st, rub, rtau)


def test_sgs_deterministic_and_invariants(E):
    cfg = synth.config("dns192", nx=48, nz=64)
    y, u = synth.make_snapshot(cfg, 5)
    f = E.Filter.from_config(cfg)
    du = _dev(u)
    a = [_host(t) for t in f.sgs_stress(du)]
    b = [_host(t) for t in f.sgs_stress(du)]
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
    ub, tau, st = a
    scale = np.abs(u).max() ** 2
    # odd components vanish at the walls (eqs. (8), (11))
    assert np.max(np.abs(ub[1][:, [0, -1]])) < 1e-12
    assert np.max(np.abs(tau[1][:, [0, -1]])) < 1e-10 * scale
    assert np.max(np.abs(tau[4][:, [0, -1]])) < 1e-10 * scale
    # realizability: trace and diagonal non-negative up to FP32 noise
    tr = tau[0] + tau[3] + tau[5]
    assert tr.min() > -1e-6 * scale


def test_two_handles_on_two_streams_match_one_stream(E):
    """Snapshots alternating between two streams, each with a filter handle
    of its own, give outputs bitwise equal to one handle on one stream (the
    handles share no state; each snapshot's buffers stay on one stream)."""
    import torch
    cfg = synth.config("dns192", nx=48, nz=64)
    us = [_dev(synth.make_snapshot(cfg, s)[1]) for s in (5, 6, 7, 8)]
    fa = E.Filter.from_config(cfg, tail_tol=1e-8)
    fb = E.Filter.from_config(cfg, tail_tol=1e-8)
    ref = [[_host(t) for t in fa.sgs_stress(u)] for u in us]
    outs = [[torch.empty((3,) + fa.shape, device="cuda"), torch.empty((6,) + fa.shape, device="cuda"),
             torch.empty((9, cfg.ny), dtype=torch.float64, device="cuda")] for _ in us]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for rep in range(3):
        for k, u in enumerate(us):
            with torch.cuda.stream(streams[k % 2]):
                (fa, fb)[k % 2].sgs_stress(u, *outs[k])
    torch.cuda.synchronize()
    for k in range(len(us)):
        for got, want in zip(outs[k], ref[k]):
            assert np.array_equal(_host(got), want), k


@pytest.mark.parametrize("mode", ["bf16x3", "bf16"])
def test_sgs_reduced_precision_y_pass(E, mode):
    """The reduced-precision y arithmetics on the full 192 x 129 x 192
    channel (the benchmark grid). The BF16x3 split holds each operand to
    2^-16 relative (two BF16 of 8 significant bits each) instead of FP32's
    2^-24, so the FP32 rule max(1e-5, 8 kappa 2^-24) becomes
    max(2e-5, kappa_ij 2^-16); the 2e-5 target itself is checked on the
    512 x 257 x 512 and 1024 x 385 x 768 configurations, where BF16x3 is the
    configured arithmetic. Plain BF16 (8 bits) is reported, within 5e-2."""
    cfg = synth.config("dns192")
    y, u, ub, tau, st, _ = _sgs_case(E, cfg, 0, mode=mode)
    ops = R.Operators.from_config(cfg)
    rub, rtau = R.sgs_stress(u.astype(np.float64), ops)
    errs = [_rel(ub[k], rub[k], y) for k in range(3)] + [_rel(tau[k], rtau[k], y) for k in range(6)]
    print(mode, " ".join(f"{e:.2e}" for e in errs), flush=True)
    if mode == "bf16":
        assert max(errs) < 5e-2
        return
    u64 = u.astype(np.float64)
    v = u64.copy()
    v[0] -= R.plane_mean(u64[0])[None, :, None]
    for k in range(3):
        assert errs[k] < 2e-5, ("ubar", k, errs[k])
    for k, (i, j) in enumerate(R.PAIRS):
        big = R.filt(v[i] * v[j], R.PARITY[i] * R.PARITY[j], ops)
        kap = math.sqrt(np.sum(big ** 2) / np.sum(rtau[k] ** 2))
        tol = max(2e-5, kap * 2.0 ** -16)
        print("bf16x3 tau", R.PAIRS[k], f"{errs[3 + k]:.2e} (kappa {kap:.1f}, tol {tol:.1e})", flush=True)
        assert errs[3 + k] < tol, ("tau", R.PAIRS[k], errs[3 + k], tol)


def test_profile_pass_mask_times_only_the_selected_passes(E):
    """Timing one pass leaves the others untimed and the outputs unchanged;
    an empty mask or a pass past the last is rejected."""
    cfg = synth.config("dns192", nx=48, nz=64)
    y, u = synth.make_snapshot(cfg, 6)
    f = E.Filter.from_config(cfg)
    du = _dev(u)
    ref = [_host(t) for t in f.sgs_stress(du)]
    E.filter_profile_begin(f.h, 3, passes=[E.PASS_NAMES.index("y")])
    for _ in range(3):
        out = [_host(t) for t in f.sgs_stress(du)]
    prof = E.filter_profile_end(f.h)
    for p, q in zip(ref, out):
        assert np.array_equal(p, q)
    assert prof["y"][1] == 3 and prof["y"][0] > 0.0
    assert all(n == 0 for k, (ms, n) in prof.items() if k != "y")
    for mask in (0, 1 << E.NPASS):
        assert E.lib.filter_profile_begin(f.h, 3, mask) == E.ELES_EINVAL
