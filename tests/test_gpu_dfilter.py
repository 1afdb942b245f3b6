"""GPU parity of the differential filter (Sec. 3, eq. (12)) through the C ABI
against the FP64 oracle (oracle.dfilter_ref).

Inputs are the seeded synthetic channel fields rounded to FP32; the oracle
evaluates the same rounded values in FP64. Tolerances: the filtered fields
to 2e-6 relative L2 (dense FP32 transforms of at most a few hundred terms
and a diagonally dominant tridiagonal solve), the stress per component to
max(1e-5, kappa (8 + 2 sqrt(nx/2) + 2 sqrt(nz/2)) 2^-24) with
kappa = |F(u_i' u_j')| / |tau_ij| (u1 shifted by its plane mean): the
rounding of the larger term carried into the difference, a folded forward
and inverse transform of n/2 terms each per periodic axis (rounding of a
K-term FP32 sum ~ sqrt(K) 2^-24) and a few products.
"""
import math

import numpy as np
import pytest

from oracle import dfilter_ref as D
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


GRIDS = [
    ("tiny", "tiny", dict()),
    ("min_sizes", "tiny", dict(nx=8, nz=9, ny=6, ykind="tanh", stretch=2.0)),
    ("odd_sizes", "tiny", dict(nx=10, nz=13, ny=21, ykind="tanh", stretch=2.0)),
    ("dns192_small", "dns192", dict(nx=40, nz=36, ny=33)),
    # long axes: several cosine tile groups, tables read from memory
    ("long_x", "tiny", dict(nx=270, nz=12, ny=9, lx=8.0)),
    ("long_z", "tiny", dict(nx=10, nz=300, ny=7, lz=9.0)),
    # 512 nodes: table slices of 112 / 128 KB staged in LDS where the device allows
    ("x512", "tiny", dict(nx=512, nz=16, ny=9, lx=16.0)),
]


@pytest.mark.parametrize("label,base,over", GRIDS)
def test_dfilter_fields_match_oracle(E, label, base, over):
    cfg = synth.config(base, **over)
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    rng = np.random.default_rng(21)
    par = [1, -1, 1, -1]
    v = rng.standard_normal((len(par), cfg.nx, cfg.ny, cfg.nz)).astype(np.float32) + 0.7
    for k, p in enumerate(par):
        if p < 0:
            v[k][:, [0, -1], :] = 0.0
    f = E.DFilter.from_config(cfg)
    out = _host(f.filter_fields(_dev(v), par))
    ops = D.DOperators.from_config(cfg)
    for k, p in enumerate(par):
        ref = D.dfilt(v[k].astype(np.float64), p, ops)
        err = R.rel_l2(out[k], ref, y)
        print(label, k, f"{err:.2e}", flush=True)
        assert err < 2e-6, (label, k, err)
        if p < 0:
            assert np.all(out[k][:, [0, -1], :] == 0.0)


def _tolerances(u, ops, tau):
    u = u.astype(np.float64)
    v = u.copy()
    v[0] -= R.plane_mean(u[0])[None, :, None]
    depth = 8 + 2 * math.sqrt(ops.nx / 2) + 2 * math.sqrt(ops.nz / 2)
    tol = []
    for k, (i, j) in enumerate(D.PAIRS):
        big = D.dfilt(v[i] * v[j], D.PARITY[i] * D.PARITY[j], ops)
        kappa = math.sqrt(np.sum(big ** 2) / np.sum(tau[k] ** 2))
        tol.append(max(1e-5, kappa * depth * 2.0 ** -24))
    return tol


SGS = [
    ("tiny", "tiny", dict(), 0),
    ("min_sizes", "tiny", dict(nx=8, nz=9, ny=6, ykind="tanh", stretch=2.0), 4),
    ("odd_sizes", "tiny", dict(nx=10, nz=13, ny=21, ykind="tanh", stretch=2.0), 1),
    ("dns192_small", "dns192", dict(nx=40, nz=36, ny=33), 2),
    ("long_xz", "tiny", dict(nx=264, nz=290, ny=7, lx=8.0, lz=9.0), 5),
    ("x512_z512", "tiny", dict(nx=512, nz=512, ny=5, lx=16.0, lz=16.0), 6),
    ("dns192", "dns192", dict(), 3),
]


@pytest.mark.parametrize("label,base,over,seed", SGS)
def test_dfilter_sgs_stress_matches_oracle(E, label, base, over, seed):
    cfg = synth.config(base, **over)
    y, u = synth.make_snapshot(cfg, seed)
    f = E.DFilter.from_config(cfg)
    ub, tau, st = [_host(t) for t in f.sgs_stress(_dev(u))]
    ops = D.DOperators.from_config(cfg)
    rub, rtau = D.sgs_stress(u.astype(np.float64), ops)
    tol = _tolerances(u, ops, rtau)
    for k in range(3):
        err = R.rel_l2(ub[k], rub[k], y)
        assert err < 1e-5, ("ubar", k, err)
    for k in range(6):
        err = R.rel_l2(tau[k], rtau[k], y)
        print(label, "tau", D.PAIRS[k], f"{err:.2e} (tol {tol[k]:.1e})", flush=True)
        assert err < tol[k], ("tau", k, err)
    # odd outputs vanish at the walls
    for q in (ub[1], tau[1], tau[4]):
        assert np.all(q[:, [0, -1], :] == 0.0)
    # FP64 plane statistics equal the plane means of the outputs
    mine = np.concatenate([R.plane_mean(ub), R.plane_mean(tau)])
    assert np.max(np.abs(st - mine)) < 1e-12 * (1 + np.abs(mine).max())


# ---- the inverse filter and the error measures (eqs. (11), (13)-(15))

@pytest.mark.parametrize("label,base,over", GRIDS)
def test_dfilter_inverse_matches_oracle(E, label, base, over):
    """u = (1 - a^2 lap) ubar against the oracle's operator. Its eigenvalues
    are >= 1, so the FP32 transform roundings stay a few 2^-24 sqrt(n) of
    the output: 2e-6 relative L2, as for the filter."""
    cfg = synth.config(base, **over)
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    rng = np.random.default_rng(31)
    par = [1, -1, 1]
    v = rng.standard_normal((len(par), cfg.nx, cfg.ny, cfg.nz)).astype(np.float32) - 0.3
    v[1][:, [0, -1], :] = 0.0
    f = E.DFilter.from_config(cfg)
    out = _host(f.inverse(_dev(v), par))
    ops = D.DOperators.from_config(cfg)
    for k, p in enumerate(par):
        ref = D.laplacian_apply(v[k].astype(np.float64), p, ops)
        err = R.rel_l2(out[k], ref, y)
        print(label, "inverse", k, f"{err:.2e}", flush=True)
        assert err < 2e-6, (label, k, err)
        if p < 0:
            assert np.all(out[k][:, [0, -1], :] == 0.0)


@pytest.mark.parametrize("label,base,over", GRIDS[:4] + [("dns192", "dns192", dict())])
def test_dfilter_round_trip_and_eq11(E, label, base, over):
    """inverse(filter(u)) = u on the GPU; with the eq. (7) parities the
    filtered u2 vanishes on the walls and the inverse returns the no-slip
    wall values (eq. (11)); with the eq. (9) parities ubar_2 does not."""
    cfg = synth.config(base, **over)
    y, u = synth.make_snapshot(cfg, 7)
    f = E.DFilter.from_config(cfg)
    du = _dev(u)
    ub = f.filter_fields(du, [1, -1, 1])
    back = _host(f.inverse(ub, [1, -1, 1]))
    # the inverse multiplies the FP32 rounding of ubar by up to the operator's
    # infinity norm 1 + a^2 (kx_max^2 + kz_max^2) + a^2 max_j sum |D_jk|
    # (large next to clustered wall nodes)
    ops = D.DOperators.from_config(cfg)
    lo, di, hi = D.second_difference(ops.y, 1)
    norm = 1.0 + ops.a ** 2 * (np.max(ops.k2) + np.max(np.abs(lo) + np.abs(di) + np.abs(hi)))
    for k in range(3):
        err = R.rel_l2(back[k], u[k], y)
        tol_k = max(2e-5, 8 * 2.0 ** -24 * norm)
        print(label, "round trip", k, f"{err:.2e} (tol {tol_k:.1e}, operator norm {norm:.0f})", flush=True)
        assert err < tol_k, (label, k, err)
    assert np.all(_host(ub)[1][:, [0, -1], :] == 0.0)
    tol = 32 * 2.0 ** -24 * norm * float(np.max(np.abs(_host(ub))))
    wall = float(np.max(np.abs(back[:, :, [0, -1], :])))
    print(label, f"wall {wall:.2e} (tol {tol:.1e})", flush=True)
    assert wall < tol
    bad = _host(f.filter_fields(du[1:2].clone(), [1]))[0]   # own allocation: 16-byte aligned
    rms = lambda a: float(np.sqrt(np.mean(a ** 2)))
    assert rms(bad[:, 0, :]) > 0.1 * rms(bad[:, 1, :])


@pytest.mark.parametrize("label,base,over", [GRIDS[0], GRIDS[2], ("dns192", "dns192", dict())])
def test_dfilter_errors_match_oracle(E, label, base, over):
    from oracle import metrics_ref as M
    cfg = synth.config(base, **over)
    y, u = synth.make_snapshot(cfg, 8)
    _, w = synth.make_snapshot(cfg, 9)
    les = (u + 0.05 * w).astype(np.float32)
    f = E.DFilter.from_config(cfg)
    got = _host(f.errors(_dev(les), _dev(u), 1.07, 1.0))
    ref = M.errors(les.astype(np.float64), u.astype(np.float64), 1.07, 1.0, y)
    print(label, "errors", got, ref, flush=True)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-10
    same = _host(f.errors(_dev(u), _dev(u), 1.0, 1.0))
    assert np.all(same == 0.0)


# ---- full size: an eigenmode of the operator (closed form at any size)

def _eigenmode(cfg, parity, nth):
    """phi(y) with D phi = lam phi for the reflected three-point difference of
    the given parity (numpy's eigen-solver on the ny x ny tridiagonal), the
    nth smoothest mode; odd: zero on the walls."""
    y = synth.ygrid(cfg.ny, cfg.ykind, cfg.stretch)
    lo, di, hi = D.second_difference(y, parity)
    m = len(di)
    A = np.diag(di) + np.diag(lo[1:], -1) + np.diag(hi[:-1], 1)
    lam, vec = np.linalg.eig(A)
    order = np.argsort(-lam.real)                     # smallest |lambda| first (lambda <= 0)
    k = order[nth]
    phi = np.real(vec[:, k])
    phi /= np.max(np.abs(phi))
    if parity < 0:
        phi = np.concatenate([[0.0], phi, [0.0]])
    return y, phi, float(lam[k].real)


@pytest.mark.parametrize("wl", ["dns512", "dns1024"])
@pytest.mark.parametrize("parity,nth,sx,sz", [(1, 3, 5, 2), (-1, 2, 3, 4)])
def test_dfilter_eigenmode_full_size(E, wl, parity, nth, sx, sz):
    """F(cos(kx x + kz z) phi(y)) = that / (1 + a^2 (kx^2 + kz^2) - a^2 lam), and the
    inverse multiplies by the same factor; the field is formed on the device.
    Tolerance of the filter: max(2e-6, 4 (sqrt(nx/2) + sqrt(nz/2)) 2^-24), the
    folded transforms' sum lengths. The inverse applies the operator to
    coefficients that carry FP32 rounding, which it amplifies by up to its
    infinity norm (large next to clustered wall nodes): 8 2^-24 ||A||."""
    import torch
    cfg = synth.config(wl)
    y, phi, lam = _eigenmode(cfg, parity, nth)
    a = 0.1
    kx, kz = 2 * math.pi * sx / cfg.lx, 2 * math.pi * sz / cfg.lz
    g = 1.0 + a * a * (kx * kx + kz * kz) - a * a * lam
    dev = torch.device("cuda")
    x = torch.arange(cfg.nx, device=dev, dtype=torch.float64) * (cfg.lx / cfg.nx)
    z = torch.arange(cfg.nz, device=dev, dtype=torch.float64) * (cfg.lz / cfg.nz)
    xz = torch.cos(kx * x[:, None] + kz * z[None, :] + 0.25)                 # [nx, nz]
    ph = torch.from_numpy(phi).to(dev)
    u = (xz[:, None, :] * ph[None, :, None]).to(torch.float32).unsqueeze(0).contiguous()
    f = E.DFilter.from_config(cfg)
    w = torch.from_numpy(R.trapezoid(y)).to(dev)[None, :, None]
    tol = max(2e-6, 4 * (math.sqrt(cfg.nx / 2) + math.sqrt(cfg.nz / 2)) * 2.0 ** -24)

    def rel(a_, b_):
        d = a_[0].double() - b_
        return math.sqrt(float((w * d * d).sum()) / float((w * b_ * b_).sum()))

    ops = D.DOperators.from_config(cfg)
    lo, di, hi = D.second_difference(ops.y, 1)
    norm = 1.0 + a * a * (np.max(ops.k2) + np.max(np.abs(lo) + np.abs(di) + np.abs(hi)))
    tol_inv = max(tol, 8 * 2.0 ** -24 * norm)
    out = f.filter_fields(u, [parity])
    e1 = rel(out, u[0].double() / g)
    back = f.inverse(u, [parity])
    e2 = rel(back, u[0].double() * g)
    print(wl, parity, f"filter {e1:.2e} (tol {tol:.1e}) inverse {e2:.2e} (tol {tol_inv:.1e}, "
          f"operator norm {norm:.0f})", flush=True)
    assert e1 < tol and e2 < tol_inv
    if parity < 0:
        assert float(out[0][:, [0, -1], :].abs().max()) == 0.0
    del out, back, u
    torch.cuda.empty_cache()


def test_dfilter_profile_pass_mask(E):
    """Timing the x forward transform alone leaves the other passes untimed
    and the outputs unchanged; an empty mask or a pass past the last is
    rejected."""
    cfg = synth.config("tiny", nx=24, nz=20, ny=17)
    y, u = synth.make_snapshot(cfg, 3)
    f = E.DFilter.from_config(cfg)
    du = _dev(u)
    ref = [_host(t) for t in f.sgs_stress(du)]
    E.dfilter_profile_begin(f.h, 2, passes=[E.DPASS_NAMES.index("x_fwd")])
    for _ in range(2):
        out = [_host(t) for t in f.sgs_stress(du)]
    prof = E.dfilter_profile_end(f.h)
    for p, q in zip(ref, out):
        assert np.array_equal(p, q)
    assert prof["x_fwd"][1] == 2 and prof["x_fwd"][0] > 0.0
    assert all(n == 0 for k, (ms, n) in prof.items() if k != "x_fwd")
    for mask in (0, 1 << E.DNPASS):
        assert E.lib.dfilter_profile_begin(f.h, 2, mask) == E.ELES_EINVAL
