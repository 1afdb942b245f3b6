"""GPU parity of the LES-grid stress and the commutation error through the C
ABI against the FP64 oracle (oracle.les_ref).

Inputs are seeded synthetic stand-ins for the DNS-grid filtered velocity
and stress (the synthetic channel velocity for ubar, products of its
components for tau), rounded to FP32; the oracle evaluates the same values
in FP64. T_ij on the LES grid: relative L2 <= 1e-6 (a few FP32 roundings of
eight-term weighted sums); the commutation error (FP64 sums with the
interpolation weights stored in FP32, exact where LES and DNS nodes
coincide): 1e-6 relative; LES = DNS grid: T equals tau exactly.
"""
import numpy as np
import pytest

from oracle import filter_ref as R
from oracle import les_ref as L
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


def _inputs(cfg, seed):
    y, u = synth.make_snapshot(cfg, seed)
    ub = u.astype(np.float32)
    tau = np.stack([(u[i] * u[j] - 0.3 * u[i]) for i, j in L.PAIRS]).astype(np.float32)
    return y, ub, tau


CASES = [
    # label, base config, overrides, LES grid: (nx_les, y_les builder, nz_les)
    ("tiny_les2", "tiny", dict(), "ratio2"),
    ("between", "tiny", dict(nx=10, nz=13, ny=21, ykind="tanh", stretch=2.0), "between"),
    ("identity", "tiny", dict(nx=12, nz=10, ny=17), "identity"),
    ("dns192_les2", "dns192", dict(), "ratio2"),
    ("dns192_les4", "dns192", dict(), "ratio4"),
]


def _les_grid(cfg, y, kind):
    if kind == "identity":
        return cfg.nx, y, cfg.nz
    if kind == "between":
        return 7, np.linspace(-1.0, 1.0, 9), 5
    r = 2 if kind == "ratio2" else 4
    return cfg.nx // r, synth.ygrid((cfg.ny - 1) // r + 1, cfg.ykind, cfg.stretch), cfg.nz // r


@pytest.mark.parametrize("label,base,over,kind", CASES)
def test_les_stress_matches_oracle(E, label, base, over, kind):
    cfg = synth.config(base, **over)
    y, ub, tau = _inputs(cfg, 11)
    nxl, yl, nzl = _les_grid(cfg, y, kind)
    g = E.LesGrid(cfg.nx, cfg.ny, cfg.nz, y, nxl, len(yl), nzl, yl)
    ul, T = [_host(t) for t in g.stress(_dev(ub), _dev(tau))]
    I = L.Interp(cfg.nx, cfg.ny, cfg.nz, y, nxl, nzl, yl)
    ub64, tau64 = ub.astype(np.float64), tau.astype(np.float64)
    fuu = np.stack([tau64[k] + ub64[i] * ub64[j] for k, (i, j) in enumerate(L.PAIRS)])
    rul, rT = L.les_stress(ub64, fuu, I)
    for k in range(3):
        err = R.rel_l2(ul[k], rul[k], yl)
        assert err < 1e-6, ("ubar", k, err)
    for k in range(6):
        err = R.rel_l2(T[k], rT[k], yl)
        print(label, "T", L.PAIRS[k], f"{err:.2e}", flush=True)
        assert err < 1e-6, ("T", k, err)
    if kind == "identity":
        assert np.all(T == tau64) and np.all(ul == ub64)


@pytest.mark.parametrize("label,base,over,kind", CASES)
def test_les_commutation_matches_oracle(E, label, base, over, kind):
    cfg = synth.config(base, **over)
    y, ub, tau = _inputs(cfg, 12)
    nxl, yl, nzl = _les_grid(cfg, y, kind)
    g = E.LesGrid(cfg.nx, cfg.ny, cfg.nz, y, nxl, len(yl), nzl, yl)
    I = L.Interp(cfg.nx, cfg.ny, cfg.nz, y, nxl, nzl, yl)
    for name, field in (("ubar1", ub[0]), ("tau12", tau[1])):
        got = float(_host(g.commutation(_dev(field)))[0])
        ref = L.commutation_error(field.astype(np.float64), I)
        print(label, "commutation", name, got, ref, flush=True)
        assert abs(got - ref) <= 1e-6 * abs(ref), (name, got, ref)
