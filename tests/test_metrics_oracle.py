"""Pins of the FP64 oracle of the error measures, eqs. (13)-(15).

Each test checks the oracle against something other than itself: closed
forms of scaled or shifted fields, numpy's trapezoid rule, the rms of a
sinusoid, and the norms of oracle.filter_ref (pinned in test_oracle_pins).
"""
import math

import numpy as np
import pytest

from oracle import filter_ref as R
from oracle import metrics_ref as E
from paper_1902_02508_amd import synth


def _fields(seed=0, nx=12, ny=17, nz=10):
    cfg = synth.config("tiny", nx=nx, ny=ny, nz=nz)
    y, u = synth.make_snapshot(cfg, seed)
    return y, u.astype(np.float64)


def test_identical_fields_and_friction_scaling_give_zero():
    y, u = _fields()
    assert np.all(E.errors(u, u, 1.0, 1.0, y) == 0.0)
    # the same normalised field: les = dns * (utau_les / utau_dns)
    err = E.errors(u * 1.7, u, 1.7, 1.0, y)
    assert np.max(np.abs(err)) < 1e-14


@pytest.mark.parametrize("eps", [1e-3, -0.2])
def test_uniform_scaling_closed_form(eps):
    """les = (1 + eps) dns, equal friction velocities: every error is |eps|
    (means and rms scale by 1 + eps)."""
    y, u = _fields(1)
    err = E.errors((1 + eps) * u, u, 1.0, 1.0, y)
    assert np.max(np.abs(err - abs(eps))) < 1e-12


def test_trapezoid_weights_match_numpy():
    y = synth.ygrid(21, "tanh", 2.0)
    f = np.cos(3 * y) + y ** 2
    assert abs(np.sum(E.trapezoid_weights(y) * f) - np.trapezoid(f, y)) < 1e-14


def test_mean_profile_offset_closed_form():
    """u1 = U(y) with no fluctuation, les1 = U + c: the eq. (14) error is
    c [int_{-1}^0 1]^(1/2) / [int_{-1}^0 U^2]^(1/2), trapezoid rule on the
    lower-half nodes (numpy's)."""
    nx, ny, nz = 6, 33, 4
    y = synth.ygrid(ny, "cgl", 0.0)
    U = 1.0 - y ** 2
    dns = np.zeros((3, nx, ny, nz))
    dns[0] = U[None, :, None]
    x = np.arange(nx) / nx
    dns[1] = dns[2] = np.sin(2 * math.pi * x)[:, None, None]   # nonzero intensities
    les = dns.copy()
    c = 0.05
    les[0] += c
    k = y <= 0.0
    ref = c * math.sqrt(np.trapezoid(np.ones(k.sum()), y[k])) / math.sqrt(np.trapezoid(U[k] ** 2, y[k]))
    assert abs(E.errors(les, dns, 1.0, 1.0, y)[1] - ref) < 1e-13


def test_rms_of_a_sinusoid():
    """u2 = A(y) sin(2 pi x / L) on a periodic grid: rms = A / sqrt(2)."""
    nx, ny, nz = 16, 9, 3
    y = np.linspace(-1, 1, ny)
    A = 1.0 + y ** 2
    x = np.arange(nx) / nx
    f = A[None, :, None] * np.sin(2 * math.pi * x)[:, None, None] * np.ones((1, 1, nz))
    assert np.max(np.abs(E.plane_rms(f) - A / math.sqrt(2))) < 1e-14


def test_agrees_with_the_pinned_norms():
    y, u = _fields(2)
    _, v = _fields(3)
    les = u + 0.1 * v
    err = E.errors(les, u, 1.3, 1.1, y)
    assert abs(err[0] - R.rel_l2(les[0] / 1.3, u[0] / 1.1, y)) < 1e-13
    assert abs(err[1] - R.profile_error(R.plane_mean(les[0]) / 1.3, R.plane_mean(u[0]) / 1.1, y, half=True)) < 1e-13


def test_planted_rms_without_mean_removal_is_caught():
    """An rms that forgets to subtract the mean differs from the intensity
    by far more than rounding on a field with a mean profile."""
    y, u = _fields(4)
    f = u[0] + 5.0
    wrong = np.sqrt((f ** 2).mean(axis=(0, 2)))
    assert np.max(np.abs(wrong - E.plane_rms(f))) > 1.0
