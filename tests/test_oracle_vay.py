"""Pins of the FP64 reference of Vay's pusher (the relativistic correction
to the Boris push the paper cites, Sec. 3.3).

The pusher is defined by the implicit, time-centred momentum equation
u^{n+1/2} - u^{n-1/2} = (q dt / m) (E + (v^{n+1/2} + v^{n-1/2})/2 x B);
the reference solves it in closed form.  Pins: the defining equation holds
for the result (residual at FP64 rounding, random inputs); a pure electric
field gives the exact impulse; a pure magnetic field keeps |u| and turns u
by the Boris angle 2 atan(|q| B dt / (2 gamma m)) (the two pushers coincide
there); a particle at the E x B drift velocity of crossed fields feels no
force (the property the correction exists for; the Boris push does not
have it); Boris and Vay agree to third order in dt for one step.
"""

import numpy as np
import pytest

import synth
from oracle.pic import boris, vay

C = 299792458.0
QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS


def _cross(a, b):
    # right-handed basis (rho, phi, z)
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _gamma(u):
    return np.sqrt(1.0 + u @ u / C ** 2)


def test_vay_solves_its_defining_equation():
    rng = np.random.default_rng(3)
    for _ in range(200):
        u0 = rng.normal(size=3) * 10.0 ** rng.uniform(5, 9.5)
        E = rng.normal(size=3) * 10.0 ** rng.uniform(3, 8)
        B = rng.normal(size=3) * 10.0 ** rng.uniform(-2, 1)
        k = QE / ME * 10.0 ** rng.uniform(-14, -11.5) / 2
        u1 = vay(u0, E, B, k)
        v0, v1 = u0 / _gamma(u0), u1 / _gamma(u1)
        rhs = 2 * k * (E + _cross(0.5 * (v0 + v1), B))
        scale = np.abs(u0).max() + np.abs(u1).max() + np.abs(rhs).max()
        assert np.abs((u1 - u0) - rhs).max() <= 1e-13 * scale


def test_vay_uniform_electric_field():
    u0 = np.array([1.0e7, -2.0e6, 3.0e7])
    E = np.array([4.0e5, 0.0, -7.0e5])
    k = QE / ME * 1e-13 / 2
    np.testing.assert_allclose(vay(u0, E, np.zeros(3), k), u0 + 2 * k * E, rtol=1e-14)


def test_vay_uniform_magnetic_rotation():
    u0 = np.array([2.0e8, 1.0e8, 5.0e7])
    B = np.array([0.0, 0.0, 1.5])
    dt = 2e-12
    g = _gamma(u0)
    u1 = vay(u0, np.zeros(3), B, QE / ME * dt / 2)
    assert np.linalg.norm(u1) == pytest.approx(np.linalg.norm(u0), rel=1e-14)
    ang = np.arctan2(u0[0] * u1[1] - u0[1] * u1[0], u0[0] * u1[0] + u0[1] * u1[1])
    assert abs(ang) == pytest.approx(2 * np.arctan(abs(QE) * 1.5 * dt / (2 * g * ME)), rel=1e-12)
    assert u1[2] == pytest.approx(u0[2], rel=1e-14)


@pytest.mark.parametrize("beta_d", [0.1, 0.9, 0.99])
def test_vay_exb_drift_is_force_free(beta_d):
    """E = E_rho rho-hat, B = B_z z-hat, v = E x B / B^2 = -(E_rho / B_z) phi-hat:
    E + v x B = 0, so u must not change; the Boris push changes it (by more
    as the drift becomes relativistic)."""
    Bz = 1.0
    Er = beta_d * C * Bz
    E = np.array([Er, 0.0, 0.0])
    B = np.array([0.0, 0.0, Bz])
    v = _cross(E, B) / Bz ** 2
    np.testing.assert_allclose(E + _cross(v, B), 0.0, atol=1e-9 * Er)
    u0 = v / np.sqrt(1.0 - v @ v / C ** 2)
    k = QE / ME * 1e-12 / 2
    uv = vay(u0, E, B, k)
    ub = boris(u0, E, B, k)
    assert np.abs(uv - u0).max() <= 1e-12 * np.abs(u0).max()
    assert np.abs(ub - u0).max() > 1e3 * np.abs(uv - u0).max()


def test_boris_and_vay_agree_to_third_order():
    u0 = np.array([1.0e8, 2.0e8, -1.5e8])
    E = np.array([3.0e6, 1.0e6, -2.0e6])
    B = np.array([0.3, 0.7, 1.1])
    diffs = []
    for dt in (4e-13, 2e-13, 1e-13):
        k = QE / ME * dt / 2
        diffs.append(np.linalg.norm(vay(u0, E, B, k) - boris(u0, E, B, k)))
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 7.0 < r1 < 9.0 and 7.0 < r2 < 9.0
