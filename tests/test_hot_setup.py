"""Host-side pieces of the BWO hot test (CPU): the beam-wave synchronism
against closed forms, and the emitting annulus of the tube mesh."""

import numpy as np

from paper_1701_03784_amd import bwo_hot_test as hot

C = 299792458.0


def test_synchronism_of_a_flat_band_is_the_band():
    v, d, F = 0.86 * C, 0.0167, 9.0e9
    assert abs(hot.synchronism([F] * 5, d, v) / F - 1) < 1e-12


def test_synchronism_of_a_linear_band():
    """Band a + b psi (psi in [0, pi]) mirrored into (pi, 2 pi) meets the beam
    line k phi (k = v / (2 pi d)) at phi* = (a + 2 pi b) / (k + b)."""
    v, d = 0.86 * C, 0.0167
    a, b = 7.5e9, 0.8e9
    k = v / (2 * np.pi * d)
    psi = np.linspace(0.0, np.pi, 9)
    phi = (a + 2 * np.pi * b) / (k + b)
    assert np.pi < phi < 2 * np.pi
    assert abs(hot.synchronism(a + b * psi, d, v) / (k * phi) - 1) < 1e-9


def test_no_synchronism_when_the_beam_is_too_slow():
    assert hot.synchronism([20e9] * 5, 0.0167, 0.1 * C) is None


def test_tube_emitter_is_the_annulus_on_the_cathode_plate():
    m, L = hot.tube_mesh(0.5e-3)
    em = m.seg[m.tag == 3]
    assert len(em) > 0
    p = m.nodes[em]
    assert np.all(p[..., 0] == 0.0)
    assert p[..., 1].min() >= 0.009 - 0.5e-3 and p[..., 1].max() <= 0.011 + 0.5e-3
    assert np.all(m.signed_areas() > 0)
    assert abs(L - m.nodes[:, 0].max()) < 1e-12
