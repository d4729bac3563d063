"""Pins of the FP64 emission (continuous injection) reference.

SplitMix64 against the reference outputs of its published generator;
emission uniform per unit area of a disk emitter (rho^2 uniform, a
closed-form property of the sampling); charge conservation at emission;
momentum frame on a z = 0 cathode.
"""

import numpy as np
import pytest

import synth
from synth import configs
from oracle.inject import Emitter, splitmix64


def test_splitmix64_reference_outputs():
    # first five outputs of SplitMix64 seeded with 1234567 (reference implementation)
    out = splitmix64(1234567, np.arange(1, 6, dtype=np.uint64))
    assert [int(v) for v in out] == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                     4593380528125082431, 16408922859458223821]


@pytest.fixture(scope="module")
def diode():
    from oracle.pic import OracleSim
    m = configs.diode_mesh(h=1.0e-3)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    return m, sim


def test_emission_is_uniform_per_area(diode):
    m, sim = diode
    em = Emitter(sim.topo)
    R = max(em.rb.max(), em.ra.max())
    rho = np.concatenate([em.emit(n, 20000, 11, np.zeros(3), 0.0)[1] for n in range(10)])
    x = np.sort((rho / R) ** 2)
    ks = np.abs(x - (np.arange(1, len(x) + 1) / len(x))).max()
    assert ks < 0.01                     # Kolmogorov-Smirnov distance, 2e5 samples
    z = np.concatenate([em.emit(n, 1000, 11, np.zeros(3), 0.0)[0] for n in range(3)])
    assert np.all(z == 0.0)


def test_emission_conserves_nodal_charge_and_sets_momentum(diode):
    from oracle.pic import OracleSim
    m, _ = diode
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    sp = sim.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 1000)
    um = np.array([0.0, 0.0, 5.9e5])
    sim.set_injector(sp, 500, um, 1.0e5, seed=3)
    Q0 = sim.charge()
    sim._inject_step()
    Q1 = sim.charge()
    assert np.abs(Q1 - Q0).max() <= 1e-12 * np.abs(sim.sp_qw[sp] / (2 * np.pi))
    zr, u, _ = sim.particles()
    assert len(zr) == 500
    # cathode at z = 0: inward normal +z, tangent along rho
    assert np.all(np.abs(u[:, 2] - um[2]) <= 1.0e5 * (1 + 1e-12))
    assert np.all(np.abs(u[:, 0]) <= 1.0e5 * (1 + 1e-12))
    assert abs(u[:, 2].mean() - um[2]) < 0.1 * 1.0e5
