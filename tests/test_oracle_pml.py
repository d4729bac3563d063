"""Pins of the FP64 stretched-coordinate absorbing layer (the PML of the
ports and cathode side, Sec. 5.1).

The layer stretches z by s_z = 1 + sigma / (j omega eps0): eps_rho = eps0 s_z,
eps_z = eps0 / s_z, mu_phi = mu0 s_z, with auxiliary face and edge
variables integrated by the trapezoidal rule.  Pins: the z and rho parts
of the local Hodge add up to it and a uniform axial field has energy only
in the z part (eps0 E_z^2 int rho dA, a closed form); a vanishing
conductivity reproduces the scheme without the layer; a TM01 pulse in a
circular guide (R = 1 cm, 20 GHz) that meets a 2 cm layer comes back at
below 1e-3 of its amplitude, where a conductor end returns all of it; and
after the pulse the fields in the layered guide fall below 1e-2 of their
peak and do not grow over 30,000 steps (what remains is the cutoff mode,
uniform in z, which no z-stretching can absorb).
"""

import numpy as np
import pytest

import synth
from oracle.hodge import EPS0, hodge_eps, pml_parts
from oracle.pic import OracleSim
from oracle.topology import build_topology

R = 0.01
SRC = (0.0103, 0.00517, 1.0, 0.6e-9, 0.15e-9, 2 * np.pi * 20e9)   # z, rho, amplitude, t0, sigma, omega
PROBE = (0.0403, 0.00517)


def _guide(L):
    tags = {"bottom": synth.BC_AXIS, "top": synth.BC_PEC, "left": synth.BC_PEC, "right": synth.BC_PEC}
    return synth.rect_mesh(0.0, L, R, 1.0e-3, seed=0, tags=tags, jitter=0.0)


def test_hodge_parts_add_up_and_split_a_uniform_field():
    m = synth.rect_mesh(0.0, 0.02, 0.01, 2.0e-3, seed=3)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo).toarray()
    faces = np.arange(topo.n2)
    Az, Ar = pml_parts(topo, faces)
    S = np.zeros_like(A)
    for t in faces:
        ed = topo.tri_edges[t]
        S[np.ix_(ed, ed)] += Az[t] + Ar[t]
    assert np.abs(S - A).max() <= 1e-13 * np.abs(A).max()
    # uniform E_z: edge values E_z (z_head - z_tail); its energy lies in the z part only
    Ez = 3.0e5
    e = Ez * (m.nodes[topo.edges[:, 1], 0] - m.nodes[topo.edges[:, 0], 0])
    int_rho = sum(topo.area[t] * m.nodes[m.tris[t], 1].mean() for t in faces)
    wz = sum(e[topo.tri_edges[t]] @ Az[t] @ e[topo.tri_edges[t]] for t in faces)
    wr = sum(e[topo.tri_edges[t]] @ Ar[t] @ e[topo.tri_edges[t]] for t in faces)
    assert wz == pytest.approx(EPS0 * Ez ** 2 * int_rho, rel=1e-12)
    assert abs(wr) <= 1e-12 * wz


def _pulse_run(L, pml, dt=None, steps=None):
    m = _guide(L)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=dt, pml=pml)
    sim.add_point_source(*SRC)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(*PROBE)
    sim.step(steps if steps is not None else int(1.9e-9 / sim.dt))
    return sim, np.array(sim.probe_signal)


@pytest.fixture(scope="module")
def reference():
    """A guide long enough that nothing comes back to the probe within 1.9 ns."""
    return _pulse_run(0.36, None)


def test_vanishing_conductivity_reproduces_the_plain_scheme(reference):
    ref, sb = reference
    a, sa = _pulse_run(0.08, dict(z_right=0.06, sigma_max=1e-9, order=3), dt=ref.dt, steps=600)
    b, sp = _pulse_run(0.08, None, dt=ref.dt, steps=600)
    assert a.pml is not None and len(a.pml["face"]) > 100
    assert np.abs(sa - sp).max() <= 1e-10 * np.abs(sp).max()
    assert np.abs(a.E - b.E).max() <= 1e-10 * np.abs(b.E).max()


def test_layer_absorbs_the_guided_pulse(reference):
    ref, sb = reference
    n = len(sb)
    _, s_pec = _pulse_run(0.08, None, dt=ref.dt, steps=n)
    _, s_pml = _pulse_run(0.08, dict(z_right=0.06, sigma_max=3.66, order=3), dt=ref.dt, steps=n)
    peak = np.abs(sb).max()
    r_pec = np.abs(s_pec - sb).max() / peak
    r_pml = np.abs(s_pml - sb).max() / peak
    assert r_pec > 0.5
    assert r_pml < 1e-3


def test_layered_guide_decays_without_growth(reference):
    ref, _ = reference
    m = _guide(0.08)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=ref.dt, pml=dict(z_right=0.06, sigma_max=3.66, order=3))
    sim.add_point_source(*SRC)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    peak = 0.0
    norms = []
    for _ in range(30):
        sim.step(1000)
        norms.append(np.abs(sim.E).max())
        peak = max(peak, norms[-1])
    # what stays is the guide's cutoff mode (uniform in z, zero group velocity:
    # it never enters the layer), at 1e-3 of the peak; it must not grow
    assert max(norms[-5:]) < 1e-2 * peak
    assert max(norms[15:]) <= 2.0 * max(norms[5:15])
