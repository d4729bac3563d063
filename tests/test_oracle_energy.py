"""Pins of the oracle's energy diagnostic and of the face-field gather that
drives the push.

The step reports the energies of its starting time level n:
W_E = 1/2 E^n [*eps]_a E^n, W_B = 1/2 B^{n+1/2} H B^{n-1/2} and
W_K = 1/2 (K^{n-1/2} + K^{n+1/2}).  What fixes them independently:
- without sources W_E + W_B is the invariant of the leapfrog pair
  (full_d_dfl)/(full_d_dal) (Sec. 3.1), so it must stay constant to
  rounding (a wrong time level or pairing in either term oscillates at
  O(omega dt));
- the TM010 mode of a PEC cylinder (Sec. 4.1) has the closed-form energy
  (eps0/2) E0^2 h (a^2/2) J1(x01)^2 per radian; at t = 0 it is all electric
  and a quarter period later all magnetic;
- a mono-energetic beam has W_K = N w m c^2 (gamma - 1) / (2 pi); a uniform
  axial B turns momenta without changing |u|, and a uniform E adds exactly
  q E dt / m to them (Boris, Sec. 3.3);
- the face field the push sees is the time average of the face fluxes
  B^{n-1/2}, B^{n+1/2} over the face area (Sec. 3.2): with E = 0 and two
  different uniform B_phi before and after the Faraday update, one step turns
  (u_rho, u_z) by exactly 2 atan(q Bbar dt / (2 gamma m)) about phi-hat.
"""

import numpy as np
import pytest
import scipy.special

import synth
from synth import configs
from oracle.pic import OracleSim
from oracle.hodge import EPS0

C = 299792458.0
QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS
X01 = 2.404825557695773


@pytest.fixture(scope="module")
def cavity():
    m = configs.cavity_mesh()
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=configs.CAVITY_DT)
    return m, sim


def _fresh(cavity, **kw):
    m, s0 = cavity
    return OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=s0.dt, M=s0.M, **kw)


def _tm010(sim, e0=1e6):
    E0, B0, omega = synth.tm010_fields(sim.topo.nodes, sim.topo.tris, sim.topo.edges, configs.CAVITY_A, e0,
                                       sim.dt)
    sim.set_fields(E0, B0)
    return omega


def _w_closed(e0=1e6):
    a, h = configs.CAVITY_A, configs.CAVITY_H
    return 0.5 * EPS0 * e0 ** 2 * h * 0.5 * a * a * scipy.special.j1(X01) ** 2


# ------------------------------------------------------------ field energy
def test_field_energy_is_the_leapfrog_invariant(cavity):
    sim = _fresh(cavity)
    _tm010(sim)
    sim.log_energies = True
    sim.step(600)
    log = np.array(sim.energy_log)
    assert np.array_equal(log[:, 0], np.arange(600))
    W = log[:, 1] + log[:, 2]
    assert np.abs(W / W[0] - 1).max() < 1e-11
    # the energy really moves between the two terms (so the test is not vacuous)
    assert log[:, 1].min() < 0.05 * W[0] and log[:, 2].max() > 0.95 * W[0]
    # a wrong pairing, B^{n+1/2} H B^{n+1/2}, is not invariant
    sim2 = _fresh(cavity)
    _tm010(sim2)
    bad = []
    for _ in range(200):
        E, D = sim2.E.copy(), sim2.D.copy()
        sim2.step(1)
        bad.append(0.5 * E @ D + 0.5 * sim2.B @ (sim2.H * sim2.B))
    bad = np.array(bad)
    assert np.abs(bad / bad[0] - 1).max() > 1e-4


def test_tm010_energy_closed_form(cavity):
    """Electric energy at t = 0 and magnetic energy a quarter period later
    against the continuum mode's energy (mesh error O(h^2): h/a = 0.049)."""
    sim = _fresh(cavity)
    omega = _tm010(sim)
    sim.log_energies = True
    quarter = int(round(0.25 * 2 * np.pi / omega / sim.dt))
    sim.step(quarter + 1)
    log = np.array(sim.energy_log)
    W = _w_closed()
    n0, WE0, WB0, WK0, WEx0 = log[0]
    assert WEx0 == pytest.approx(W, rel=1e-3)          # exact Hodge (measured 2.6e-4)
    assert WE0 == pytest.approx(WEx0, rel=2e-3)        # the SPAI's [*eps]_a
    assert abs(WB0) < 1e-4 * W                         # B ~ 0 at t = 0
    assert WK0 == 0.0
    q = log[quarter]
    assert q[2] == pytest.approx(WE0 + WB0, rel=5e-4)  # all magnetic a quarter period later
    assert q[1] < 1e-4 * W


def test_tm010_energy_converges_at_second_order():
    """The exact-Hodge electric energy of the interpolated mode converges to
    the closed form as h^2 (two meshes, h and h/2)."""
    errs = []
    for h in (1.0e-3, 0.5e-3):
        m = configs.cavity_mesh(h=h)
        from oracle.topology import build_topology
        from oracle.hodge import hodge_eps
        topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
        A = hodge_eps(topo)
        E0, _, _ = synth.tm010_fields(topo.nodes, topo.tris, topo.edges, configs.CAVITY_A, 1e6, 1e-13)
        E0 = np.where(topo.edge_free, E0, 0.0)
        errs.append(abs(0.5 * E0 @ (A @ E0) / _w_closed() - 1))
    assert errs[1] < errs[0] / 2.5


# --------------------------------------------------------- kinetic energy
def _beam(sim, n, u, seed=4):
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.006, 0.014, n)
    r = rng.uniform(0.002, 0.006, n)
    sp = sim.add_species(QE, ME, configs.CAVITY_WEIGHT)
    sim.inject(sp, np.stack([z, r], axis=1), np.tile(u, (n, 1)))


def test_kinetic_energy_of_a_mono_energetic_beam(cavity):
    g = 1.7
    u = np.array([0.0, 0.0, C * np.sqrt(g * g - 1)])
    want = 300 * configs.CAVITY_WEIGHT * ME * C * C * (g - 1) / (2 * np.pi)
    sim = _fresh(cavity)
    _beam(sim, 300, u)
    assert sim.kinetic_energy() == pytest.approx(want, rel=1e-13)
    sim.log_energies = True
    sim.step(1)                      # zero fields at step 0: u^{1/2} = u^{-1/2}
    assert sim.energy_log[0][3] == pytest.approx(want, rel=1e-13)
    assert sim.kinetic_energy() == pytest.approx(want, rel=1e-13)
    # a uniform axial field turns u_perp and keeps |u|
    sim = _fresh(cavity, bz=3.0)
    _beam(sim, 300, np.array([0.6 * C, 0.9 * C, 0.8 * C]))
    g = np.sqrt(1 + (0.36 + 0.81 + 0.64))
    want = 300 * configs.CAVITY_WEIGHT * ME * C * C * (g - 1) / (2 * np.pi)
    sim.log_energies = True
    u0 = sim.pu.copy()
    sim.step(1)
    assert not np.allclose(sim.pu[:, 0], u0[:, 0])
    assert sim.energy_log[0][3] == pytest.approx(want, rel=1e-13)


def test_kinetic_energy_is_the_half_step_mean(cavity):
    """Uniform E (faces without conductor sides see it exactly): u^{1/2} =
    u^{-1/2} + q E dt / m, and W_K^0 is the mean of the two half steps."""
    sim = _fresh(cavity)
    ez, er = 2.0e8, -1.0e8
    sim.set_fields(synth.uniform_field_dofs(sim.topo.nodes, sim.topo.edges, ez, er), np.zeros(sim.topo.n2))
    interior = np.flatnonzero(sim.topo.edge_free[sim.topo.tri_edges].all(axis=1))
    rng = np.random.default_rng(9)
    tri = rng.choice(interior, 50, replace=False)
    pts = sim.topo.nodes[sim.topo.tris[tri]].mean(axis=1)
    u0 = np.array([0.1 * C, 0.0, 0.3 * C])
    sp = sim.add_species(QE, ME, configs.CAVITY_WEIGHT)
    sim.inject(sp, pts, np.tile(u0, (50, 1)))
    sim.log_energies = True
    sim.step(1)
    u1 = u0 + QE / ME * sim.dt * np.array([er, 0.0, ez])

    def kin(u):
        w2 = (u @ u) / C ** 2
        return 50 * configs.CAVITY_WEIGHT * ME * C * C * w2 / (np.sqrt(1 + w2) + 1) / (2 * np.pi)

    # columns: (n, W_E, W_B, W_K, W_E_exact)
    wk = sim.energy_log[0][3]
    assert wk == pytest.approx(0.5 * (kin(u0) + kin(u1)), rel=1e-12)
    assert wk != pytest.approx(kin(u0), rel=1e-3) and wk != pytest.approx(kin(u1), rel=1e-3)
    assert sim.kinetic_energy() == pytest.approx(kin(u1), rel=1e-12)


# ------------------------------------------------------------- face gather
@pytest.mark.parametrize("ba,bb,g", [(4.0, 12.0, 1.2), (-6.0, 2.0, 2.5), (9.0, -3.0, 1.05)])
def test_push_sees_the_time_centred_face_field(cavity, ba, bb, g):
    """E = 0, B^{-1/2} = ba per unit area on every face; a magnetic point
    source in the particle's face brings it to bb at +1/2 (the source term of
    the Faraday update is -dt M).  The push must turn (u_rho, u_z) about
    phi-hat by 2 atan(q (ba + bb)/2 dt / (2 gamma m))."""
    sim = _fresh(cavity)
    nodes, tris = sim.topo.nodes, sim.topo.tris
    v = nodes[tris]
    area = 0.5 * ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
                  - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))
    assert (area > 0).all()
    sim.set_fields(np.zeros(sim.topo.n1), ba * area)
    zr = np.array([[0.0101, 0.0047]])
    t = int(sim.locate(zr)[0])
    sim.add_point_source(zr[0, 0], zr[0, 1], (ba - bb) * area[t] / sim.dt, 0.0, 1.0, 0.0)
    ut = C * np.sqrt(g * g - 1)
    u0 = np.array([0.6 * ut, 0.0, 0.8 * ut])
    sp = sim.add_species(QE, ME, 1)
    sim.inject(sp, zr, u0[None, :])
    sim.step(1)
    assert sim.B[t] == pytest.approx(bb * area[t], rel=1e-12)
    bbar = 0.5 * (ba + bb)
    th = 2 * np.arctan(QE / ME * bbar * sim.dt / (2 * g))
    want_r = u0[0] * np.cos(th) - u0[2] * np.sin(th)
    want_z = u0[0] * np.sin(th) + u0[2] * np.cos(th)
    u1 = sim.pu[0]
    assert u1[1] == 0.0
    np.testing.assert_allclose([u1[0], u1[2]], [want_r, want_z], rtol=1e-12, atol=1e-12 * ut)
    # neither end value alone, nor the opposite sense, gives this rotation
    for wrong in (ba, bb, -bbar):
        tw = 2 * np.arctan(QE / ME * wrong * sim.dt / (2 * g))
        assert abs(u1[0] - (u0[0] * np.cos(tw) - u0[2] * np.sin(tw))) > 1e-6 * ut
