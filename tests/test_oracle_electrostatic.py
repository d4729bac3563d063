"""Pins of the FP64 electrostatic initial state (oracle/electrostatic.py).

With the exact Hodge A, D~div A D~div^T is the rho-weighted P1 stiffness
matrix, so the state is the Galerkin solution of div(rho grad phi) = 0:
a planar gap (conductor plates at z = 0 and z = d, natural boundaries on
the axis and the outer cylinder) gives phi = V z / d exactly, and a smooth
boundary potential gives the Bessel-mode solution with second-order
convergence.  With a full-pattern SPAI (M = A^-1) the scheme's state equals
the exact-Hodge one.  With the level-3 SPAI and a charged beam the state
satisfies the scheme's Gauss law on the free nodes, is curl-free (so one
field step leaves it unchanged), and the charge induced on the conductor
nodes is minus the free charge.
"""

import numpy as np
import pytest
import scipy.special

import synth
from synth import configs
from oracle.electrostatic import electrostatic
from oracle.hodge import hodge_eps
from oracle.spai import spai
from oracle.topology import build_topology

V = 1.0e5


def _gap_mesh(h, seed=0, d=0.01, R=0.02):
    tags = {"bottom": synth.BC_AXIS, "top": synth.BC_OPEN, "left": synth.BC_PEC, "right": synth.BC_PEC}
    return synth.rect_mesh(0.0, d, R, h, seed=seed, tags=tags)


def _plates(m, topo, d):
    phi = np.where(m.nodes[:, 0] > 0.5 * d, V, 0.0)
    assert np.all(np.isclose(m.nodes[~topo.node_free, 0], 0.0) | np.isclose(m.nodes[~topo.node_free, 0], d))
    return phi


def test_planar_gap_is_linear_for_the_exact_hodge():
    d = 0.01
    m = _gap_mesh(1.0e-3)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    phi, E, D, res = electrostatic(topo, A, _plates(m, topo, d), np.zeros(topo.n0), inverse=False)
    np.testing.assert_allclose(phi, V * m.nodes[:, 0] / d, rtol=0, atol=1e-10 * V)
    dz = m.nodes[topo.edges[:, 1], 0] - m.nodes[topo.edges[:, 0], 0]
    np.testing.assert_allclose(E[topo.edge_free], -(V / d) * dz[topo.edge_free], rtol=0, atol=1e-9 * V)
    assert np.abs(res).max() <= 1e-12 * np.abs(D).max()


def test_full_pattern_spai_state_equals_exact_hodge_state():
    d = 0.01
    m = _gap_mesh(3.4e-3, seed=1, R=0.008)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    M = spai(A, topo.edge_free, level=30, drop_tol=0.0)
    assert topo.node_free.sum() >= 3
    phi_c = _plates(m, topo, d)
    pa, Ea, Da, _ = electrostatic(topo, A, phi_c, np.zeros(topo.n0), inverse=False)
    pm, Em, Dm, res = electrostatic(topo, M, phi_c, np.zeros(topo.n0), inverse=True)
    np.testing.assert_allclose(pm, V * m.nodes[:, 0] / d, rtol=0, atol=1e-8 * V)
    np.testing.assert_allclose(pm, pa, rtol=0, atol=1e-8 * V)
    np.testing.assert_allclose(Dm, Da, rtol=0, atol=1e-8 * np.abs(Da).max())


def test_bessel_mode_converges_at_second_order():
    """Closed cylinder 0 <= z <= L, rho <= R: phi = V sin(pi z / L) on the
    side wall, 0 on the end plates; exact phi = V sin(pi z/L) I0(pi rho/L) / I0(pi R/L)."""
    L, R = 0.02, 0.01
    rms, mx = [], []
    for h in (1.0e-3, 0.5e-3):
        m = synth.rect_mesh(0.0, L, R, h, seed=2, jitter=0.0)     # a regular lattice: a clean order
        topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
        A = hodge_eps(topo)
        z, r = m.nodes[:, 0], m.nodes[:, 1]
        exact = V * np.sin(np.pi * z / L) * scipy.special.i0(np.pi * r / L) / scipy.special.i0(np.pi * R / L)
        phi, _, _, _ = electrostatic(topo, A, exact, np.zeros(topo.n0), inverse=False)
        err = np.abs(phi - exact) / V
        rms.append(np.sqrt((err ** 2).mean()))
        mx.append(err.max())
    assert mx[1] < 1e-3
    assert rms[0] / rms[1] > 3.5 and mx[0] / mx[1] > 3.0


def test_gauss_operator_is_the_weighted_p1_stiffness():
    """D~div A D~div^T equals the P1 stiffness of div(rho grad), assembled
    here face by face from the gradients of the nodal hat functions and the
    exact integral of rho over each face (area times the mean vertex rho)."""
    import scipy.sparse as sp
    m = _gap_mesh(2.0e-3, seed=5)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    K = sp.lil_matrix((topo.n0, topo.n0))
    for tri in m.tris:
        p = m.nodes[tri]
        Mx = np.column_stack([np.ones(3), p])
        grads = np.linalg.inv(Mx)[1:, :].T               # row i: grad of the hat function of vertex i
        area = 0.5 * abs(np.linalg.det(Mx))
        Ke = 8.8541878128e-12 * p[:, 1].mean() * area * grads @ grads.T
        for a in range(3):
            for b in range(3):
                K[tri[a], tri[b]] += Ke[a, b]
    L = topo.Ddiv @ A @ topo.Ddiv.T
    assert abs(L - K.tocsr()).max() <= 1e-12 * abs(K).max()


@pytest.fixture(scope="module")
def charged_diode():
    from oracle.pic import OracleSim
    m = configs.diode_mesh(h=1.0e-3)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    zr, u = synth.disk_beam(4000, 0.015, 0.002, 0.008, 0.3, seed=8)
    sim.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 2.0e6)
    sim.inject(0, zr, u)
    phi_c = np.where(m.nodes[:, 0] > 0.5 * configs.DIODE_GAP, configs.DIODE_VOLTS, 0.0)
    Q = sim.charge()
    return m, sim, phi_c, Q


def test_scheme_state_with_charge_is_gauss_consistent_and_curl_free(charged_diode):
    m, sim, phi_c, Q = charged_diode
    topo = sim.topo
    phi, E, D, res = electrostatic(topo, sim.M, phi_c, Q)
    scale = np.abs(topo.Ddiv).dot(np.abs(D)).max()
    assert np.abs(res).max() <= 1e-12 * scale
    assert np.abs(Q[topo.node_free]).max() > 1e3 * np.abs(res).max()        # the charge matters
    assert np.abs(topo.C @ E).max() <= 1e-12 * np.abs(E).max()
    # charge induced on the conductor nodes: minus the free charge
    induced = (topo.Ddiv @ D)[~topo.node_free]
    assert induced.sum() == pytest.approx(-Q[topo.node_free].sum(), rel=1e-10)
    # conductor potentials are kept
    np.testing.assert_array_equal(phi[~topo.node_free], phi_c[~topo.node_free])


def test_scheme_state_without_charge_is_static(charged_diode):
    from oracle.pic import OracleSim
    m, sim, phi_c, _ = charged_diode
    topo = sim.topo
    phi, E, D, res = electrostatic(topo, sim.M, phi_c, np.zeros(topo.n0))
    o = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim.dt, M=sim.M)
    o.set_fields(E, np.zeros(topo.n2))
    o.step(5)
    assert np.abs(o.B).max() <= 1e-12 * np.abs(E).max()
    np.testing.assert_allclose(o.E, E, rtol=0, atol=1e-10 * np.abs(E).max())
