"""Magnetic point sources and the field probe (Sec. 4.1) on the GPU against
the FP64 oracle, both precisions.

Workload: the paper's cavity (a = 0.5 m, h = 1 m) on a coarse 25 mm mesh,
its two Gaussian-modulated sources and the probe at (z = 0.71, rho = 0.39),
3,000 steps at half the stability limit (28 ns: the first pulse rises).
Bounds: the probe signal and the final E to rel-L2 1e-9 (FP64 step) /
1e-5 (mixed: E in FP32); steps replayed from graphs give the same signal
as eager steps, bit for bit (the mixed field update has no atomics).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

A_CAV, H_CAV = 0.5, 1.0
TG, SIG, WG = 40e-9, 1e-9, np.pi * 1e9
SOURCES = [(0.2, 0.37, 0.7, TG / 2), (0.7, 0.08, 0.5, TG)]
PROBE = (0.71, 0.39)
STEPS = 3000


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def cavity():
    from oracle.pic import OracleSim
    m = synth.rect_mesh(0.0, H_CAV, A_CAV, 0.025, seed=0)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    for z, rho, a, t0 in SOURCES:
        sim.add_point_source(z, rho, a, t0, SIG, WG)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(*PROBE)
    sim.step(STEPS)
    return m, sim


def _ctx(axp, m, dt, prec, use_graph=1):
    c = axp.make_ctx(m, dt=dt, precision=axp.PREC_PLAIN_FP64 if prec == "plain" else axp.PREC_MIXED,
                     use_graph=use_graph)
    for z, rho, a, t0 in SOURCES:
        c.add_point_source(z, rho, a, t0, SIG, WG)
    c.set_probe(*PROBE, STEPS)
    return c


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_probe_signal_matches_oracle(axp, cavity, prec):
    m, sim = cavity
    print(f"[gpu] sources {prec}", flush=True)
    c = _ctx(axp, m, sim.dt, prec)
    c.step(STEPS)
    sig = c.get_probe()
    ref = np.array(sim.probe_signal)
    assert sig.shape == ref.shape == (STEPS, 2)
    tol = 1e-9 if prec == "plain" else 1e-5
    e_sig = _rel_l2(sig, ref)
    E, B = c.get_fields()
    e_E = _rel_l2(E, sim.E)
    print(f"[gpu] {prec}: probe rel-L2 {e_sig:.2e}, E rel-L2 {e_E:.2e}", flush=True)
    assert np.abs(ref).max() > 0.0
    assert e_sig <= tol and e_E <= tol
    c.close()


def test_graph_replay_gives_the_eager_signal(axp, cavity):
    m, sim = cavity
    out = []
    for g in (0, 1):
        c = _ctx(axp, m, sim.dt, "mixed", use_graph=g)
        c.step(STEPS // 2)
        c.step(STEPS - STEPS // 2)
        out.append((c.get_probe(), c.get_fields()[0]))
        c.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_sources_and_probe_arguments(axp, cavity):
    m, sim = cavity
    c = axp.make_ctx(m, dt=sim.dt)
    with pytest.raises(axp.AxpError):
        c.add_point_source(2.0, 0.1, 1.0, 0.0, SIG, WG)          # outside the cavity
    with pytest.raises(axp.AxpError):
        c.add_point_source(0.5, 0.1, 1.0, 0.0, 0.0, WG)          # sigma must be positive
    for _ in range(8):
        c.add_point_source(0.5, 0.1, 1.0, 0.0, SIG, WG)
    with pytest.raises(axp.AxpError):
        c.add_point_source(0.5, 0.1, 1.0, 0.0, SIG, WG)          # at most 8
    c.clear_point_sources()
    c.set_probe(0.5, 0.1, 10)
    c.step(25)
    assert c.get_probe().shape == (10, 2)                        # capacity caps the record
    c.set_probe(0.5, 0.1, 0)
    assert c.get_probe().shape == (0, 2)
    c.close()


def test_cold_test_band_edges_of_a_uniform_cell(axp):
    """The cold-test driver on a smooth cylinder cell: its two lowest modes
    are the TM01 band edges c x_01/(2 pi r0) and c/(2 pi) sqrt((x_01/r0)^2 + (pi/d)^2)."""
    from paper_1701_03784_amd import cold_test
    r0, d = 0.015, 0.0167
    m = cold_test.cell_mesh(r0, 0.0, d, 0.4e-3)
    f0 = cold_test.C_LIGHT / (2 * np.pi) * cold_test.X01 / r0
    fp = cold_test.C_LIGHT / (2 * np.pi) * np.hypot(cold_test.X01 / r0, np.pi / d)
    peaks, faces, steps = cold_test.cell_modes(lambda mm: axp.make_ctx(mm), m, r0, d, 20.0, 0.5 * f0, 1.3 * fp)
    print(f"[gpu] uniform cell: {faces} faces, {steps} steps, modes {[p / 1e9 for p in peaks]} GHz", flush=True)
    assert len(peaks) == 2
    assert abs(peaks[0] / f0 - 1) < 2e-3 and abs(peaks[1] / fp - 1) < 2e-3


def test_cold_test_dispersion_of_a_uniform_guide(axp):
    """Four smooth-guide periods between the plates, on the mapped grid: the
    five lowest modes are the TM01 dispersion curve at phase advance k pi / 4
    per period, c/(2 pi) sqrt((x_01/r0)^2 + (k pi / (4 d))^2)."""
    from paper_1701_03784_amd import cold_test
    r0, d, N = 0.015, 0.0167, 4
    m = cold_test.cell_mesh(r0, 0.0, d, 0.4e-3, kind="grid", periods=N)
    ref = cold_test.uniform_dispersion(r0, d, np.pi * np.arange(N + 1) / N)
    peaks, faces, steps = cold_test.cell_modes(lambda mm: axp.make_ctx(mm), m, r0, d, 40.0, 0.5 * ref[0],
                                               1.3 * ref[-1], count=N + 1)
    print(f"[gpu] 4-period guide: {faces} faces, {steps} steps, modes {[p / 1e9 for p in peaks]} GHz", flush=True)
    assert len(peaks) == N + 1
    np.testing.assert_allclose(np.array(peaks) / ref, 1.0, rtol=0, atol=2e-3)



def test_cold_test_modes_are_the_discrete_eigenvalues(axp):
    """Rippled cell, which has no closed form: the driver's two lowest modes
    are eigenfrequencies of the semi-discrete operator M K.  Here M is the
    oracle's SPAI and K = C^T [*mu^-1] C on free edges, found by a
    shift-invert eigensolve.  Each is mapped through the leapfrog's own time
    dispersion, omega_h = (2/dt) asin(omega dt / 2).  Bound: 1e-5 relative,
    set by the spectral peak estimate."""
    import scipy.sparse.linalg as spla
    from paper_1701_03784_amd import cold_test
    from oracle.topology import build_topology
    from oracle.hodge import hodge_eps, hodge_mu_inv
    from oracle.cfl import curl_curl, cfl_dt
    from oracle.spai import spai
    r0, amp, d = 0.015, 0.0025, 0.0167
    m = cold_test.cell_mesh(r0, amp, d, 0.8e-3)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A, H = hodge_eps(topo), hodge_mu_inv(topo)
    M = spai(A, topo.edge_free, 3, 1e-3)
    dt = 0.4 * cfl_dt(topo, H, M)[0]
    idx = np.flatnonzero(topo.edge_free)
    MK = (M[idx][:, idx] @ curl_curl(topo, H)[idx][:, idx]).tocsc()
    lam = spla.eigs(MK, k=6, sigma=(2 * np.pi * 8.5e9) ** 2, which="LM", return_eigenvectors=False).real
    omega = np.sort(np.sqrt(lam[lam > (2 * np.pi * 1e9) ** 2]))[:2]
    f_ref = 2.0 / dt * np.arcsin(0.5 * omega * dt) / (2 * np.pi)
    f_lo = 0.5 * cold_test.uniform_dispersion(r0, d, 0.0)
    f_hi = 1.3 * cold_test.uniform_dispersion(r0, d, np.pi)
    peaks, faces, steps = cold_test.cell_modes(lambda mm: axp.make_ctx(mm, dt=dt), m, r0, d, 60.0, f_lo, f_hi)
    print(f"[gpu] rippled cell: modes {[p / 1e9 for p in peaks]} GHz, eigen {list(f_ref / 1e9)} GHz", flush=True)
    assert len(peaks) == 2
    np.testing.assert_allclose(np.array(peaks) / f_ref, 1.0, rtol=0, atol=1e-5)
