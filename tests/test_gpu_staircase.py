"""Staircased walls on the GPU against the FP64 oracle.

A staircased slow-wave cell (the step-cell wall of a structured grid:
vertical risers and re-entrant corners, r0 = 15 mm, ripple 2.5 mm, period
16.7 mm, 0.8 mm grid) with a Gaussian-modulated magnetic point source and a
probe, 1,500 steps (the pulse and its ringing), both precisions: probe
signal and final E to rel-L2 1e-9 (FP64 step) / 1e-5 (mixed).  Then
2,000 single-electron particles at 0.5 c in random directions, 40 steps,
many of them striking the steps: continuity exact (mixed) or to FP64
rounding, no walk overflow or non-finite value, the same number absorbed,
positions to 1e-8 m (mixed) / 1e-12 m (FP64), momenta to 1e-5 / 1e-10 of
the largest, the last step's currents to 1e-4 / 1e-10 of the largest.  The
mixed current bound follows from the momentum bound: a particle's deposit
is proportional to its displacement v dt, so after 40 steps of FP32 pushes
in the self-field it is off by up to 1e-5 of the largest single deposit, and
an edge sums the deposits of the particles in its faces (up to about ten
per face here).
"""

import numpy as np
import pytest
import scipy.spatial

import synth

pytestmark = pytest.mark.gpu

R0, AMP, D, H = 0.015, 0.0025, 0.0167, 0.8e-3
SRC = (D / 3.0, 0.6 * R0, 1.0, 0.3e-9, 0.04e-9, 2 * np.pi * 10e9)
PROBE = (0.21 * D, 0.31 * R0)
STEPS = 1500
QE, ME, C = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 299792458.0


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def cell():
    from paper_1701_03784_amd import cold_test
    return cold_test.cell_mesh(R0, AMP, D, H, kind="staircase")


@pytest.fixture(scope="module")
def ringing(cell):
    from oracle.pic import OracleSim
    sim = OracleSim(cell.nodes, cell.tris, cell.seg, cell.tag)
    sim.add_point_source(*SRC)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(*PROBE)
    sim.step(STEPS)
    return sim


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_staircased_cell_rings_like_the_oracle(axp, cell, ringing, prec):
    sim = ringing
    print(f"[gpu] staircase fields {prec}: {cell.n_tris} faces", flush=True)
    c = axp.make_ctx(cell, dt=sim.dt, precision=axp.PREC_PLAIN_FP64 if prec == "plain" else axp.PREC_MIXED)
    c.set_fields(np.zeros(c.info()["n_edges"]), np.zeros(c.info()["n_faces"]))
    c.add_point_source(*SRC)
    c.set_probe(*PROBE, STEPS)
    c.step(STEPS)
    sig, ref = c.get_probe(), np.array(sim.probe_signal)
    E, _ = c.get_fields()
    e_sig, e_E = _rel_l2(sig, ref), _rel_l2(E, sim.E)
    print(f"[gpu] staircase {prec}: probe rel-L2 {e_sig:.2e}, E rel-L2 {e_E:.2e}", flush=True)
    tol = 1e-9 if prec == "plain" else 1e-5
    assert np.abs(ref).max() > 0.0
    assert e_sig <= tol and e_E <= tol
    c.close()


def _particles(m, n=2000, seed=29):
    rng = np.random.default_rng(seed)
    area = m.signed_areas()
    t = rng.choice(len(area), n, p=area / area.sum())
    a, b = rng.uniform(size=(2, n))
    flip = a + b > 1
    a[flip], b[flip] = 1 - a[flip], 1 - b[flip]
    p = m.nodes[m.tris[t]]
    zr = p[:, 0] + a[:, None] * (p[:, 1] - p[:, 0]) + b[:, None] * (p[:, 2] - p[:, 0])
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    g = 0.5 / np.sqrt(1 - 0.25) * C * (1.0 + 0.2 * np.arange(n) / n)      # distinct speeds
    return zr, v * g[:, None]


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_particles_strike_the_steps_like_the_oracle(axp, cell, prec):
    from oracle.pic import OracleSim
    sim = OracleSim(cell.nodes, cell.tris, cell.seg, cell.tag)
    zr, u = _particles(cell)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.add_species(QE, ME, 1)
    sim.inject(0, zr, u)
    tight = prec == "plain"
    c = axp.make_ctx(cell, dt=sim.dt, diag_every=1,
                     precision=axp.PREC_PLAIN_FP64 if tight else axp.PREC_MIXED)
    c.set_fields(np.zeros(c.info()["n_edges"]), np.zeros(c.info()["n_faces"]))
    sp = c.add_species(QE, ME, 1)
    c.inject(sp, zr, u)
    c.diag()
    print(f"[gpu] staircase particles {prec}: {len(zr)} particles", flush=True)
    for _ in range(40):
        c.step(1)
        sim.step(1)
        d = c.diag()
        if tight:
            assert d["dce_max_rel"] <= 1e-12
        else:
            assert d["dce_max_abs"] == 0
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0
    assert int(sim.stats[1]) > 100
    assert d["n_absorbed"] == int(sim.stats[1])
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = sim.particles()
    assert len(zr_g) == len(zr_o)
    sa = np.concatenate([zr_g / 1e-6, u_g / 1e3], axis=1)
    sb = np.concatenate([zr_o / 1e-6, u_o / 1e3], axis=1)
    _, idx = scipy.spatial.cKDTree(sb).query(sa)
    assert len(np.unique(idx)) == len(idx)
    assert np.abs(zr_g - zr_o[idx]).max() < (1e-12 if tight else 1e-8)
    assert np.abs(u_g - u_o[idx]).max() < (1e-10 if tight else 1e-5) * np.abs(u_o).max()
    _, Jdt, _ = c.get_sources()
    J_o = sim.J * sim.dt
    assert np.abs(Jdt - J_o).max() <= (1e-10 if tight else 1e-4) * np.abs(J_o).max()
    c.close()
