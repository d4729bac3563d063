"""Absorbing layers (axp_set_layers) on the GPU against the FP64 oracle.

Workload: a circular guide (R = 1 cm, conductor walls, regular 1 mm mesh),
a 20 GHz Gaussian-modulated point source at z = 1 cm, the probe at
z = 4 cm, a 2 cm layer beyond z = 6 cm (sigma_max = 3.66 S/m, cubic).
Bounds: the SPAI of the stretched Hodge equals the oracle's to 1e-12; the
probe signal and E after 2,000 steps equal the oracle's to rel-L2 1e-9
(FP64 step) / 1e-5 (mixed); the pulse that meets the layer comes back
below 1e-3 of its amplitude against a guide long enough to return nothing
in the window; graph replay equals eager steps bit for bit (mixed).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

R = 0.01
SRC = (0.0103, 0.00517, 1.0, 0.6e-9, 0.15e-9, 2 * np.pi * 20e9)
PROBE = (0.0403, 0.00517)
LAYER = dict(z_right=0.06, sigma_max=3.66, order=3)


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


def _guide(L):
    tags = {"bottom": synth.BC_AXIS, "top": synth.BC_PEC, "left": synth.BC_PEC, "right": synth.BC_PEC}
    return synth.rect_mesh(0.0, L, R, 1.0e-3, seed=0, tags=tags, jitter=0.0)


@pytest.fixture(scope="module")
def oracle_runs():
    from oracle.pic import OracleSim
    long_m = _guide(0.36)
    ref = OracleSim(long_m.nodes, long_m.tris, long_m.seg, long_m.tag)
    dt = ref.dt
    m = _guide(0.08)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=dt, pml=LAYER)
    sim.add_point_source(*SRC)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(*PROBE)
    sim.step(2000)
    return long_m, m, dt, sim


def _ctx(axp, m, dt, prec, layers=LAYER, use_graph=1, steps=2000):
    c = axp.make_ctx(m, dt=dt, precision=axp.PREC_PLAIN_FP64 if prec == "plain" else axp.PREC_MIXED,
                     layers=layers, use_graph=use_graph)
    c.set_fields(np.zeros(c.info()["n_edges"]), np.zeros(c.info()["n_faces"]))
    c.add_point_source(*SRC)
    c.set_probe(*PROBE, steps)
    return c


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_stretched_spai_matches_oracle(axp, oracle_runs):
    _, m, dt, sim = oracle_runs
    c = _ctx(axp, m, dt, "mixed")
    assert c.info()["n_layer_faces"] == len(sim.pml["face"]) > 0
    M = c.get_spai().toarray()
    Mo = sim.M.toarray()
    assert np.abs(M - Mo).max() <= 1e-12 * np.abs(Mo).max()
    c.close()


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_layered_guide_matches_oracle(axp, oracle_runs, prec):
    _, m, dt, sim = oracle_runs
    print(f"[gpu] layers {prec}", flush=True)
    c = _ctx(axp, m, dt, prec)
    c.step(2000)
    sig = c.get_probe()
    E, _ = c.get_fields()
    ref = np.array(sim.probe_signal)
    e_sig, e_E = _rel_l2(sig, ref), _rel_l2(E, sim.E)
    print(f"[gpu] layers {prec}: probe rel-L2 {e_sig:.2e}, E rel-L2 {e_E:.2e}", flush=True)
    tol = 1e-9 if prec == "plain" else 1e-5
    assert e_sig <= tol and e_E <= tol
    c.close()


def test_layer_absorbs_the_pulse_on_the_gpu(axp, oracle_runs):
    long_m, m, dt, _ = oracle_runs
    n = int(1.9e-9 / dt)
    out = {}
    for name, mesh, layers in (("ref", long_m, None), ("layer", m, LAYER), ("pec", m, None)):
        c = _ctx(axp, mesh, dt, "mixed", layers=layers, steps=n)
        c.step(n)
        out[name] = c.get_probe()
        c.close()
    peak = np.abs(out["ref"]).max()
    r_layer = np.abs(out["layer"] - out["ref"]).max() / peak
    r_pec = np.abs(out["pec"] - out["ref"]).max() / peak
    print(f"[gpu] reflection: layer {r_layer:.2e}, conductor end {r_pec:.2e}", flush=True)
    assert r_pec > 0.5
    assert r_layer < 1e-3


def test_layers_graph_replay_equals_eager(axp, oracle_runs):
    _, m, dt, _ = oracle_runs
    out = []
    for g in (0, 1):
        c = _ctx(axp, m, dt, "mixed", use_graph=g)
        c.step(1000)
        out.append((c.get_probe(), c.get_fields()[0]))
        c.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_layer_restrictions(axp, oracle_runs, tmp_path):
    _, m, dt, _ = oracle_runs
    c = _ctx(axp, m, dt, "mixed")
    with pytest.raises(axp.AxpError):
        c.save(str(tmp_path / "x.ckpt"))
    rc = c.lib.axp_set_layers(c.h, 2, 0.0, 0.06, 3.66, 3)
    assert rc != 0                                               # after axp_build
    c.close()
    c2 = axp.make_ctx(m, dt=dt, layers=LAYER)                    # no sources or probe
    c2.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 1000)
    with pytest.raises(axp.AxpError):
        axp.Batch([c2])
    c2.close()


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_particles_crossing_into_the_layer_match_oracle(axp, prec):
    """A beam that crosses into the layer and reaches the end wall: 3,000
    electrons (weight 10^4) in 4.5 cm <= z <= 7.5 cm at 0.5 c along z in
    B_z = 0.5 T, 250 steps.  The layer stretches only the fields; the
    particles deposit into layer faces like any other, so continuity stays
    exact (mixed) or to FP64 rounding.  E to rel-L2 1e-9 (FP64 step) /
    1e-4 (mixed); the same number absorbed; the survivors' positions to
    1e-12 m / 2e-7 m (the FP32 rounding of 250 steps, as in the diode).
    With no applied field, E is the beam's own field, so its mixed error is
    the current's.  The FP32 momenta are off by up to 1e-5 of the largest,
    each deposit follows its particle's displacement, and a face sums the
    deposits of its particles: the bound of the staircased-wall test."""
    from oracle.pic import OracleSim
    m = _guide(0.08)
    rng = np.random.default_rng(31)
    n = 3000
    zr = np.stack([rng.uniform(0.045, 0.075, n), np.sqrt(rng.uniform(0.0, 0.008 ** 2, n))], axis=1)
    g = 0.5 / np.sqrt(0.75) * 299792458.0
    u = np.zeros((n, 3))
    u[:, 2] = g * (1.0 + 0.1 * np.arange(n) / n)
    u[:, 0] = 0.05 * g * rng.standard_normal(n)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, bz=0.5, pml=LAYER)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 10000)
    sim.inject(0, zr, u)
    tight = prec == "plain"
    c = axp.make_ctx(m, dt=sim.dt, diag_every=1, layers=LAYER,
                     precision=axp.PREC_PLAIN_FP64 if tight else axp.PREC_MIXED)
    c.set_fields(np.zeros(c.info()["n_edges"]), np.zeros(c.info()["n_faces"]))
    c.set_external_bz(0.5)
    sp = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, 10000)
    c.inject(sp, zr, u)
    c.diag()
    print(f"[gpu] layer with particles {prec}", flush=True)
    for _ in range(5):
        c.step(50)
        sim.step(50)
        d = c.diag()
        if tight:
            assert d["dce_max_rel"] <= 1e-12
        else:
            assert d["dce_max_abs"] == 0
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0
    assert int(sim.stats[1]) > 500
    assert d["n_absorbed"] == int(sim.stats[1])
    E, _ = c.get_fields()
    e_E = _rel_l2(E, sim.E)
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = sim.particles()
    assert len(zr_g) == len(zr_o)
    import scipy.spatial
    _, idx = scipy.spatial.cKDTree(np.concatenate([zr_o / 1e-6, u_o / 1e3], axis=1)).query(
        np.concatenate([zr_g / 1e-6, u_g / 1e3], axis=1))
    assert len(np.unique(idx)) == len(idx)
    e_pos = np.abs(zr_g - zr_o[idx]).max()
    print(f"[gpu] layer with particles {prec}: absorbed {d['n_absorbed']}, E rel-L2 {e_E:.2e}, positions {e_pos:.1e} m",
          flush=True)
    assert e_E <= (1e-9 if tight else 1e-4)
    assert e_pos <= (1e-12 if tight else 2e-7)
    c.close()
