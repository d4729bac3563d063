"""Parity of the FP64 GPU step (AXP_PREC_PLAIN_FP64) with the FP64 oracle.

Same cavity workload as the mixed-precision parity tests.  Every quantity
of this step is FP64, so the bounds are those of FP64 rounding: the GPU
keeps D = [*eps]_a E and recomputes E = M D each step while the oracle
updates E directly (equal in exact arithmetic), and the currents are summed
by FP64 atomics in varying order.  Bounds: fields rel-L2 <= 1e-9 after
1,000 steps; particles 1e-12 m / 1e-10 relative after one step; the
continuity residual <= 1e-12 of max |Q| (eq. DCE in FP64); the Gauss
residual stays at its initial value to 1e-13 of the D scale.
"""

import numpy as np
import pytest
import scipy.spatial

import synth
from synth import configs

pytestmark = pytest.mark.gpu

QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def cavity():
    from oracle.pic import OracleSim
    m = configs.cavity_mesh()
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=configs.CAVITY_DT)
    E0, B0, omega = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, configs.CAVITY_A, 1e6, sim.dt)
    return m, sim, E0, B0


def _ctx(axp, m, **kw):
    print(f"[gpu] build plain ctx faces={m.n_tris} {kw}", flush=True)
    kw.setdefault("dt", configs.CAVITY_DT)
    return axp.make_ctx(m, precision=axp.PREC_PLAIN_FP64, **kw)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_plain_field_only_1000_steps(axp, cavity):
    from oracle.pic import OracleSim
    m, sim0, E0, B0 = cavity
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    sim.set_fields(E0, B0)
    c = _ctx(axp, m)
    assert c.info()["precision"] == axp.PREC_PLAIN_FP64
    c.set_fields(E0, B0)
    c.step(1000)
    sim.step(1000)
    E, B = c.get_fields()
    print(f"[gpu] plain field-only: relL2 E {_rel_l2(E, sim.E):.2e} B {_rel_l2(B, sim.B):.2e}", flush=True)
    assert _rel_l2(E, sim.E) <= 1e-9
    assert _rel_l2(B, sim.B) <= 1e-9


def test_plain_one_step_particles(axp, cavity):
    from oracle.pic import OracleSim
    m, sim0, E0, B0 = cavity
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    sim.set_fields(E0, B0)
    sp_o = sim.add_species(QE, ME, configs.CAVITY_WEIGHT)
    zr, u = configs.cavity_beam()
    sim.inject(sp_o, zr, u)
    c = _ctx(axp, m)
    c.set_fields(E0, B0)
    sp = c.add_species(QE, ME, configs.CAVITY_WEIGHT)
    c.inject(sp, zr, u)
    c.step(1)
    sim.step(1)
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = sim.particles()
    assert len(zr_g) == len(zr_o)
    d, idx = scipy.spatial.cKDTree(np.concatenate([zr_o / 1e-6, u_o / 1e3], 1)).query(
        np.concatenate([zr_g / 1e-6, u_g / 1e3], 1))
    assert len(np.unique(idx)) == len(idx)
    assert np.abs(zr_g - zr_o[idx]).max() < 1e-12
    assert np.abs(u_g - u_o[idx]).max() < 1e-10 * np.abs(u_o).max()
    D, Jdt, Q = c.get_sources()
    J_o = sim.J * sim.dt
    assert np.abs(Jdt - J_o).max() <= 1e-10 * np.abs(J_o).max()
    E, B = c.get_fields()
    assert _rel_l2(E, sim.E) <= 1e-10
    assert _rel_l2(B, sim.B) <= 1e-10


def test_plain_pic_1000_steps(axp, cavity):
    from oracle.pic import OracleSim
    m, sim0, E0, B0 = cavity
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    sim.set_fields(E0, B0)
    sp_o = sim.add_species(QE, ME, configs.CAVITY_WEIGHT)
    zr, u = configs.cavity_beam()
    sim.inject(sp_o, zr, u)
    c = _ctx(axp, m, diag_every=1)
    c.set_fields(E0, B0)
    sp = c.add_species(QE, ME, configs.CAVITY_WEIGHT)
    c.inject(sp, zr, u)
    c.diag()
    for chunk in range(10):
        c.step(100)
        sim.step(100)
        d = c.diag()
        E, B = c.get_fields()
        print(f"[gpu] plain pic step {d['step']}: live {d['n_live']} absorbed {d['n_absorbed']} "
              f"dce rel {d['dce_max_rel']:.2e} gauss drift {d['gauss_max_drift']:.3e} / {d['gauss_scale']:.3e} "
              f"relL2 E {_rel_l2(E, sim.E):.2e} B {_rel_l2(B, sim.B):.2e}", flush=True)
        assert d["dce_max_rel"] <= 1e-12
        assert d["gauss_max_drift"] <= 1e-13 * d["gauss_scale"]
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0
    assert _rel_l2(E, sim.E) <= 1e-9
    assert _rel_l2(B, sim.B) <= 1e-9
    assert d["n_absorbed"] == int(sim.stats[1])


def test_plain_and_mixed_agree_on_energy(axp, cavity):
    """Both precisions advance the same scheme: over 200 diagnostic steps
    their energy records agree to the mixed step's FP32 level."""
    m, _, E0, B0 = cavity
    zr, u = configs.cavity_beam(4000, seed=9)
    out = {}
    for prec in (axp.PREC_PLAIN_FP64, axp.PREC_MIXED):
        c = axp.make_ctx(m, precision=prec, dt=configs.CAVITY_DT, diag_every=1)
        c.set_fields(E0, B0)
        sp = c.add_species(QE, ME, configs.CAVITY_WEIGHT)
        c.inject(sp, zr, u)
        c.step(200)
        out[prec] = (c.energies(), c.diag())
        c.close()
    (ra, a), (rb, b) = out[axp.PREC_PLAIN_FP64], out[axp.PREC_MIXED]
    assert len(ra) == len(rb) == 200
    wf = ra["W_E"][0] + ra["W_B"][0]
    assert np.abs(rb["W_E"] - ra["W_E"]).max() <= 5e-5 * wf
    assert np.abs(rb["W_B"] - ra["W_B"]).max() <= 5e-5 * wf
    assert np.abs(rb["W_K"] - ra["W_K"]).max() <= 2e-5 * ra["W_K"].max()
    assert np.array_equal(ra["n_live"], rb["n_live"])
    assert a["n_absorbed"] == b["n_absorbed"]


def test_plain_graph_replay_matches_eager(axp, cavity):
    """Steps replayed from graphs advance the FP64 state as the eager steps
    do; only the order of the FP64 atomic sums differs, so the bound is FP64
    rounding carried through 48 steps."""
    m, _, E0, B0 = cavity
    zr, u = configs.cavity_beam(4000, seed=5)
    out = []
    for g in (0, 1):
        c = _ctx(axp, m, use_graph=g, sort_period=2)
        c.set_fields(E0, B0)
        sp = c.add_species(QE, ME, configs.CAVITY_WEIGHT)
        c.inject(sp, zr, u)
        c.step(48)
        E, B = c.get_fields()
        zr_g, u_g, _ = c.get_particles()
        o = np.lexsort((u_g[:, 2], zr_g[:, 1], zr_g[:, 0]))
        out.append((E, B, zr_g[o], u_g[o], c.diag()))
        c.close()
    (Ea, Ba, za, ua, da), (Eb, Bb, zb, ub, db) = out
    assert da["step"] == db["step"] == 48
    assert len(za) == len(zb)
    assert _rel_l2(Eb, Ea) <= 1e-11
    assert _rel_l2(Bb, Ba) <= 1e-11
    assert np.abs(zb - za).max() <= 1e-13
    assert np.abs(ub - ua).max() <= 1e-11 * np.abs(ua).max()
