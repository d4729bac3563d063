"""Vay's pusher on the GPU (both precisions) against the FP64 oracle's.

Workload: the diode mesh (h = 1 mm) with a static radial field
E_rho = E0 rho / R (edge values from the potential -E0 rho^2 / (2 R), zero
on conductor edges), E0 = 320 MV/m at R = 1 cm, and B_z = 2 T; 3,000
electrons drifting at the local E x B velocity (0.27 c to 0.8 c).  There the
Boris push differs from Vay's by 5e-5 of |u| after one step and 4e-2 after
20 (the spurious force of the Boris rotation at a relativistic drift), so
the bounds below tell the two apart.  Bounds after 20 steps: positions
1e-8 m (mixed: FP32 momenta, 2^-23 element-local coordinates) / 1e-12 m
(FP64); momenta 1e-5 / 1e-10 of the largest; fields rel-L2 1e-5 / 1e-9;
continuity exact in fixed point / 1e-12 of max |Q|.
"""

import numpy as np
import pytest
import scipy.spatial

import synth
from synth import configs

pytestmark = pytest.mark.gpu

QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS
C = 299792458.0
BZ, E0, R = 2.0, 3.2e8, 0.01
STEPS = 20


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def drift():
    from oracle.pic import OracleSim
    m = configs.diode_mesh(h=1.0e-3)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    phi = -E0 * m.nodes[:, 1] ** 2 / (2 * R)
    ed = sim.topo.edges
    Ee = np.where(sim.topo.edge_free, -(phi[ed[:, 1]] - phi[ed[:, 0]]), 0.0)
    rng = np.random.default_rng(4)
    n = 3000
    rho = rng.uniform(0.005, 0.015, n)
    z = rng.uniform(0.002, 0.008, n)
    vd = -(E0 * rho / R) / BZ               # E x B / B^2 along phi-hat
    g = 1.0 / np.sqrt(1.0 - (vd / C) ** 2)
    u = np.stack([np.zeros(n), g * vd, np.zeros(n)], 1)
    zr = np.stack([z, rho], 1)
    runs = {}
    for pusher in (0, 1):
        o = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim.dt, M=sim.M)
        o.pusher = pusher
        o.bz = BZ
        o.set_fields(Ee, np.zeros(o.topo.n2))
        o.add_species(QE, ME, 1000)
        o.inject(0, zr, u)
        o.step(STEPS)
        runs[pusher] = o
    return m, sim.dt, Ee, zr, u, runs


def _match(zr_a, u_a, zr_b, u_b):
    sa = np.concatenate([zr_a / 1e-6, u_a / 1e5], axis=1)
    sb = np.concatenate([zr_b / 1e-6, u_b / 1e5], axis=1)
    _, idx = scipy.spatial.cKDTree(sb).query(sa)
    assert len(np.unique(idx)) == len(idx)
    return idx


def test_the_workload_tells_the_pushers_apart(drift):
    _, _, _, _, _, runs = drift
    # the oracle keeps its particles in injection order; none is absorbed here
    assert runs[0].stats[1] == runs[1].stats[1] == 0
    zb, ub, _ = runs[0].particles()
    zv, uv, _ = runs[1].particles()
    assert np.abs(ub - uv).max() > 100 * 1e-5 * np.abs(uv).max()
    assert np.abs(zb - zv).max() > 100 * 1e-8


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_vay_parity(axp, drift, prec):
    m, dt, Ee, zr, u, runs = drift
    o = runs[1]
    tight = prec == "plain"
    print(f"[gpu] vay parity {prec}", flush=True)
    c = axp.make_ctx(m, dt=dt, precision=axp.PREC_PLAIN_FP64 if tight else axp.PREC_MIXED,
                     pusher=axp.PUSH_VAY, diag_every=1)
    c.set_fields(Ee, np.zeros(c.info()["n_faces"]))
    c.set_external_bz(BZ)
    sp = c.add_species(QE, ME, 1000)
    c.inject(sp, zr, u)
    c.diag()
    for _ in range(STEPS):
        c.step(1)
        d = c.diag()
        if tight:
            assert d["dce_max_rel"] <= 1e-12
        else:
            assert d["dce_max_abs"] == 0
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = o.particles()
    assert len(zr_g) == len(zr_o) and d["n_absorbed"] == int(o.stats[1])
    idx = _match(zr_g, u_g, zr_o, u_o)
    dz = np.abs(zr_g - zr_o[idx]).max()
    du = np.abs(u_g - u_o[idx]).max() / np.abs(u_o).max()
    E, B = c.get_fields()
    rel = float(np.linalg.norm(E - o.E) / np.linalg.norm(o.E))
    print(f"[gpu] vay {prec}: max dpos {dz:.2e} m, max du/|u| {du:.2e}, E rel-L2 {rel:.2e}", flush=True)
    assert dz < (1e-12 if tight else 1e-8)
    assert du < (1e-10 if tight else 1e-5)
    assert rel <= (1e-9 if tight else 1e-5)
    c.close()


def test_batch_needs_one_pusher(axp):
    m = configs.cavity_mesh()
    a = axp.make_ctx(m, dt=configs.CAVITY_DT)
    b = axp.make_ctx(m, dt=configs.CAVITY_DT, pusher=axp.PUSH_VAY)
    for c in (a, b):
        c.add_species(QE, ME, 1000)
    with pytest.raises(axp.AxpError):
        axp.Batch([a, b])
    a.close()
    b.close()
