"""Parity with the FP64 oracle at the benchmarked scale, over many steps, in
the launch configuration the benchmark times.

Tube: two ripple periods of the benchmarked tube (32,123 faces, h = 0.19 mm,
the same mesh generator and seed) at the benchmark's beam density
(1,200,000 macro-electrons, ~37 per face as in the full tube), B_z = 1 T,
mixed precision, sort period 16, 64 steps replayed from HIP graphs (two
32-step windows) with a diagnostic step every step.  The beam's head leaves
through the open end, so absorption at a port is part of the run.

Diode: the benchmarked diode (20,485 faces, 100 kV over 1 cm, emitter rho <
2 cm), 2,000 electrons emitted per step with the benchmark's weight, sort
period 8, graphs, diagnostics every 8 steps, 400 steps (800,000 live at the
end; the first electrons reach the anode only after ~1,300 steps, so
absorption at the anode is left to the 1 mm diode of test_gpu_inject.py).
Both precisions; the mixed step's particle bounds are stated against the
oracle's own sensitivity (see the test).

Checks after the run: every particle paired with the oracle's (mutual
nearest neighbours in position and momentum, each scaled by its expected
error), positions and momenta within
the bounds below; E and B rel-L2 <= 1e-5; the edge currents J dt to 1e-5 of
the largest; live and absorbed counts (a particle that one side keeps and
the other absorbs must end within rounding of the port); continuity exact at
every step and the Gauss residual's drift at FP64 rounding of D; the energy
records of the diagnostic steps against the oracle's energies of the same
levels (field energies to 1e-5 of the largest field energy of the run, W_K
to 2e-5).

Bounds.  Positions are fixed point in the element (quantum h 2^-23 ~ 2e-11
m), so their error comes from the FP32 momenta.  A Boris push rounds u four
times (two half kicks, the two products of the rotation), each by up to
2^-24 ~ 6e-8 relative:
  - tube (|u| constant, ~1.8e-5 m a step): momenta 4 n 6e-8 ~ 1.5e-5 after
    n = 64 steps, bound 3e-5 (measured 1.2e-5); positions n^2/2 * 2.4e-7 *
    1.8e-5 m ~ 9e-9 m, bound 2e-8 m (measured 3.5e-9 m);
  - diode: FP32 bounds 4e-8 m and 3e-5 for the bulk of the particles.
The fields start at zero (tube) or at the applied field (diode) and the
beam's own fields carry the FP32 rounding of the gather and SpMV (measured
rel-L2 ~1e-6).
"""

import numpy as np
import pytest
import scipy.spatial

import synth
from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS
C_LIGHT = 299792458.0


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _pair(zr_g, u_g, zr_o, u_o, pos_scale, mom_scale):
    """Mutual nearest neighbours in (position / pos_scale, momentum /
    mom_scale), the scales being the expected errors, so that a particle's
    partner is far closer than its neighbours (~7 um apart at this density,
    with nearly equal momenta in the cold beam); returns the paired indices
    on both sides and the unpaired ones."""
    sa = np.concatenate([zr_g / pos_scale, u_g / mom_scale], axis=1)
    sb = np.concatenate([zr_o / pos_scale, u_o / mom_scale], axis=1)
    _, go = scipy.spatial.cKDTree(sb).query(sa)
    _, og = scipy.spatial.cKDTree(sa).query(sb)
    mutual = og[go] == np.arange(len(go))
    ig = np.flatnonzero(mutual)
    io = go[ig]
    un_g = np.flatnonzero(~mutual)
    un_o = np.setdiff1d(np.arange(len(zr_o)), io)
    return ig, io, un_g, un_o


def _particles(c, sim, z_port, pos_bound, mom_bound, what):
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = sim.particles()
    umax = np.abs(u_o).max()
    ig, io, un_g, un_o = _pair(zr_g, u_g, zr_o, u_o, pos_bound, mom_bound * umax)
    ez = np.abs(zr_g[ig] - zr_o[io]).max(axis=1)
    eu = np.abs(u_g[ig] - u_o[io]).max(axis=1) / umax
    dz, du = ez.max(), eu.max()
    print(f"[gpu] {what}: {len(ig)} particles paired, unpaired {len(un_g)} (GPU) / {len(un_o)} (oracle); "
          f"positions {dz:.2e} m, momenta {du:.2e} of the largest", flush=True)
    for q in np.argsort(ez)[-4:][::-1]:
        print(f"[gpu]   worst pair: GPU zr {zr_g[ig[q]].tolist()} u {u_g[ig[q]].tolist()}; "
              f"oracle zr {zr_o[io[q]].tolist()} u {u_o[io[q]].tolist()}", flush=True)
    for q in un_g[:4]:
        print(f"[gpu]   unpaired GPU particle zr {zr_g[q].tolist()} u {u_g[q].tolist()}", flush=True)
    for q in un_o[:4]:
        print(f"[gpu]   unpaired oracle particle zr {zr_o[q].tolist()} u {u_o[q].tolist()}", flush=True)
    assert dz < pos_bound and du < mom_bound
    # only a wall decision taken in FP32 here and in FP64 by the oracle may
    # differ, for particles that end within rounding of the port
    assert len(un_g) <= 4 and len(un_o) <= 4
    band = 2 * pos_bound + 1e-9
    if len(un_g):
        assert np.all(np.abs(zr_g[un_g, 0] - z_port) < band)
    if len(un_o):
        assert np.all(np.abs(zr_o[un_o, 0] - z_port) < band)
    return len(zr_g), len(zr_o)


def _compare_energies(rec, log, what):
    """GPU energy records against the oracle's log rows of the same levels
    (a particle or two decided differently at a port moves W_K by ~1e-6)."""
    rows = log[rec["step"]]
    assert np.array_equal(rows[:, 0].astype(np.int64), rec["step"])
    wf = max(np.abs(log[:, 1] + log[:, 2]).max(), 1e-300)
    dwe = np.abs(rec["W_E"] - rows[:, 1]).max() / wf
    dwb = np.abs(rec["W_B"] - rows[:, 2]).max() / wf
    wk = rows[:, 3]
    k = wk > 0
    dwk = (np.abs(rec["W_K"][k] - wk[k]) / wk[k]).max() if k.any() else 0.0
    print(f"[gpu] {what}: {len(rec)} energy records, max |dW_E| {dwe:.2e}, |dW_B| {dwb:.2e} of the field "
          f"energy, |dW_K| {dwk:.2e}", flush=True)
    assert dwe <= 1e-5 and dwb <= 1e-5 and dwk <= 2e-5


def test_tube_two_periods_64_steps(axp):
    from oracle.pic import OracleSim
    m = configs.bwo_mesh(seed=3, n_periods=2, up=0.0, down=0.0)
    L = m.meta["length"]
    n = int(round(8_000_000 * (L - 0.001) / (0.217 - 0.001)))
    zr, u = configs.bwo_beam(n, L, seed=3)
    w = configs.bwo_weight(n, L)
    print(f"[gpu] tube slice: {m.n_tris} faces, {n} particles; oracle setup", flush=True)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, bz=configs.BWO_BZ)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.inject(sim.add_species(QE, ME, w), zr, u)
    sim.log_energies = True

    c = axp.make_ctx(m, dt=sim.dt, sort_period=16, use_graph=1, diag_every=1)
    assert c.info()["n_edges"] == sim.topo.n1
    c.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    c.set_external_bz(configs.BWO_BZ)
    c.inject(c.add_species(QE, ME, w), zr, u)
    recs = []
    for chunk in range(2):
        print(f"[gpu] tube slice: 32 steps (graph window {chunk})", flush=True)
        c.step(32)
        recs.append(c.energies())
        d = c.diag()
        assert d["dce_max_abs"] == 0 and d["walk_overflow"] == 0 and d["nan_count"] == 0
        assert d["gauss_max_drift"] <= 1e-13 * d["gauss_scale"]
    print("[gpu] tube slice: oracle 64 steps", flush=True)
    sim.step(64)
    rec = np.concatenate(recs)
    assert np.array_equal(rec["step"], np.arange(64))
    _compare_energies(rec, np.array(sim.energy_log), "tube slice")

    absorbed_o = int(sim.stats[1])
    n_g, n_o = _particles(c, sim, L, 2e-8, 3e-5, "tube slice")
    print(f"[gpu] tube slice: live {n_g} / oracle {n_o}, absorbed {d['n_absorbed']} / oracle {absorbed_o}",
          flush=True)
    assert absorbed_o > 1000                       # the beam's head has left through the port
    assert n_g + d["n_absorbed"] == n_o + absorbed_o == n
    assert abs(d["n_absorbed"] - absorbed_o) <= 4
    E, B = c.get_fields()
    D, Jdt, Q = c.get_sources()
    Jdt_o = sim.J * sim.dt
    eE, eB = _rel_l2(E, sim.E), _rel_l2(B, sim.B)
    eJ = np.abs(Jdt - Jdt_o).max() / np.abs(Jdt_o).max()
    print(f"[gpu] tube slice: rel-L2 E {eE:.2e} B {eB:.2e}, J dt {eJ:.2e} of the largest", flush=True)
    assert eE <= 1e-5 and eB <= 1e-5 and eJ <= 1e-5
    c.close()


def _diode_oracle(m, dt, E0, w, per_step, u_emit, M=None):
    from oracle.pic import OracleSim
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=dt, M=M)
    sim.set_fields(E0, np.zeros(sim.topo.n2))
    sim.set_injector(sim.add_species(QE, ME, w), per_step, u_emit, 0.0, seed=11)
    return sim


DIODE_STEPS, DIODE_PER_STEP = 400, 2000


@pytest.fixture(scope="module")
def diode(axp):
    """The benchmarked diode and the oracle's 400 steps of it."""
    EPS0 = 8.8541878128e-12
    V, d_gap, Re = configs.DIODE_VOLTS, configs.DIODE_GAP, 0.02
    I_cl = 4 * EPS0 / 9 * np.sqrt(2 * abs(QE) / ME) * V ** 1.5 / d_gap ** 2 * np.pi * Re ** 2
    u_emit = np.array([0.0, 0.0, np.sqrt((1 + 1.0 / 511e3) ** 2 - 1) * C_LIGHT])
    m = configs.diode_mesh()
    c = axp.make_ctx(m)
    dt, edges = c.info()["dt"], c.get_edges()
    c.close()
    phi = V * m.nodes[:, 0] / d_gap
    E0 = -(phi[edges[:, 1]] - phi[edges[:, 0]])
    w = int(round(2 * I_cl * dt / (DIODE_PER_STEP * abs(QE))))
    print(f"[gpu] diode: {m.n_tris} faces; oracle setup and {DIODE_STEPS} steps", flush=True)
    sim = _diode_oracle(m, dt, E0, w, DIODE_PER_STEP, u_emit)
    assert np.array_equal(edges, sim.topo.edges)
    sim.log_energies = True
    sim.step(DIODE_STEPS)
    return dict(m=m, dt=dt, E0=E0, w=w, u_emit=u_emit, sim=sim, d_gap=d_gap)


@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_diode_400_steps(axp, diode, prec):
    """FP64 step: the oracle's result to FP64 rounding, particle by particle
    (positions 1e-11 m, momenta 1e-9 of the largest, fields and currents
    1e-9, as for the 1 mm diode).

    Mixed step: the space-charge-limited diode has particles whose paths
    fork: a position within rounding of a face side picks the face whose
    Whitney field the next gather samples, and the normal component jumps
    there.  The oracle shows it against itself: a second oracle run whose
    applied field differs by FP32 rounding (2^-24 relative, once, at t = 0)
    keeps all but ~5 of the 800,000 particles within 2e-11 m and 2e-8 and
    moves those few by up to 1e-7 m and 3e-4.  The mixed step rounds in FP32
    at every step, so more paths fork.  Bounds: 99.9 % of the particles
    within the FP32 bounds (4e-8 m, 3e-5), at most 0.1 % beyond them, none
    beyond 10 times the oracle's own largest excursion; E (applied plus space
    charge) to rel-L2 1e-5; the beam's own B_phi, which integrates the
    current of the forked paths, to 1e-3 and the edge currents to 2e-4 of the
    largest (measured 1.1e-4 and 1.8e-5); the energies as in the tube."""
    tight = prec == "plain"
    sim = diode["sim"]
    m, dt = diode["m"], diode["dt"]
    c = axp.make_ctx(m, dt=dt, sort_period=8, diag_every=8,
                     precision=axp.PREC_PLAIN_FP64 if tight else axp.PREC_MIXED)
    c.set_fields(diode["E0"], np.zeros(c.info()["n_faces"]))
    c.set_injector(c.add_species(QE, ME, diode["w"]), DIODE_PER_STEP, diode["u_emit"], 0.0, 11)
    recs = []
    for chunk in range(5):
        print(f"[gpu] diode {prec}: steps {80 * chunk}..{80 * chunk + 79}", flush=True)
        c.step(80)
        recs.append(c.energies())
        d = c.diag()
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0
        if tight:
            assert d["dce_max_rel"] <= 1e-12
        else:
            assert d["dce_max_abs"] == 0
        assert d["gauss_max_drift"] <= 1e-13 * d["gauss_scale"]
    rec = np.concatenate(recs)
    assert np.array_equal(rec["step"], np.arange(7, DIODE_STEPS, 8))
    _compare_energies(rec, np.array(sim.energy_log), f"diode {prec}")
    assert d["n_absorbed"] == int(sim.stats[1]) == 0
    E, B = c.get_fields()
    D, Jdt, Q = c.get_sources()
    Jdt_o = sim.J * sim.dt
    eE, eB = _rel_l2(E, sim.E), _rel_l2(B, sim.B)
    eJ = np.abs(Jdt - Jdt_o).max() / np.abs(Jdt_o).max()
    print(f"[gpu] diode {prec}: rel-L2 E {eE:.2e} B {eB:.2e}, J dt {eJ:.2e} of the largest", flush=True)
    zr_o, u_o, _ = sim.particles()
    zr_g, u_g, _ = c.get_particles()
    n = DIODE_STEPS * DIODE_PER_STEP
    assert len(zr_g) == len(zr_o) == n
    umax = np.abs(u_o).max()
    if tight:
        assert eE <= 1e-9 and eB <= 1e-9 and eJ <= 1e-9
        n_g, n_o = _particles(c, sim, diode["d_gap"], 1e-11, 1e-9, f"diode {prec}")
        c.close()
        return
    assert eE <= 1e-5 and eB <= 1e-3 and eJ <= 2e-4

    print("[gpu] diode: oracle against itself, applied field rounded to FP32", flush=True)
    rng = np.random.default_rng(5)
    E0s = diode["E0"] * (1 + 2.0 ** -24 * rng.uniform(-1, 1, len(diode["E0"])))
    sim2 = _diode_oracle(m, dt, E0s, diode["w"], DIODE_PER_STEP, diode["u_emit"], M=sim.M)
    sim2.step(DIODE_STEPS)
    zr_s, u_s, _ = sim2.particles()
    POS, MOM = 4e-8, 3e-5
    ez_s = np.abs(zr_s - zr_o).max(axis=1)
    eu_s = np.abs(u_s - u_o).max(axis=1) / umax
    far_s = int(((ez_s > POS) | (eu_s > MOM)).sum())
    print(f"[gpu] diode: oracle vs itself: {far_s} particles beyond ({POS} m, {MOM}), largest {ez_s.max():.2e} m, "
          f"{eu_s.max():.2e}; rel-L2 E {_rel_l2(sim2.E, sim.E):.2e} B {_rel_l2(sim2.B, sim.B):.2e}", flush=True)
    ig, io, un_g, un_o = _pair(zr_g, u_g, zr_o, u_o, POS, MOM * umax)
    ez = np.abs(zr_g[ig] - zr_o[io]).max(axis=1)
    eu = np.abs(u_g[ig] - u_o[io]).max(axis=1) / umax
    far = int(((ez > POS) | (eu > MOM)).sum()) + len(un_g)
    print(f"[gpu] diode mixed: {len(ig)} paired, {len(un_g)} unpaired, {far} beyond the FP32 bounds, "
          f"largest {ez.max():.2e} m, {eu.max():.2e}; 99.9 % {np.quantile(ez, 0.999):.2e} m, "
          f"{np.quantile(eu, 0.999):.2e}", flush=True)
    assert np.quantile(ez, 0.999) < POS and np.quantile(eu, 0.999) < MOM
    assert far <= 1e-3 * n
    assert ez.max() <= 10 * max(ez_s.max(), POS) and eu.max() <= 10 * max(eu_s.max(), MOM)
    c.close()
