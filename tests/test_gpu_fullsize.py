"""The full-size tube workload, in the launch configuration of the benchmark,
against the FP64 oracle on what the oracle can compute at that size.

Workload: the rippled-wall tube of ten periods plus drifts (207,935 faces,
313,136 edges, h = 0.19 mm), 8,000,000 macro-electrons of the 500 keV
annular beam, B_z = 1 T, SPAI level 3, mixed precision, sort period 16,
steps replayed from HIP graphs; dt = 6e-14 s on both sides.

One step from E^0 = 0 (so D^0 = 0) and a seeded smooth B_phi at t^{-1/2}
uses [*eps]^-1 only in its last line, E^1 = M D^1.  So the oracle runs the
whole step, with an identity stand-in for M whose E^1 is not used, and the
check covers:
  - every particle: a 200,000-particle sample of the library's, each matched
    to the oracle's nearest in position and momentum, positions to 1e-8 m
    and momenta to 1e-5 of the largest, the same live and absorbed counts;
  - every edge current J dt and every D^1, to 1e-5 of the largest;
  - B^{1/2} on every face, to FP32 rounding;
  - E^1 on 200 sampled free edges, against those rows of the oracle's SPAI
    (computed alone, from the column problems they need) applied to the
    oracle's D^1, to 1e-5 of the row's sum of |M| |D|;
  - the same rows of the library's SPAI, to 1e-12.
Then, after 15 more eager steps, 64 steps replayed from graphs (two
32-step windows) equal the same steps launched eagerly, bit for bit, with
continuity exact, no overflow or non-finite value, and the particle count
conserved.
"""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.spatial

import synth
from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N = 8_000_000
DT = 6.0e-14
SORT = 16
QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


@pytest.fixture(scope="module")
def tube():
    m = configs.bwo_mesh(seed=3)
    L = m.meta["length"]
    zr, u = configs.bwo_beam(N, L, seed=3)
    w = configs.bwo_weight(N, L)
    B0 = synth.face_flux_integrals(m.nodes, m.tris,
                                   lambda z, r: 0.05 * (r / 0.015) * np.sin(2 * np.pi * z / 0.0167))
    return m, zr, u, w, B0


@pytest.fixture(scope="module")
def oracle_one_step(tube):
    from oracle.pic import OracleSim
    m, zr, u, w, B0 = tube
    n1 = len(synth.canonical_edges(m.tris))
    print(f"[gpu] full size: oracle setup ({m.n_tris} faces, {n1} edges)", flush=True)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=DT, bz=configs.BWO_BZ, M=sp.identity(n1, format="csr"))
    sim.set_fields(np.zeros(n1), B0)
    sim.add_species(QE, ME, w)
    sim.inject(0, zr, u)
    print(f"[gpu] full size: oracle step of {N} particles", flush=True)
    sim.step(1)
    return sim


def _ctx(axp, tube, use_graph):
    m, zr, u, w, B0 = tube
    c = axp.make_ctx(m, dt=DT, sort_period=SORT, use_graph=use_graph)
    c.set_fields(np.zeros(c.info()["n_edges"]), B0)
    c.set_external_bz(configs.BWO_BZ)
    sp_ = c.add_species(QE, ME, w)
    c.inject(sp_, zr, u)
    return c


@pytest.fixture(scope="module")
def graph_ctx(axp, tube):
    c = _ctx(axp, tube, 1)
    print("[gpu] full size: library step 1", flush=True)
    c.step(1)
    yield c
    c.close()


def test_one_full_size_step_matches_the_oracle(axp, graph_ctx, oracle_one_step):
    from oracle.spai import spai_rows
    c, sim = graph_ctx, oracle_one_step
    d = c.diag()
    assert d["dce_max_abs"] == 0 and d["walk_overflow"] == 0 and d["nan_count"] == 0
    assert d["n_absorbed"] == int(sim.stats[1])
    # particles
    zr_g, u_g, _ = c.get_particles()
    zr_o, u_o, _ = sim.particles()
    assert len(zr_g) == len(zr_o) == d["n_live"]
    rng = np.random.default_rng(7)
    pick = rng.choice(len(zr_g), 200_000, replace=False)
    tree = scipy.spatial.cKDTree(np.concatenate([zr_o / 1e-6, u_o / 1e3], axis=1))
    _, idx = tree.query(np.concatenate([zr_g[pick] / 1e-6, u_g[pick] / 1e3], axis=1))
    assert len(np.unique(idx)) == len(idx)
    e_pos = np.abs(zr_g[pick] - zr_o[idx]).max()
    e_u = np.abs(u_g[pick] - u_o[idx]).max() / np.abs(u_o).max()
    # currents, D^1, B^{1/2}
    E_g, B_g = c.get_fields()
    D_g, Jdt_g, _ = c.get_sources()
    Jdt_o = sim.J * sim.dt
    e_J = np.abs(Jdt_g - Jdt_o).max() / np.abs(Jdt_o).max()
    e_D = np.abs(D_g - sim.D).max() / np.abs(sim.D).max()
    e_B = np.abs(B_g - sim.B).max() / np.abs(sim.B).max()
    # E^1 on sampled rows, and those rows of the SPAI
    rows = np.sort(rng.choice(np.flatnonzero(sim.topo.edge_free), 200, replace=False))
    Mr = spai_rows(sim.A, sim.topo.edge_free, rows)
    E_ref = Mr @ sim.D
    scale = abs(Mr) @ np.abs(sim.D)
    e_E = (np.abs(E_g[rows] - E_ref) / np.maximum(scale, 1e-300)).max()
    Mg = c.get_spai().tocsr()[rows]
    e_M = abs(Mg - Mr).max() / abs(Mr).max()
    print(f"[gpu] full size step 1: positions {e_pos:.1e} m, momenta {e_u:.1e}, J {e_J:.1e}, D {e_D:.1e}, "
          f"B {e_B:.1e}, E rows {e_E:.1e}, M rows {e_M:.1e}", flush=True)
    assert e_pos < 1e-8 and e_u < 1e-5
    assert e_J <= 1e-5 and e_D <= 1e-5
    assert e_B <= 1e-7
    assert e_E <= 1e-5
    assert e_M <= 1e-12


def _state(c):
    E, B = c.get_fields()
    D, J, Q = c.get_sources()
    zr, u, sp_ = c.get_particles()
    order = np.lexsort((u[:, 2], u[:, 1], u[:, 0], zr[:, 1], zr[:, 0]))
    return dict(E=E, B=B, D=D, J=J, Q=Q, zr=zr[order], u=u[order], sp=sp_[order])


def test_graph_replays_at_full_size_equal_eager_steps(axp, tube, graph_ctx):
    """Up to step SORT eagerly (graph windows start at multiples of the sort
    period), then 4 SORT steps: two replays of a 2 SORT-step graph."""
    c = graph_ctx
    c.step(SORT - 1)
    c.step(4 * SORT)
    dg = c.diag()
    ce = _ctx(axp, tube, 0)
    ce.step(1)
    ce.step(SORT - 1)
    ce.step(4 * SORT)
    de = ce.diag()
    print(f"[gpu] full size: {dg['step']} steps, live {dg['n_live']}, absorbed {dg['n_absorbed']}", flush=True)
    for dd in (dg, de):
        assert dd["dce_max_abs"] == 0 and dd["walk_overflow"] == 0 and dd["nan_count"] == 0
        assert dd["fixed_overflow"] == 0
        assert dd["n_live"] + dd["n_absorbed"] == N
    assert dg["step"] == de["step"] == 5 * SORT
    a, b = _state(c), _state(ce)
    for k in a:
        assert np.array_equal(a[k], b[k]), (k, float(np.abs(a[k] - b[k]).max()))
    ce.close()
