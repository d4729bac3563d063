"""Nodes with long incident lists in the node pass of the evaluations.

The node pass gathers each node's face corners and edges from padded lists,
a few entries per round.  The meshes of the workloads have at most eight
per node; here the cavity's rectangle has three nodes with 13, 14 and 15
faces (each the centre of a ring of lattice points), so the gather runs
four rounds there.  With a beam crossing them and a diagnostic step every
step, in both precisions:
- the nodal charge the in-step evaluation leaves (axp_get_sources) equals
  the charge of the particles' positions spread to the corners of their
  faces by their barycentric coordinates (the definition of the charge
  deposit, eq. charge, computed here with numpy: Delaunay point location on
  the same triangles), to the mixed step's coordinate rounding;
- the continuity residual of every evaluation is exactly zero (mixed) or at
  FP64 rounding (plain), and the Gauss residual stays at its reference
  (Sec. 3.5.1-3.5.2): a node that lost an edge or a corner would show both.
"""

import numpy as np
import pytest
import scipy.spatial

import synth
from synth import meshes
from synth.meshes import BC_AXIS, BC_PEC, Mesh

pytestmark = pytest.mark.gpu

QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS
C = 299792458.0
WEIGHT = 1000.0


@pytest.fixture(scope="module")
def axp():
    import paper_1701_03784_amd as pkg
    pkg.load_library()
    return pkg


def star_mesh(h=0.49e-3, z1=0.02, rho1=0.01, centres=((0.006, 0.004), (0.013, 0.006), (0.010, 0.0025)),
              ring=(13, 14, 15)):
    """Hexagonal lattice on the rectangle; the lattice points within 1.6 h of
    each centre are replaced by the centre and a ring of points at 1.1 h, so
    the centre is a vertex of as many faces as the ring has points."""
    rng = np.random.default_rng(5)
    ny = max(2, int(round(rho1 / (h * np.sqrt(3.0) / 2.0))))
    p = meshes._hex_lattice(0.0, z1, h, ny, 0.0, rng) * np.array([1.0, rho1])
    keep = np.ones(len(p), bool)
    extra = []
    for (zc, rc), k in zip(centres, ring):
        keep &= np.hypot(p[:, 0] - zc, p[:, 1] - rc) > 1.6 * h
        a = 2 * np.pi * (np.arange(k) + 0.5) / k
        extra.append([zc, rc])
        extra.extend(np.stack([zc + 1.1 * h * np.cos(a), rc + 1.1 * h * np.sin(a)], axis=1).tolist())
    p = np.concatenate([p[keep], np.array(extra)], axis=0)
    tris = meshes._triangulate(p)
    seg = meshes._boundary_segments(tris)
    a, b = p[seg[:, 0]], p[seg[:, 1]]
    tag = np.where((np.abs(a[:, 1]) < 1e-12) & (np.abs(b[:, 1]) < 1e-12), BC_AXIS, BC_PEC).astype(np.uint8)
    return Mesh(nodes=p.astype(np.float64), tris=tris, seg=seg, tag=tag, meta={"h": h})


def deposited_charge(m, zr, q_per_particle):
    """Nodal charge per radian of particles at zr: q w / (2 pi) spread to the
    corners of each particle's face by its barycentric coordinates."""
    tri = scipy.spatial.Delaunay(m.nodes)
    # the same triangles: locate with an explicit barycentric test on the mesh's own faces
    t = tri.find_simplex(zr)
    assert np.all(t >= 0)
    own = {tuple(sorted(f)): i for i, f in enumerate(m.tris.tolist())}
    face = np.array([own[tuple(sorted(tri.simplices[k]))] for k in t])
    p = m.nodes[m.tris[face]]
    d = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    l1 = ((zr[:, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (zr[:, 1] - p[:, 0, 1])) / d
    l2 = ((p[:, 1, 0] - p[:, 0, 0]) * (zr[:, 1] - p[:, 0, 1]) - (zr[:, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])) / d
    lam = np.stack([1.0 - l1 - l2, l1, l2], axis=1)
    Q = np.zeros(len(m.nodes))
    np.add.at(Q, m.tris[face].ravel(), (lam * (q_per_particle / (2 * np.pi))).ravel())
    return Q


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_nodes_with_long_lists(axp, prec):
    m = star_mesh()
    corners = np.bincount(m.tris.ravel(), minlength=len(m.nodes))
    assert sorted(corners)[-3:] == [13, 14, 15]
    kw = {"precision": axp.PREC_PLAIN_FP64} if prec == "plain" else {}
    c = axp.make_ctx(m, diag_every=1, sort_period=4, **kw)
    info = c.info()
    c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
    # a beam over the three centres (rho 2-7 mm), away from the plates
    rng = np.random.default_rng(11)
    n = 20000
    zr = np.stack([rng.uniform(0.004, 0.016, n), rng.uniform(0.0015, 0.0075, n)], axis=1)
    u = rng.normal(0.0, 0.05 * C, (n, 3))           # gamma v [m/s], |v| of a few per cent of c
    c.inject(c.add_species(QE, ME, WEIGHT), zr, u)
    q0 = c.diag()["Q_total"]
    zr0, _, _ = c.get_particles()
    print(f"[gpu] {prec}: {len(m.tris)} faces, longest node lists {corners.max()}", flush=True)
    for k in range(3):
        c.step(8)
        d = c.diag()
        D, J, Q = c.get_sources()
        zr_now, _, _ = c.get_particles()
        moved = np.abs(np.sort(zr_now[:, 0]) - np.sort(zr0[:, 0])).max()
        print(f"[gpu] {prec}: particles moved up to {moved:.2e} m in z, |J dt| max {np.abs(J).max():.2e} C/rad",
              flush=True)
        assert moved > 1e-5 and np.abs(J).max() > 0     # the beam moves and carries current
        assert d["walk_overflow"] == 0 and d["nan_count"] == 0 and d["fixed_overflow"] == 0
        Qref = deposited_charge(m, zr_now, QE * WEIGHT)
        scale = np.abs(Qref).max()
        err = np.abs(Q - Qref).max() / scale
        print(f"[gpu] {prec}: step {8 * (k + 1)}: live {d['n_live']}, nodal charge vs deposit {err:.2e}, "
              f"dce {d['dce_max_abs']} / {d['dce_max_rel']:.1e}, gauss drift {d['gauss_max_drift']:.2e} of scale "
              f"{d['gauss_scale']:.2e} (|D| max {np.abs(D).max():.2e}, |Q| max {scale:.2e})", flush=True)
        assert d["n_live"] == n                       # nothing reaches the walls in 24 steps
        assert err <= (1e-6 if prec == "mixed" else 1e-12)
        hub = np.argsort(corners)[-3:]
        assert np.all(np.abs(Qref[hub]) > 1e-3 * scale)   # the beam does cover the centres
        assert d["gauss_max_drift"] <= 1e-12 * d["gauss_scale"]
        if prec == "mixed":
            assert d["dce_max_abs"] == 0
        else:
            assert d["dce_max_rel"] <= 1e-12
        assert abs(d["Q_total"] - q0) <= 1e-12 * abs(q0)
    c.close()
