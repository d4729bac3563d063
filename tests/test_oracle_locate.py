"""Pin of the oracle's point location (CPU): for random interior points,
edge midpoints and mesh vertices, OracleSim.locate returns a face that
contains the point (smallest barycentric coordinate >= -1e-12).  Away
from faces' boundaries it is the face a brute-force scan of every face
finds; on an edge or a vertex every containing face is acceptable, so only
containment is checked there."""

import numpy as np

from synth import configs
from oracle.pic import OracleSim
from oracle.topology import build_topology


def _bary_min(nodes, tri, p):
    a, b, c = nodes[tri[:, 0]], nodes[tri[:, 1]], nodes[tri[:, 2]]
    det = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (b[:, 1] - a[:, 1])
    l1 = ((p[..., 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (c[:, 0] - a[:, 0]) * (p[..., 1] - a[:, 1])) / det
    l2 = ((b[:, 0] - a[:, 0]) * (p[..., 1] - a[:, 1]) - (p[..., 0] - a[:, 0]) * (b[:, 1] - a[:, 1])) / det
    return np.minimum(np.minimum(1.0 - l1 - l2, l1), l2)


def test_locate_against_brute_force():
    m = configs.bwo_mesh(seed=5, h=0.6e-3, n_periods=2, up=0.005, down=0.005)
    # locate needs only the topology: skip the SPAI and stability setup
    sim = OracleSim.__new__(OracleSim)
    sim.topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    sim._tree = None
    rng = np.random.default_rng(4)
    area = m.signed_areas()
    t = rng.choice(len(area), 3000, p=area / area.sum())
    a, b = rng.uniform(0.01, 0.98, size=(2, 3000))
    f = a + b > 0.99
    a[f], b[f] = 0.99 - a[f], 0.99 - b[f]
    P = m.nodes[m.tris[t]]
    inner = P[:, 0] + a[:, None] * (P[:, 1] - P[:, 0]) + b[:, None] * (P[:, 2] - P[:, 0])
    mids = 0.5 * (m.nodes[m.tris[:, 0]] + m.nodes[m.tris[:, 1]])[rng.choice(len(m.tris), 1000, replace=False)]
    verts = m.nodes[rng.choice(len(m.nodes), 1000, replace=False)]
    tris = np.asarray(m.tris, dtype=np.int64)
    for pts, exact in ((inner, True), (mids, False), (verts, False)):
        got = sim.locate(pts)
        own = np.array([_bary_min(m.nodes, tris[[g]], q[None, :])[0] for g, q in zip(got, pts)])
        assert own.min() >= -1e-12
        if exact:
            brute = np.array([int(np.argmax(_bary_min(m.nodes, tris, q[None, :]))) for q in pts])
            assert np.array_equal(got, brute)
