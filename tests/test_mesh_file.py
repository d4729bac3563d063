"""The text mesh format of axp_spai_model_train (CPU): write_mesh output
holds the header, the counts and every node, triangle and tagged segment,
and the coordinates read back exactly."""

import numpy as np

import paper_1701_03784_amd as axp
from synth import configs


def test_write_mesh_round_trip(tmp_path):
    m = configs.bwo_mesh(seed=310, h=0.5e-3, amp=0.0012, period=0.013, n_periods=2, up=0.004, down=0.004)
    p = tmp_path / "tube.mesh"
    axp.write_mesh(p, m)
    tok = p.read_text().split()
    assert tok[:2] == ["axpic-mesh", "1"]
    nn, nt, ns = map(int, tok[2:5])
    assert (nn, nt, ns) == (m.n_nodes, m.n_tris, len(m.seg))
    v = tok[5:]
    assert len(v) == 2 * nn + 3 * nt + 3 * ns
    nodes = np.array(v[:2 * nn], dtype=np.float64).reshape(-1, 2)
    tris = np.array(v[2 * nn:2 * nn + 3 * nt], dtype=np.int64).reshape(-1, 3)
    seg = np.array(v[2 * nn + 3 * nt:], dtype=np.int64).reshape(-1, 3)
    assert np.array_equal(nodes, m.nodes)
    assert np.array_equal(tris, m.tris)
    assert np.array_equal(seg[:, :2], m.seg) and np.array_equal(seg[:, 2], m.tag)
