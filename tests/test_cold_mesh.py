"""Mesh of the cold-test cell (CPU): its conductor wall follows
r0 + amp cos(2 pi z / d) exactly at the wall nodes, the faces are
counter-clockwise, and the wall is mirror-symmetric about z = d/2 (the
plates lie at symmetry planes, which makes the cell's modes Floquet modes
of phase advance 0 and pi)."""

import numpy as np

from paper_1701_03784_amd import cold_test


def test_cell_mesh_follows_the_wall():
    r0, amp, d, h = 0.015, 0.0025, 0.0167, 0.4e-3
    m = cold_test.cell_mesh(r0, amp, d, h)
    assert np.all(m.signed_areas() > 0)
    nodes = np.unique(m.seg[m.tag == 1])
    z, r = m.nodes[nodes, 0], m.nodes[nodes, 1]
    wall = (z > 1e-9) & (z < d - 1e-9) & (r > 0.5 * r0)
    np.testing.assert_allclose(r[wall], r0 + amp * np.cos(2 * np.pi * z[wall] / d), rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.sort(d - z[wall]), np.sort(z[wall]), atol=1e-12)


R0, AMP, D = 0.015, 0.0025, 0.0167


def _wall(z):
    return R0 + AMP * np.cos(2 * np.pi * np.asarray(z) / D)


def _n_edges(m):
    import synth
    return len(synth.canonical_edges(m.tris))


def test_grid_meshes_are_simply_connected_and_positive():
    """Both grid kinds: counter-clockwise faces, V - E + F = 1 (a disc; the
    paper's mesh table satisfies it for every row but one), every edge on
    one or two faces, the axis covered exactly once."""
    for kind in ("grid", "staircase"):
        for h in (0.8e-3, 0.5e-3, 0.3e-3):
            m = cold_test.cell_mesh(R0, AMP, D, h, kind=kind)
            assert np.all(m.signed_areas() > 0)
            assert m.n_nodes - _n_edges(m) + m.n_tris == 1
            t = np.sort(np.concatenate([m.tris[:, [0, 1]], m.tris[:, [1, 2]], m.tris[:, [2, 0]]]), axis=1)
            _, cnt = np.unique(t, axis=0, return_counts=True)
            assert cnt.max() == 2 and (cnt == 1).sum() == len(m.seg)
            ax = m.seg[m.tag == 2]
            assert np.all(m.nodes[ax, 1] == 0.0)
            assert abs(np.abs(np.diff(m.nodes[ax, 0], axis=1)).sum() - D) < 1e-15


def test_mapped_grid_follows_the_wall():
    """Mapped grid: wall nodes on R(z) exactly; the area is the trapezoid sum
    of R over the columns, which a full period of the cosine makes exact."""
    m = cold_test.cell_mesh(R0, AMP, D, 0.4e-3, kind="grid")
    wall = np.unique(m.seg[(m.tag == 1)])
    z, r = m.nodes[wall, 0], m.nodes[wall, 1]
    on = (z > 0) & (z < D)
    np.testing.assert_allclose(r[on], _wall(z[on]), rtol=0, atol=1e-15)
    assert abs(m.signed_areas().sum() - R0 * D) < 1e-15


def test_staircased_wall_is_made_of_grid_lines():
    """Staircase: every wall segment is horizontal or vertical, there are
    vertical risers between the plates, each column's top is the wall
    radius at its centre rounded to whole rows, and the area is the sum of
    the columns; the wall is mirror-symmetric about z = d/2."""
    h = 0.4e-3
    m = cold_test.cell_mesh(R0, AMP, D, h, kind="staircase")
    s = m.seg[m.tag == 1]
    a, b = m.nodes[s[:, 0]], m.nodes[s[:, 1]]
    horiz = a[:, 1] == b[:, 1]
    vert = a[:, 0] == b[:, 0]
    assert np.all(horiz | vert)
    interior_risers = vert & (a[:, 0] > 0) & (a[:, 0] < D)
    assert interior_risers.sum() > 0
    nz = int(round(D / h))
    dz = D / nz
    zc = dz * (np.arange(nz) + 0.5)
    rows = np.rint(_wall(zc) / h)
    top = horiz & (a[:, 1] > 0)
    col = np.minimum(np.floor(0.5 * (a[top, 0] + b[top, 0]) / dz).astype(int), nz - 1)
    np.testing.assert_allclose(a[top, 1], rows[col] * h, rtol=0, atol=1e-15)
    assert len(np.unique(col)) == nz
    assert abs(m.signed_areas().sum() - (rows * h * dz).sum()) < 1e-15
    np.testing.assert_array_equal(rows, rows[::-1])


def test_staircase_of_a_whole_row_cylinder_is_the_mapped_grid():
    """A constant radius that is a whole number of rows has no steps: the
    staircased and the mapped grid are the same mesh."""
    import synth
    R = lambda z: np.full_like(np.asarray(z, dtype=np.float64), 0.012)
    m1 = synth.grid_mesh(R, 0.0, D, 0.4e-3, staircase=False)
    m2 = synth.grid_mesh(R, 0.0, D, 0.4e-3, staircase=True)
    np.testing.assert_array_equal(m1.tris, m2.tris)
    np.testing.assert_allclose(m1.nodes, m2.nodes, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(m1.seg, m2.seg)
    np.testing.assert_array_equal(m1.tag, m2.tag)
