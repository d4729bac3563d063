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
