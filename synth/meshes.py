"""Seeded triangular meshes of the meridian (z, rho) half-plane.

Every mesh is built the same way: a jittered hexagonal point lattice in a
reference rectangle (z, s) with s in [0, 1], a Delaunay triangulation of that
convex point set (scipy/qhull), and the map rho = s * R(z) onto the physical
domain 0 <= rho <= R(z).  For a constant R this is a plain seeded Delaunay
mesh of a rectangle; for a rippled wall R(z) it is the image of one under a
smooth orientation-preserving map, so every wall node lies exactly on R(z).

Boundary segments are the triangulation edges with a single adjacent
triangle; each gets a tag from the caller's rule (PEC wall, symmetry axis,
emitting cathode, open/free boundary).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.spatial

# Boundary tags.  The numeric values are part of the library interface
# (they match the AXP_BC_* constants of the C ABI).
BC_PEC = 1      # perfect electric conductor: tangential E = 0, particles absorbed
BC_AXIS = 2     # symmetry axis rho = 0: natural (free) edges, particles stay in rho >= 0
BC_EMITTER = 3  # conductor that also injects particles (a PEC for the field)
BC_OPEN = 4     # free (natural) field boundary; particles leaving are absorbed
BC_NAMES = {BC_PEC: "pec", BC_AXIS: "axis", BC_EMITTER: "emitter", BC_OPEN: "open"}


@dataclass
class Mesh:
    """A triangulated meridian domain.

    nodes : (N0, 2) float64, columns (z, rho) in metres
    tris  : (N2, 3) int32, node ids, counter-clockwise in the (z, rho) plane
    seg   : (Nb, 2) int32, boundary segments (node ids, unordered)
    tag   : (Nb,) uint8, BC_* tag of each boundary segment
    """

    nodes: np.ndarray
    tris: np.ndarray
    seg: np.ndarray
    tag: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    def signed_areas(self) -> np.ndarray:
        p = self.nodes[self.tris]
        return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                      - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))


def canonical_edges(tris: np.ndarray) -> np.ndarray:
    """All edges of a triangulation as (tail, head) with tail < head, sorted
    lexicographically.  This is the indexing convention of edge-based
    degrees of freedom used at the library interface: edge i runs from
    node tail_i to node head_i (ascending node index)."""
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return e.astype(np.int32)


def _hex_lattice(z0, z1, h, ny, jitter, rng):
    """Jittered hexagonal lattice in the reference rectangle [z0,z1] x [0,1].

    Rows sit at s_j = j/ny; odd rows are shifted by half a spacing and also
    carry the two end points so that every row spans the full width.  Points
    on the four sides stay on their side (they only move along it)."""
    nx = max(2, int(round((z1 - z0) / h)))
    dx = (z1 - z0) / nx
    pts = []
    for j in range(ny + 1):
        s = j / ny
        if j % 2 == 0:
            z = z0 + dx * np.arange(nx + 1)
            z[-1] = z1                      # exact end point: it must stay on the side z = z1
        else:
            z = np.concatenate([[z0], z0 + dx * (np.arange(nx) + 0.5), [z1]])
        row = np.stack([z, np.full_like(z, s)], axis=1)
        interior_z = (row[:, 0] > z0) & (row[:, 0] < z1)
        if 0 < j < ny:
            row[interior_z, 0] += rng.uniform(-jitter, jitter, interior_z.sum()) * dx
            row[:, 1] += rng.uniform(-jitter, jitter, row.shape[0]) / ny
        else:
            row[interior_z, 0] += rng.uniform(-jitter, jitter, interior_z.sum()) * dx
        pts.append(row)
    p = np.concatenate(pts, axis=0)
    # z-major numbering: walk the long axis, then the short one
    order = np.lexsort((p[:, 1], np.floor((p[:, 0] - z0) / dx + 0.25)))
    return p[order]


def _triangulate(p_ref: np.ndarray) -> np.ndarray:
    d = scipy.spatial.Delaunay(p_ref)
    tris = d.simplices.astype(np.int64)
    a = p_ref[tris]
    area = 0.5 * ((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
                  - (a[:, 2, 0] - a[:, 0, 0]) * (a[:, 1, 1] - a[:, 0, 1]))
    flip = area < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    if len(np.unique(tris)) != p_ref.shape[0]:
        raise RuntimeError("triangulation dropped input points")
    # sort triangles by centroid along the long axis for a local numbering
    c = p_ref[tris].mean(axis=1)
    tris = tris[np.lexsort((c[:, 1], c[:, 0]))]
    return tris.astype(np.int32)


def _boundary_segments(tris: np.ndarray) -> np.ndarray:
    t = np.asarray(tris, dtype=np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    return uniq[cnt == 1].astype(np.int32)


def _classify(p_ref, seg, z0, z1):
    """Side of each boundary segment in reference space."""
    a, b = p_ref[seg[:, 0]], p_ref[seg[:, 1]]
    tol = 1e-12
    side = np.full(len(seg), "", dtype=object)
    side[(np.abs(a[:, 1]) < tol) & (np.abs(b[:, 1]) < tol)] = "bottom"
    side[(np.abs(a[:, 1] - 1) < tol) & (np.abs(b[:, 1] - 1) < tol)] = "top"
    side[(np.abs(a[:, 0] - z0) < tol) & (np.abs(b[:, 0] - z0) < tol)] = "left"
    side[(np.abs(a[:, 0] - z1) < tol) & (np.abs(b[:, 0] - z1) < tol)] = "right"
    if np.any(side == ""):
        raise RuntimeError("boundary segment not on a side of the reference rectangle")
    return side


def _build(z0, z1, radius_fn, h, seed, jitter, tag_rule, meta):
    rng = np.random.default_rng(seed)
    r_mean = float(np.mean(radius_fn(np.linspace(z0, z1, 257))))
    ny = max(2, int(round(r_mean / (h * np.sqrt(3.0) / 2.0))))
    p_ref = _hex_lattice(z0, z1, h, ny, jitter, rng)
    # triangulate where the lattice is isotropic: (z, s * mean radius)
    tris = _triangulate(p_ref * np.array([1.0, r_mean]))
    nodes = np.stack([p_ref[:, 0], p_ref[:, 1] * radius_fn(p_ref[:, 0])], axis=1)
    seg = _boundary_segments(tris)
    side = _classify(p_ref, seg, z0, z1)
    mid = 0.5 * (nodes[seg[:, 0]] + nodes[seg[:, 1]])
    tag = np.array([tag_rule(s, m[0], m[1]) for s, m in zip(side, mid)], dtype=np.uint8)
    mesh = Mesh(nodes=nodes.astype(np.float64), tris=tris, seg=seg, tag=tag, meta=dict(meta))
    if np.any(mesh.signed_areas() <= 0):
        raise RuntimeError("mapped mesh has a non-positive triangle")
    mesh.meta.update(h=h, seed=seed, ny=ny)
    return mesh


def rect_mesh(z0, z1, rho1, h, seed, jitter=0.3, tags=None):
    """Seeded Delaunay mesh of [z0, z1] x [0, rho1].

    tags: dict side -> tag, or a callable (side, z_mid, rho_mid) -> tag,
    sides being 'bottom' (rho = 0), 'top' (rho = rho1), 'left' (z = z0) and
    'right' (z = z1).  Default: axis at the bottom, PEC elsewhere (a closed
    cylindrical cavity)."""
    if tags is None:
        tags = {"bottom": BC_AXIS, "top": BC_PEC, "left": BC_PEC, "right": BC_PEC}
    rule = tags if callable(tags) else (lambda s, z, r: tags[s])
    return _build(z0, z1, lambda z: np.full_like(np.asarray(z, float), rho1), h, seed, jitter,
                  rule, dict(kind="rect", z0=z0, z1=z1, rho1=rho1))


def rippled_mesh(radius_fn, z0, z1, h, seed, jitter=0.3, tags=None, meta=None):
    """Seeded mesh of 0 <= rho <= R(z), z0 <= z <= z1 (rippled-wall tube).

    Default tags: axis at rho = 0, PEC on the wall and both end plates."""
    if tags is None:
        tags = {"bottom": BC_AXIS, "top": BC_PEC, "left": BC_PEC, "right": BC_PEC}
    rule = tags if callable(tags) else (lambda s, z, r: tags[s])
    m = dict(kind="rippled", z0=z0, z1=z1)
    m.update(meta or {})
    return _build(z0, z1, radius_fn, h, seed, jitter, rule, m)


def grid_mesh(radius_fn, z0, z1, h, staircase=False, tags=None, meta=None):
    """Structured mesh of 0 <= rho <= R(z) on columns of width dz = (z1 - z0) / nz,
    nz = round((z1 - z0) / h); every quadrilateral cell is split into two
    triangles, the diagonal alternating like a checkerboard.

    staircase=False: the mapped grid.  Column line i carries n rows at
      rho = k R(z_i) / n (n = round(mean R / h)), so every wall node lies on
      R(z) and the wall is the polyline through them.
    staircase=True: the step-cell wall of a structured grid.  Nodes sit at
      (z_i, k h); column j keeps the rows k < n_j = round(R(z_j + dz/2) / h),
      so the wall is made of grid lines, with vertical risers where two
      neighbouring columns differ.

    The two share the triangle topology, so comparing them isolates the error
    of the staircased wall from the grid's own dispersion.  For a constant R
    that is a whole number of rows h the two meshes coincide.

    Default tags: axis at rho = 0, PEC on the wall (risers included) and on
    both end plates; a tags dict or rule sees the sides 'bottom', 'top'
    (the wall), 'left' and 'right'."""
    if tags is None:
        tags = {"bottom": BC_AXIS, "top": BC_PEC, "left": BC_PEC, "right": BC_PEC}
    rule = tags if callable(tags) else (lambda s, z, r: tags[s])
    nz = max(1, int(round((z1 - z0) / h)))
    dz = (z1 - z0) / nz
    zi = z0 + dz * np.arange(nz + 1)
    zi[-1] = z1
    R = lambda z: np.asarray(radius_fn(np.asarray(z, dtype=np.float64)), dtype=np.float64)
    if staircase:
        rows = np.maximum(1, np.rint(R(zi[:-1] + 0.5 * dz) / h).astype(np.int64))      # rows of column j
        top = np.maximum(np.concatenate([[0], rows]), np.concatenate([rows, [0]]))       # rows at line i
        height = lambda i, k: k * h
    else:
        n = max(1, int(round(float(np.mean(R(np.linspace(z0, z1, 257)))) / h)))
        rows = np.full(nz, n, dtype=np.int64)
        top = np.full(nz + 1, n, dtype=np.int64)
        Ri = R(zi)
        height = lambda i, k: k * Ri[i] / n
    off = np.concatenate([[0], np.cumsum(top + 1)])
    nodes = np.array([[zi[i], height(i, k)] for i in range(nz + 1) for k in range(top[i] + 1)],
                     dtype=np.float64)
    tris = []
    for j in range(nz):
        for k in range(rows[j]):
            a, b = off[j] + k, off[j + 1] + k
            c, d = b + 1, a + 1
            tris += [(a, b, c), (a, c, d)] if (j + k) % 2 == 0 else [(a, b, d), (b, c, d)]
    tris = np.array(tris, dtype=np.int32)
    seg = _boundary_segments(tris)
    pa, pb = nodes[seg[:, 0]], nodes[seg[:, 1]]
    side = np.full(len(seg), "top", dtype=object)
    side[(pa[:, 1] == 0.0) & (pb[:, 1] == 0.0)] = "bottom"
    side[(pa[:, 0] == z0) & (pb[:, 0] == z0)] = "left"
    side[(pa[:, 0] == z1) & (pb[:, 0] == z1)] = "right"
    mid = 0.5 * (pa + pb)
    tag = np.array([rule(s, q[0], q[1]) for s, q in zip(side, mid)], dtype=np.uint8)
    m = dict(kind="staircase" if staircase else "grid", z0=z0, z1=z1, h=h, nz=nz)
    m.update(meta or {})
    mesh = Mesh(nodes=nodes, tris=tris, seg=seg, tag=tag, meta=m)
    if np.any(mesh.signed_areas() <= 0):
        raise RuntimeError("grid mesh has a non-positive triangle")
    return mesh


def tiny_mesh(kind: str) -> Mesh:
    """Hand-built meshes for brute-force checks.

    'two'   : unit square [0,1]x[1,2] split by its diagonal (2 triangles)
    'eight' : [0,2]x[0,1] square pair, each split into 4 by its centre
              (8 triangles, one interior node per square; rho = 0 on the axis)
    """
    if kind == "two":
        nodes = np.array([[0.0, 1.0], [1.0, 1.0], [1.0, 2.0], [0.0, 2.0]])
        tris = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    elif kind == "eight":
        nodes = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0],
                          [0.0, 1.0], [1.0, 1.0], [2.0, 1.0],
                          [0.5, 0.5], [1.5, 0.5]])
        tris = np.array([[0, 1, 6], [1, 4, 6], [4, 3, 6], [3, 0, 6],
                         [1, 2, 7], [2, 5, 7], [5, 4, 7], [4, 1, 7]], dtype=np.int32)
    else:
        raise ValueError(kind)
    seg = _boundary_segments(tris)
    mid = 0.5 * (nodes[seg[:, 0]] + nodes[seg[:, 1]])
    tag = np.where(np.abs(mid[:, 1]) < 1e-12, BC_AXIS, BC_PEC).astype(np.uint8)
    m = Mesh(nodes=nodes, tris=tris, seg=seg, tag=tag, meta=dict(kind=kind))
    assert np.all(m.signed_areas() > 0)
    return m
