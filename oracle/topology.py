"""Mesh topology and incidence matrices (Sec. 3.1; App. A; App. D).

Edges carry the intrinsic orientation of App. D: from the lower to the higher
global node index.  Faces are counter-clockwise in the (z, rho) plane.

  C     = [D_curl], N2 x N1: +1 where the edge runs along the face's
          counter-clockwise boundary, -1 where it runs against it (App. D);
  Ddiv  = [D~_div], N0 x N1: +1 at the tail of each edge, -1 at its head
          (App. D: the edges that reach node 5 from lower-numbered nodes
          carry -1, those that leave it towards higher ones carry +1);
  the dual curl is C^T (Sec. 3.1).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

PEC, AXIS, EMITTER, OPEN = 1, 2, 3, 4


@dataclass
class Topology:
    nodes: np.ndarray        # (N0, 2) z, rho
    tris: np.ndarray         # (N2, 3)
    edges: np.ndarray        # (N1, 2) tail < head
    tri_edges: np.ndarray    # (N2, 3) edge of local side k = (node k, node k+1)
    tri_signs: np.ndarray    # (N2, 3) C[T, tri_edges[T, k]]
    tri_nbr: np.ndarray      # (N2, 3) face across local side k, -1 on the boundary
    edge_tag: np.ndarray     # (N1,) 0 interior, else boundary tag
    edge_free: np.ndarray    # (N1,) bool: E unknown (not a conductor edge)
    node_free: np.ndarray    # (N0,) bool: node touches no conductor edge
    C: sp.csr_matrix         # (N2, N1)
    Ddiv: sp.csr_matrix      # (N0, N1)
    area: np.ndarray         # (N2,) triangle areas

    @property
    def n0(self):
        return self.nodes.shape[0]

    @property
    def n1(self):
        return self.edges.shape[0]

    @property
    def n2(self):
        return self.tris.shape[0]


def build_topology(nodes, tris, seg, tag) -> Topology:
    nodes = np.asarray(nodes, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    n0, n2 = nodes.shape[0], tris.shape[0]

    p = nodes[tris]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    if np.any(area <= 0):
        raise ValueError("triangles must be counter-clockwise in (z, rho)")

    # all edges, oriented from the lower to the higher node index (App. D)
    key = {}
    edges = []
    for t in tris:
        for k in range(3):
            a, b = int(t[k]), int(t[(k + 1) % 3])
            e = (min(a, b), max(a, b))
            if e not in key:
                key[e] = None
                edges.append(e)
    edges = sorted(edges)
    index = {e: i for i, e in enumerate(edges)}
    edges = np.array(edges, dtype=np.int64)
    n1 = edges.shape[0]

    tri_edges = np.zeros((n2, 3), dtype=np.int64)
    tri_signs = np.zeros((n2, 3), dtype=np.int64)
    rows, cols, vals = [], [], []
    edge_faces = [[] for _ in range(n1)]
    for ti, t in enumerate(tris):
        for k in range(3):
            a, b = int(t[k]), int(t[(k + 1) % 3])   # counter-clockwise side a -> b
            e = index[(min(a, b), max(a, b))]
            s = 1 if a < b else -1                  # agrees with tail -> head?
            tri_edges[ti, k] = e
            tri_signs[ti, k] = s
            rows.append(ti); cols.append(e); vals.append(s)
            edge_faces[e].append((ti, k))
    C = sp.csr_matrix((vals, (rows, cols)), shape=(n2, n1))

    tri_nbr = -np.ones((n2, 3), dtype=np.int64)
    for e, fl in enumerate(edge_faces):
        if len(fl) == 2:
            (t0, k0), (t1, k1) = fl
            tri_nbr[t0, k0] = t1
            tri_nbr[t1, k1] = t0
        elif len(fl) != 1:
            raise ValueError("edge shared by more than two triangles")

    # boundary tags; every boundary edge must be tagged
    seg_tag = {}
    for (a, b), g in zip(np.asarray(seg), np.asarray(tag)):
        seg_tag[(min(int(a), int(b)), max(int(a), int(b)))] = int(g)
    edge_tag = np.zeros(n1, dtype=np.int64)
    for e, fl in enumerate(edge_faces):
        if len(fl) == 1:
            g = seg_tag.get((int(edges[e, 0]), int(edges[e, 1])))
            if g is None:
                raise ValueError(f"boundary edge {tuple(edges[e])} has no tag")
            edge_tag[e] = g
    conductor = (edge_tag == PEC) | (edge_tag == EMITTER)
    edge_free = ~conductor
    node_free = np.ones(n0, dtype=bool)
    node_free[edges[conductor].ravel()] = False

    # dual divergence: +1 at the tail, -1 at the head of every edge
    r = np.concatenate([edges[:, 0], edges[:, 1]])
    c = np.concatenate([np.arange(n1), np.arange(n1)])
    v = np.concatenate([np.ones(n1), -np.ones(n1)])
    Ddiv = sp.csr_matrix((v, (r, c)), shape=(n0, n1))

    return Topology(nodes=nodes, tris=tris, edges=edges, tri_edges=tri_edges,
                    tri_signs=tri_signs, tri_nbr=tri_nbr, edge_tag=edge_tag,
                    edge_free=edge_free, node_free=node_free, C=C, Ddiv=Ddiv, area=area)


def gradient_incidence(topo: Topology) -> sp.csr_matrix:
    """G = [D_grad], N1 x N0: -1 at the tail, +1 at the head (d of a 0-form)."""
    n1 = topo.n1
    r = np.concatenate([np.arange(n1), np.arange(n1)])
    c = np.concatenate([topo.edges[:, 0], topo.edges[:, 1]])
    v = np.concatenate([-np.ones(n1), np.ones(n1)])
    return sp.csr_matrix((v, (r, c)), shape=(n1, topo.n0))
