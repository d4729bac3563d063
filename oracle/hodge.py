"""Discrete Hodge matrices of the transformation-optics medium (Sec. 3.1,
eqs. dis_hodge_eps / dis_hodge_mu; App. B).

  [*eps]_ij   = eps0 * int_Omega rho W1_i . W1_j dz drho
  [*mu^-1]_ij = (1/mu0) * int_Omega rho W2_i . W2_j dz drho

with the Whitney proxies of App. B,
  W1_(a,b) = lam_a grad lam_b - lam_b grad lam_a,
  W2       = 2 (lam_a grad lam_b x grad lam_c + cyclic),
and rho = sum_m rho_m lam_m exactly on each triangle.  The integrands are
cubic in the barycentric coordinates, so the integrals are evaluated exactly
with  int_T lam_0^p lam_1^q lam_2^r dA = 2 Area p! q! r! / (p+q+r+2)!.
"""

from __future__ import annotations

from math import factorial

import numpy as np
import scipy.sparse as sp

from .topology import Topology

EPS0 = 8.8541878128e-12
C_LIGHT = 299792458.0
MU0 = 1.0 / (EPS0 * C_LIGHT * C_LIGHT)


def grad_lambda(nodes, tris):
    """(N2, 3, 2) gradients of the barycentric coordinates, (z, rho) parts,
    and (N2,) areas.  For counter-clockwise (i, j, k):
    grad lam_i = (rho_j - rho_k, z_k - z_j) / (2 Area)."""
    p = nodes[tris]
    z, r = p[..., 0], p[..., 1]
    area = 0.5 * ((z[:, 1] - z[:, 0]) * (r[:, 2] - r[:, 0]) - (z[:, 2] - z[:, 0]) * (r[:, 1] - r[:, 0]))
    g = np.zeros(tris.shape + (2,))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        g[:, i, 0] = (r[:, j] - r[:, k]) / (2 * area)
        g[:, i, 1] = (z[:, k] - z[:, j]) / (2 * area)
    return g, area


def _int_lam3(i, j, k, area):
    """int_T lam_i lam_j lam_k dA (local indices, repeats allowed)."""
    cnt = [0, 0, 0]
    for x in (i, j, k):
        cnt[x] += 1
    num = 1
    for c in cnt:
        num *= factorial(c)
    return 2.0 * area * num / factorial(sum(cnt) + 2)


def local_eps_matrix(nodes_T, edge_local, component=None):
    """Local [*eps]/eps0 of one triangle (3x3) for sides given as oriented
    local node pairs edge_local[k] = (a, b): W1_k = lam_a grad lam_b - lam_b grad lam_a.
    component 'z' or 'rho' keeps only that component of W1_k . W1_l (the two
    parts add up to the whole; used by the stretched-coordinate layer)."""
    tri = np.array([[0, 1, 2]])
    g, area = grad_lambda(np.asarray(nodes_T, float), tri)
    g, area = g[0], float(area[0])
    rho = np.asarray(nodes_T, float)[:, 1]
    if component is None:
        gg = g @ g.T
    else:
        c = {"z": 0, "rho": 1}[component]
        gg = np.outer(g[:, c], g[:, c])
    T = np.zeros((3, 3))
    for k, (a, b) in enumerate(edge_local):
        for l, (c, d) in enumerate(edge_local):
            s = 0.0
            for m in range(3):
                s += rho[m] * (_int_lam3(m, a, c, area) * gg[b, d]
                               - _int_lam3(m, a, d, area) * gg[b, c]
                               - _int_lam3(m, b, c, area) * gg[a, d]
                               + _int_lam3(m, b, d, area) * gg[a, c])
            T[k, l] = s
    return T


def _local_edges(topo, t):
    tri = topo.tris[t]
    loc = []
    for k in range(3):
        tail, head = topo.edges[topo.tri_edges[t, k]]
        loc.append((int(np.where(tri == tail)[0][0]), int(np.where(tri == head)[0][0])))
    return loc


def pml_parts(topo: Topology, faces):
    """eps0 times the z and rho parts of the local [*eps] of the given faces:
    two (len(faces), 3, 3) arrays over each face's sides k = 0, 1, 2."""
    Az = np.zeros((len(faces), 3, 3))
    Ar = np.zeros((len(faces), 3, 3))
    for i, t in enumerate(faces):
        loc = _local_edges(topo, t)
        Az[i] = EPS0 * local_eps_matrix(topo.nodes[topo.tris[t]], loc, "z")
        Ar[i] = EPS0 * local_eps_matrix(topo.nodes[topo.tris[t]], loc, "rho")
    return Az, Ar


def hodge_eps(topo: Topology) -> sp.csr_matrix:
    """[*eps] (N1 x N1, symmetric positive definite), all edges."""
    rows, cols, vals = [], [], []
    for t in range(topo.n2):
        tri = topo.tris[t]
        loc = []
        for k in range(3):
            e = topo.tri_edges[t, k]
            tail, head = topo.edges[e]
            a = int(np.where(tri == tail)[0][0])
            b = int(np.where(tri == head)[0][0])
            loc.append((a, b))
        T = EPS0 * local_eps_matrix(topo.nodes[tri], loc)
        for k in range(3):
            for l in range(3):
                rows.append(topo.tri_edges[t, k])
                cols.append(topo.tri_edges[t, l])
                vals.append(T[k, l])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(topo.n1, topo.n1))
    A.sum_duplicates()
    return A


def whitney2_value(nodes, tris):
    """W2 on each triangle from its App. B definition (a constant)."""
    g, _ = grad_lambda(nodes, tris)

    def cross(u, v):
        return u[..., 0] * v[..., 1] - u[..., 1] * v[..., 0]

    # sum of the three terms at the centroid (lam = 1/3 each); W2 is constant
    w = 2.0 * (cross(g[:, 1], g[:, 2]) + cross(g[:, 2], g[:, 0]) + cross(g[:, 0], g[:, 1])) / 3.0
    return w


def hodge_mu_inv(topo: Topology) -> np.ndarray:
    """Diagonal of [*mu^-1]: (1/mu0) int_T rho (W2)^2 dA, per face."""
    w2 = whitney2_value(topo.nodes, topo.tris)
    rho = topo.nodes[topo.tris][..., 1]
    # int_T rho dA = sum_m rho_m int_T lam_m dA = Area * sum_m rho_m / 3
    int_rho = topo.area * rho.sum(axis=1) / 3.0
    return int_rho * w2 * w2 / MU0
