"""FP64 reference of the electrostatic, Gauss-consistent initial state.

TEST INFRASTRUCTURE ONLY: the GPU library never imports this module.

The scheme carries the Gauss law as the invariant
res = D~div [*eps]_a E - Q on the free nodes (Sec. 3.5.2), with
[*eps]_a = M^-1 the inverse of the sparse approximate inverse; it stays at
its initial value for all steps, and it is zero only if the initial state
makes it zero (the consistency the paper asks of the initial conditions).
An applied voltage (the cathode-anode field of the diode, Sec. 4.2) enters as the
potential phi on the conductor nodes.  The initial state is then

    E = -G phi  (curl-free: C G = 0, so the face fluxes B do not move),
    D~div W (-G phi) = Q  on the free nodes,  phi given on conductor nodes,

with W the edge Hodge operator: W = M^-1 for the scheme's state, or W = A
(the exact [*eps]) for the continuous problem's Galerkin solution.  Since
-G = D~div^T, the operator K = D~div W D~div^T on the free nodes is
symmetric positive definite.  This reference forms K column by column (a
sparse LU of M on the free edges for W = M^-1) and solves it densely:
small meshes only.  E on conductor edges is 0 (the field boundary
condition), and D = W E.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .topology import gradient_incidence


def _hodge_operator(A_or_M, edge_free, inverse):
    fe = np.flatnonzero(edge_free)
    Xff = sp.csc_matrix(A_or_M[fe][:, fe])
    if inverse:
        lu = spla.splu(Xff)
        return fe, lu.solve
    return fe, lambda x: Xff @ x


def electrostatic(topo, W_matrix, phi_conductor, Q, inverse=True):
    """Potential phi (N0), field E (N1), D = W E (N1) and the Gauss residual
    on the free nodes.  W_matrix: M (inverse=True, W = M^-1) or A
    (inverse=False, W = A).  phi_conductor: potential used on the conductor
    nodes (N0; other entries ignored).  Q: nodal charge per radian (N0)."""
    G = gradient_incidence(topo)
    Dd = topo.Ddiv
    fn = np.flatnonzero(topo.node_free)
    cn = np.flatnonzero(~topo.node_free)
    fe, apply_w = _hodge_operator(W_matrix, topo.edge_free, inverse)

    def field_of(phi):
        E = -(G @ phi)
        E[~topo.edge_free] = 0.0
        D = np.zeros(topo.n1)
        D[fe] = apply_w(E[fe])
        return E, D

    # K restricted to the free nodes, column by column
    Gf = -G[:, fn].toarray()[fe]                 # E on free edges of a unit potential at each free node
    WG = apply_w(Gf)
    K = Dd[fn][:, fe] @ WG
    K = 0.5 * (K + K.T)
    phi = np.zeros(topo.n0)
    phi[cn] = np.asarray(phi_conductor, dtype=np.float64)[cn]
    _, Dc = field_of(phi)
    rhs = np.asarray(Q, dtype=np.float64)[fn] - Dd[fn] @ Dc
    phi[fn] = np.linalg.solve(K, rhs)
    E, D = field_of(phi)
    res = Dd @ D - np.asarray(Q, dtype=np.float64)
    return phi, E, D, res[fn]
