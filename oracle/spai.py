"""Plain sparse approximate inverse of [*eps] (Sec. 3.1: the explicit, local
update of the field equations uses a SPAI representation of [*eps]^-1).

The paper names the method but not its pattern or thresholds.  Reading used:
  1. Jacobi scaling  A^ = S^-1/2 A S^-1/2,  S = diag(A), free edges only;
  2. a priori pattern P_L = structure of (A^)^L;
  3. for every column k, m_k = argmin || A^(:, J_k) m - e_k ||_2 over the
     entries J_k = {j : (j, k) in P_L} (a dense least-squares problem);
  4. drop |m_jk| < tau * max_j |m_jk| within the column;
  5. symmetrise M^ <- (M^ + M^T)/2 and unscale M = S^-1/2 M^ S^-1/2.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def spai_pattern(A_hat: sp.csr_matrix, level: int) -> sp.csc_matrix:
    """Boolean structure of A_hat^level (level >= 1)."""
    S = (A_hat != 0).astype(np.int64).tocsr()
    P = S.copy()
    for _ in range(level - 1):
        P = (P @ S).astype(bool).astype(np.int64)
    return P.tocsc()


def spai(A: sp.spmatrix, free: np.ndarray, level: int = 3, drop_tol: float = 1e-3,
         symmetric: bool = True):
    """Returns M (N1 x N1 CSR, zero outside the free rows/columns).  With
    symmetric=False the column-wise least-squares solution is returned
    before step 5's averaging (still unscaled back by S^-1/2)."""
    A = sp.csr_matrix(A)
    idx = np.flatnonzero(free)
    Af = A[idx][:, idx].tocsc()
    n = Af.shape[0]
    s = np.sqrt(Af.diagonal())
    Dinv = sp.diags(1.0 / s)
    Ah = (Dinv @ Af @ Dinv).tocsc()
    P = spai_pattern(Ah.tocsr(), level)

    rows, cols, vals = [], [], []
    for k in range(n):
        J = P.indices[P.indptr[k]:P.indptr[k + 1]]
        sub = Ah[:, J]
        I = np.unique(sub.indices)
        Ad = sub[I].toarray()
        rhs = (I == k).astype(float)
        m, *_ = np.linalg.lstsq(Ad, rhs, rcond=None)
        keep = np.abs(m) >= drop_tol * np.abs(m).max()
        rows.extend(J[keep]); cols.extend([k] * int(keep.sum())); vals.extend(m[keep])
    Mh = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    if symmetric:
        Mh = 0.5 * (Mh + Mh.T)
    Mf = (Dinv @ Mh @ Dinv).tocoo()
    M = sp.csr_matrix((Mf.data, (idx[Mf.row], idx[Mf.col])), shape=A.shape)
    M.sort_indices()
    return M


def spai_residuals(A: sp.spmatrix, M: sp.spmatrix, free: np.ndarray):
    """(||I - A M||_F / sqrt(n), max column 2-norm of I - A M) on free edges;
    column k of A M - I is the least-squares residual of column k."""
    idx = np.flatnonzero(free)
    Af = sp.csr_matrix(A)[idx][:, idx]
    Mf = sp.csr_matrix(M)[idx][:, idx]
    R = (sp.identity(len(idx)) - Af @ Mf).tocsc()
    col = np.sqrt(np.asarray(R.multiply(R).sum(axis=0)).ravel())
    return float(np.sqrt((col ** 2).sum() / len(idx))), float(col.max())
