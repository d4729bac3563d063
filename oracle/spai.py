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
    P = P.tocsc()
    P.sort_indices()
    return P


def _scaled(A: sp.spmatrix, free: np.ndarray):
    """Step 1: free-edge ids, the scaled block A^ (CSC) and diag(A)^1/2."""
    A = sp.csr_matrix(A)
    idx = np.flatnonzero(free)
    Af = A[idx][:, idx].tocsc()
    s = np.sqrt(Af.diagonal())
    Dinv = sp.diags(1.0 / s)
    return idx, (Dinv @ Af @ Dinv).tocsc(), s


def _column(Ah: sp.csc_matrix, J: np.ndarray, k: int, drop_tol: float):
    """Steps 3-4 for column k over the pattern entries J (ascending): the
    kept rows and values of m_k."""
    sub = Ah[:, J]
    I = np.unique(sub.indices)
    Ad = sub[I].toarray()
    rhs = (I == k).astype(float)
    m, *_ = np.linalg.lstsq(Ad, rhs, rcond=None)
    keep = np.abs(m) >= drop_tol * np.abs(m).max()
    return J[keep], m[keep]


def spai(A: sp.spmatrix, free: np.ndarray, level: int = 3, drop_tol: float = 1e-3,
         symmetric: bool = True):
    """Returns M (N1 x N1 CSR, zero outside the free rows/columns).  With
    symmetric=False the column-wise least-squares solution is returned
    before step 5's averaging (still unscaled back by S^-1/2)."""
    idx, Ah, s = _scaled(A, free)
    n = Ah.shape[0]
    P = spai_pattern(Ah.tocsr(), level)

    rows, cols, vals = [], [], []
    for k in range(n):
        Jk, mk = _column(Ah, P.indices[P.indptr[k]:P.indptr[k + 1]], k, drop_tol)
        rows.extend(Jk); cols.extend([k] * len(Jk)); vals.extend(mk)
    Mh = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    if symmetric:
        Mh = 0.5 * (Mh + Mh.T)
    Dinv = sp.diags(1.0 / s)
    Mf = (Dinv @ Mh @ Dinv).tocoo()
    M = sp.csr_matrix((Mf.data, (idx[Mf.row], idx[Mf.col])), shape=A.shape)
    M.sort_indices()
    return M


def spai_rows(A: sp.spmatrix, free: np.ndarray, rows, level: int = 3, drop_tol: float = 1e-3):
    """Rows `rows` (ids of free edges) of spai(A, free, level, drop_tol), as a
    len(rows) x N1 CSR matrix, from only the column problems they need.

    Row e of the symmetrised M^ is the average of column e and of entry e of
    every column k whose pattern holds e.  The pattern, the structure of a
    power of the symmetric A^, is symmetric, so those are the columns in
    the pattern of column e.  Each column is solved exactly as spai() solves
    it; the pattern of a set of columns is the structure of A^^level applied
    to them."""
    idx, Ah, s = _scaled(A, free)
    n = Ah.shape[0]
    pos = -np.ones(sp.csr_matrix(A).shape[0], dtype=np.int64)
    pos[idx] = np.arange(n)
    r = pos[np.asarray(rows, dtype=np.int64)]
    if np.any(r < 0):
        raise ValueError("spai_rows: every row must be a free edge")
    S = (Ah != 0).astype(np.int64).tocsc()

    def pattern_of(cols):
        X = S[:, cols]
        for _ in range(level - 1):
            X = (S @ X).astype(bool).astype(np.int64)
        X = X.tocsc()
        X.sort_indices()
        return X

    Pr = pattern_of(r)
    need = np.unique(np.concatenate([Pr.indices, r]))
    Pn = pattern_of(need)
    solved = {}
    for i, k in enumerate(need):
        solved[int(k)] = _column(Ah, Pn.indices[Pn.indptr[i]:Pn.indptr[i + 1]], int(k), drop_tol)
    out_r, out_c, out_v = [], [], []
    for i, e in enumerate(r):
        e = int(e)
        vals = {}
        Je, me = solved[e]                         # column e: entries M^(j, e)
        for j, v in zip(Je, me):
            vals[int(j)] = vals.get(int(j), 0.0) + 0.5 * v
        for k in Pr.indices[Pr.indptr[i]:Pr.indptr[i + 1]]:
            Jk, mk = solved[int(k)]                # entry M^(e, k) of column k
            hit = np.flatnonzero(Jk == e)
            if len(hit):
                vals[int(k)] = vals.get(int(k), 0.0) + 0.5 * mk[hit[0]]
        for j, v in vals.items():
            out_r.append(i); out_c.append(idx[j]); out_v.append(v / (s[e] * s[j]))
    return sp.csr_matrix((out_v, (out_r, out_c)), shape=(len(r), sp.csr_matrix(A).shape[0]))


def spai_residuals(A: sp.spmatrix, M: sp.spmatrix, free: np.ndarray):
    """(||I - A M||_F / sqrt(n), max column 2-norm of I - A M) on free edges;
    column k of A M - I is the least-squares residual of column k."""
    idx = np.flatnonzero(free)
    Af = sp.csr_matrix(A)[idx][:, idx]
    Mf = sp.csr_matrix(M)[idx][:, idx]
    R = (sp.identity(len(idx)) - Af @ Mf).tocsc()
    col = np.sqrt(np.asarray(R.multiply(R).sum(axis=0)).ravel())
    return float(np.sqrt((col ** 2).sum() / len(idx))), float(col.max())
