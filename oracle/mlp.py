"""FP64 reference of the learned-SPAI network: forward, weighted least-squares
loss, backward and Adam; and the pair features it reads.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper computes its SPAI by least squares (Sec. 3.1); the network is an
addition to the method and is checked, not derived, here:
  * network: n_in -> H (tanh) -> ... -> H (tanh) -> 1 (linear), with
    n_layers >= 1 hidden layers.  Parameter vector: for each layer in order,
    W[n_out][n_in] row-major, then b[n_out];
  * loss  L = sum_i w_i (p_i - y_i)^2 / sum_i w_i;
  * Adam (Kingma and Ba, 2015) with bias-corrected moments;
  * features of an edge pair (k, j) of the level-L pattern of the
    Jacobi-scaled Hodge matrix A^ = S^-1/2 A S^-1/2 (free edges).  All are
    symmetric in (k, j):
      0-3  one-hot graph distance d(k, j) = 0, 1, 2, 3 (hops in A's graph)
      4-6  (A^)_kj, (A^^2)_kj, (A^^3)_kj
      7    min(l_k, l_j) / max(l_k, l_j), l = edge length in the meridian plane
      8    |x_k - x_j| / (l_k + l_j), x = edge midpoint
      9    |cos| of the angle between the two edges
      10   min(rho_k, rho_j) / max(rho_k, rho_j), rho at the midpoints (1 if both 0)
      11   (l_k + l_j) / (rho_k + rho_j + l_k + l_j)
      12   (n_k + n_j) / 20, n = entries of row k of A^ (free neighbours incl. itself)
      13   |n_k - n_j| / 10
      14   (r_k + r_j) / 2 - 1, r = sum_i |A^_ki|
      15   d(k, j) / 3
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

N_FEATURES = 16


def layer_shapes(n_in, n_hidden, n_layers):
    shapes = [(n_hidden, n_in)] + [(n_hidden, n_hidden)] * (n_layers - 1) + [(1, n_hidden)]
    return shapes


def n_params(n_in, n_hidden, n_layers):
    return sum(o * i + o for o, i in layer_shapes(n_in, n_hidden, n_layers))


def unpack(params, n_in, n_hidden, n_layers):
    out, o0 = [], 0
    for no, ni in layer_shapes(n_in, n_hidden, n_layers):
        W = params[o0:o0 + no * ni].reshape(no, ni)
        o0 += no * ni
        b = params[o0:o0 + no]
        o0 += no
        out.append((W, b))
    return out


def forward(params, X, n_in, n_hidden, n_layers):
    """Returns (predictions p[n], activations [h_1 .. h_L])."""
    layers = unpack(np.asarray(params, np.float64), n_in, n_hidden, n_layers)
    h = np.asarray(X, np.float64)
    acts = []
    for W, b in layers[:-1]:
        h = np.tanh(h @ W.T + b)
        acts.append(h)
    W, b = layers[-1]
    return (h @ W.T + b)[:, 0], acts


def loss_grad(params, X, y, w, n_in, n_hidden, n_layers):
    """Weighted least-squares loss and its gradient (backpropagation)."""
    X = np.asarray(X, np.float64)
    p, acts = forward(params, X, n_in, n_hidden, n_layers)
    y = np.asarray(y, np.float64)
    w = np.asarray(w, np.float64)
    sw = w.sum()
    r = p - y
    loss = float((w * r * r).sum() / sw)
    layers = unpack(np.asarray(params, np.float64), n_in, n_hidden, n_layers)
    grads = []
    delta = (2.0 * w * r / sw)[:, None]                 # dL/dp, shape (n, 1)
    ins = [X] + acts
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        hin = ins[li]
        grads.append((delta.T @ hin, delta.sum(axis=0)))
        if li > 0:
            delta = (delta @ W) * (1.0 - ins[li] ** 2)      # through tanh of the layer below
    grads.reverse()
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, g


def adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------- features
def _edge_geometry(topo):
    nodes = topo.nodes
    e = topo.edges
    a, b = nodes[e[:, 0]], nodes[e[:, 1]]
    d = b - a
    length = np.sqrt((d ** 2).sum(axis=1))
    mid = 0.5 * (a + b)
    return length, mid, d / length[:, None]


def scaled_free_hodge(A, free):
    idx = np.flatnonzero(free)
    Af = sp.csr_matrix(A)[idx][:, idx]
    s = 1.0 / np.sqrt(Af.diagonal())
    Ah = sp.diags(s) @ Af @ sp.diags(s)
    return idx, sp.csr_matrix(Ah), s


def pair_features(topo, A, level=3):
    """Features of every pair of the level-`level` pattern over free edges.

    Returns (k, j, X): canonical edge indices of each pair and the FP64
    feature rows, ordered by k then j."""
    idx, Ah, s = scaled_free_hodge(A, topo.edge_free)
    n = len(idx)
    S = (Ah != 0).astype(np.int64)
    # graph distance: R_p = structure of S^p (S has its diagonal, so R_p grows
    # with p); d(k, j) = p on R_p minus R_{p-1}
    R = sp.identity(n, format="csr", dtype=np.int64)
    D = sp.csr_matrix((n, n), dtype=np.int64)
    for p in range(1, level + 1):
        Rn = (R @ S).astype(bool).astype(np.int64)
        D = D + p * (Rn - R)
        R = Rn
    reach = R
    patt = reach.tocoo()
    kk, jj = patt.row, patt.col
    order = np.lexsort((jj, kk))
    kk, jj = kk[order], jj[order]
    d = np.asarray(D[kk, jj]).ravel()
    A1 = Ah
    A2 = Ah @ Ah
    A3 = A2 @ Ah
    a1 = np.asarray(A1[kk, jj]).ravel()
    a2 = np.asarray(A2[kk, jj]).ravel()
    a3 = np.asarray(A3[kk, jj]).ravel()
    length, mid, dirv = _edge_geometry(topo)
    lk, lj = length[idx[kk]], length[idx[jj]]
    mk, mj = mid[idx[kk]], mid[idx[jj]]
    rk, rj = mk[:, 1], mj[:, 1]
    nrow = np.diff(Ah.indptr)
    rsum = np.asarray(abs(Ah).sum(axis=1)).ravel()
    X = np.zeros((len(kk), N_FEATURES))
    for q in range(4):
        X[:, q] = (d == q)
    X[:, 4], X[:, 5], X[:, 6] = a1, a2, a3
    X[:, 7] = np.minimum(lk, lj) / np.maximum(lk, lj)
    X[:, 8] = np.sqrt(((mk - mj) ** 2).sum(axis=1)) / (lk + lj)
    X[:, 9] = np.abs((dirv[idx[kk]] * dirv[idx[jj]]).sum(axis=1))
    rmax = np.maximum(rk, rj)
    X[:, 10] = np.where(rmax > 0, np.minimum(rk, rj) / np.where(rmax > 0, rmax, 1.0), 1.0)
    X[:, 11] = (lk + lj) / (rk + rj + lk + lj)
    X[:, 12] = (nrow[kk] + nrow[jj]) / 20.0
    X[:, 13] = np.abs(nrow[kk] - nrow[jj]) / 10.0
    X[:, 14] = 0.5 * (rsum[kk] + rsum[jj]) - 1.0
    X[:, 15] = d / 3.0
    return idx[kk], idx[jj], X


def scaled_targets(M, A, free, k, j):
    """Entries M^_kj = M_kj / (s_k s_j) of the Jacobi-scaled SPAI, s = diag(A)^-1/2."""
    dA = sp.csr_matrix(A).diagonal()
    s = 1.0 / np.sqrt(dA[k] * dA[j])
    return np.asarray(sp.csr_matrix(M)[k, j]).ravel() / s


def cgnr_refine(Ah, kk, jj, values, iters):
    """Conjugate gradients on the normal equations (CGNR) of every column's
    least-squares problem min ||e_k - A^(:, J_k) m||_2 on its pattern J_k,
    started from the given entries: after enough steps each column is the
    plain SPAI's least-squares column (Sec. 3.1 reading, before the drop).

    kk, jj: free indices (column, row) of the pattern entries; returns the
    refined values and the residual norm ||e_k - A^ m_k||_2 of every column."""
    n = Ah.shape[0]
    patt = sp.csc_matrix((np.ones(len(kk)), (jj, kk)), shape=(n, n))
    M = sp.csc_matrix((np.asarray(values, np.float64), (jj, kk)), shape=(n, n))
    eye = sp.identity(n, format="csc")

    def colsum(X):
        return np.asarray(X.sum(axis=0)).ravel()

    R = (eye - Ah @ M).tocsc()
    G = (Ah @ R).multiply(patt).tocsc()
    P = G.copy()
    gg = colsum(G.multiply(G))
    floor = 1e-26 * gg                       # a column has converged below this
    for _ in range(iters):
        AP = (Ah @ P).tocsc()
        den = colsum(AP.multiply(AP))
        live = (den > 0) & (gg > floor)
        a = np.where(live, gg / np.where(live, den, 1.0), 0.0)
        M = (M + P @ sp.diags(a)).tocsc()
        R = (R - AP @ sp.diags(a)).tocsc()
        G = (Ah @ R).multiply(patt).tocsc()
        gn = colsum(G.multiply(G))
        b = np.where(live, gn / np.where(live, gg, 1.0), 0.0)
        P = (G + P @ sp.diags(b)).tocsc()
        gg = gn
    R = (eye - Ah @ M).tocsc()
    res = np.sqrt(colsum(R.multiply(R)))
    return np.asarray(M[jj, kk]).ravel(), res
