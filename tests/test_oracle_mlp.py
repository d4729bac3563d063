"""Pins of the FP64 reference of the learned-SPAI network and its features.

The network and the pair features are not from the paper; they are pinned
against independent facts: central finite differences of the loss (the
backward pass), the closed form of Adam's first bias-corrected steps, the
symmetry of every feature in (k, j), the hop distance from a breadth-first
search, and the powers of the scaled matrix from dense products.
"""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import configs
from oracle import mlp as om
from oracle.hodge import hodge_eps
from oracle.topology import build_topology


def _rand_net(rng, n_in, H, L):
    return rng.normal(0, 0.5, om.n_params(n_in, H, L))


@pytest.mark.parametrize("L", [1, 2, 3])
def test_backward_matches_finite_differences(L):
    rng = np.random.default_rng(L)
    n_in, H, n = 5, 7, 23
    p = _rand_net(rng, n_in, H, L)
    X = rng.normal(size=(n, n_in))
    y = rng.normal(size=n)
    w = rng.uniform(0.2, 2.0, n)
    loss, g = om.loss_grad(p, X, y, w, n_in, H, L)
    h = 1e-6
    for q in range(len(p)):
        e = np.zeros_like(p)
        e[q] = h
        lp = om.loss_grad(p + e, X, y, w, n_in, H, L)[0]
        lm = om.loss_grad(p - e, X, y, w, n_in, H, L)[0]
        assert g[q] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)


def test_forward_of_a_hand_built_network():
    # one hidden unit: p = v tanh(a . x + b0) + c
    n_in, H, L = 3, 1, 1
    a, b0, v, c = np.array([0.3, -0.2, 0.5]), 0.1, 2.0, -0.7
    p = np.concatenate([a, [b0], [v], [c]])
    X = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0]])
    pred, _ = om.forward(p, X, n_in, H, L)
    assert pred == pytest.approx(v * np.tanh(X @ a + b0) + c, rel=1e-15)


def test_adam_closed_form_steps():
    # constant gradient g: m_t and v_t are geometric sums and the bias
    # correction makes every step exactly lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        p_new, m, v = om.adam(p, g, m, v, t, lr, 0.9, 0.999, eps)
        assert p_new - p == pytest.approx(-lr * g / (np.abs(g) + eps), rel=1e-12)
        p = p_new


@pytest.fixture(scope="module")
def cavity_pairs():
    m = configs.cavity_mesh()
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    k, j, X = om.pair_features(topo, A, 3)
    return topo, A, k, j, X


def test_features_are_symmetric(cavity_pairs):
    topo, A, k, j, X = cavity_pairs
    key = {(a, b): q for q, (a, b) in enumerate(zip(k, j))}
    for q in range(0, len(k), 7):
        r = key[(j[q], k[q])]
        assert np.allclose(X[q], X[r], rtol=1e-12, atol=1e-14)
    assert np.all(X[:, :4].sum(axis=1) == 1.0)


def test_hop_distance_and_matrix_powers_brute_force():
    m = synth.tiny_mesh("eight")
    m.tag[:] = synth.BC_OPEN                 # every edge free
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    k, j, X = om.pair_features(topo, A, 3)
    idx, Ah, s = om.scaled_free_hodge(A, topo.edge_free)
    Ad = Ah.toarray()
    n = Ad.shape[0]
    # breadth-first hop distance in the graph of A^
    dist = np.full((n, n), 99)
    for a in range(n):
        dist[a, a] = 0
        frontier = [a]
        for dd in range(1, 4):
            nxt = []
            for u in frontier:
                for v in np.flatnonzero(Ad[u]):
                    if dist[a, v] == 99:
                        dist[a, v] = dd
                        nxt.append(v)
            frontier = nxt
    pos = {e: q for q, e in enumerate(idx)}
    kk = np.array([pos[e] for e in k])
    jj = np.array([pos[e] for e in j])
    assert len(k) == int((dist <= 3).sum())
    d = X[:, :4].argmax(axis=1)
    assert np.array_equal(d, dist[kk, jj])
    assert np.allclose(np.diag(Ad), 1.0)
    A2, A3 = Ad @ Ad, Ad @ Ad @ Ad
    assert np.allclose(X[:, 4], Ad[kk, jj], atol=1e-14)
    assert np.allclose(X[:, 5], A2[kk, jj], atol=1e-13)
    assert np.allclose(X[:, 6], A3[kk, jj], atol=1e-13)


def test_scaled_targets_of_the_exact_inverse():
    # on a tiny mesh the full pattern holds the whole inverse: the scaled
    # targets of A^-1 are the entries of A^^-1
    m = synth.tiny_mesh("two")
    m.tag[:] = synth.BC_OPEN
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    k, j, X = om.pair_features(topo, A, 3)
    Minv = sp.csr_matrix(np.linalg.inv(A.toarray()))
    y = om.scaled_targets(Minv, A, topo.edge_free, k, j)
    idx, Ah, s = om.scaled_free_hodge(A, topo.edge_free)
    Ahi = np.linalg.inv(Ah.toarray())
    pos = {e: q for q, e in enumerate(idx)}
    assert np.allclose(y, Ahi[[pos[e] for e in k], [pos[e] for e in j]], rtol=1e-10)


def test_cgnr_refine_reaches_the_least_squares_column():
    # CGNR converges to the least-squares column on the pattern, i.e. the
    # unsymmetrised plain SPAI without drop
    from oracle.spai import spai
    m = configs.cavity_mesh()
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    k, j, X = om.pair_features(topo, A, 2)
    idx, Ah, s = om.scaled_free_hodge(A, topo.edge_free)
    pos = np.full(topo.edges.shape[0], -1)
    pos[idx] = np.arange(len(idx))
    kk, jj = pos[k], pos[j]
    start = (kk == jj).astype(float)
    v, res = om.cgnr_refine(Ah, kk, jj, start, 60)
    Mls = spai(A, topo.edge_free, level=2, drop_tol=0.0, symmetric=False)
    y = np.asarray(Mls[j, k]).ravel() / (s[kk] * s[jj])     # column k, row j
    assert np.abs(v - y).max() < 1e-9 * np.abs(y).max()
    # the residual never increases with the number of steps (CGNR minimises
    # the residual norm over a growing Krylov space)
    r = [om.cgnr_refine(Ah, kk, jj, start, q)[1] for q in (0, 1, 2, 4)]
    for a, b in zip(r, r[1:]):
        assert np.all(b <= a * (1 + 1e-12))
