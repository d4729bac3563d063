"""Pins of the oracle's setup: topology, Hodge matrices, SPAI, stability.

Each check compares against something other than the oracle itself: values
printed in the paper (tests/golden), closed forms, exact integer identities,
an independent quadrature, or a textbook dense routine.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import synth
from oracle import build_topology, hodge_eps, hodge_mu_inv, whitney2_value, spai, spai_residuals, cfl_dt
from oracle.topology import gradient_incidence
from oracle.hodge import local_eps_matrix, grad_lambda, EPS0

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    m = synth.rect_mesh(0.0, 0.02, 0.01, 0.49e-3, seed=0)
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    return m, topo, hodge_eps(topo), hodge_mu_inv(topo)


@pytest.fixture(scope="module")
def ripple():
    R = lambda z: 0.015 + 0.0025 * np.sin(2 * np.pi * z / 0.0167)
    m = synth.rippled_mesh(R, 0.0, 0.03, 0.6e-3, seed=3)
    return m, build_topology(m.nodes, m.tris, m.seg, m.tag)


# ------------------------------------------------------------------ topology
def test_euler_and_boundary_counts(c1, ripple):
    for m, topo in ((c1[0], c1[1]), ripple):
        assert topo.n0 - topo.n1 + topo.n2 == 1                      # simply connected disc
        nb = int(np.sum(np.bincount(topo.C.indices, minlength=topo.n1) == 1))
        assert nb == 2 * topo.n1 - 3 * topo.n2                       # 3 N2 = 2 Nint + Nb
        assert np.array_equal(topo.edges, synth.canonical_edges(m.tris))


def test_exact_sequence_identities(c1, ripple):
    for topo in (c1[1], ripple[1]):
        G = gradient_incidence(topo)
        assert abs(topo.C @ G).max() == 0                            # curl grad = 0
        assert abs(topo.Ddiv @ topo.C.T).max() == 0                  # div curl = 0 (Sec. 3.5.2)
        assert np.all(np.abs(topo.C.data) == 1) and np.all(np.diff(topo.C.indptr) == 3)


def test_appendix_d_sign_rule_by_hand():
    """App. D: an incidence entry is -1 where the intrinsic (ascending index)
    edge orientation opposes the face circulation / divergence direction.
    Hand-derived on the 8-triangle mesh (faces CCW)."""
    m = synth.tiny_mesh("eight")
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    idx = {tuple(e): i for i, e in enumerate(topo.edges)}
    C = topo.C.toarray()
    # face 0 = (0, 1, 6): 0->1 agrees, 1->6 agrees, 6->0 opposes edge (0, 6)
    assert C[0, idx[(0, 1)]] == 1 and C[0, idx[(1, 6)]] == 1 and C[0, idx[(0, 6)]] == -1
    # face 2 = (4, 3, 6): 4->3 opposes (3, 4), 3->6 agrees, 6->4 opposes (4, 6)
    assert C[2, idx[(3, 4)]] == -1 and C[2, idx[(3, 6)]] == 1 and C[2, idx[(4, 6)]] == -1
    assert np.count_nonzero(C[0]) == 3
    D = topo.Ddiv.toarray()
    # node 4: reached from 1 and 3 (lower ids) -> -1; leaves to 5, 6, 7 -> +1
    assert D[4, idx[(1, 4)]] == -1 and D[4, idx[(3, 4)]] == -1
    assert D[4, idx[(4, 5)]] == 1 and D[4, idx[(4, 6)]] == 1 and D[4, idx[(4, 7)]] == 1
    assert np.count_nonzero(D[4]) == 5
    # node 6 is the highest id around it: every incident edge gives -1
    assert set(D[6][D[6] != 0]) == {-1.0}


def test_free_edges_and_nodes(c1):
    topo = c1[1]
    pec = (topo.edge_tag == synth.BC_PEC)
    assert not np.any(topo.edge_free[pec])
    assert np.all(topo.edge_free[topo.edge_tag == synth.BC_AXIS])
    on_axis_only = np.setdiff1d(topo.edges[topo.edge_tag == synth.BC_AXIS].ravel(),
                                topo.edges[pec].ravel())
    assert np.all(topo.node_free[on_axis_only])


# --------------------------------------------------------------------- Hodge
def _read_appb():
    rows = {}
    for line in open(os.path.join(GOLDEN, "appB_local_hodge.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, *c = line.split()
        rows[name] = np.array([float(Fraction(x)) for x in c]).reshape(3, 3)
    return rows


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_appendix_b_printed_entries(seed):
    """The exact local [*eps] equals App. B's printed T11, T12, T13, T23, T33
    (local edges e1=(1->2), e2=(1->3), e3=(2->3)); T22 is printed garbled."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 1.0, (3, 2))
    g, area = grad_lambda(v, np.array([[0, 1, 2]]))
    if area[0] < 0:
        v = v[[0, 2, 1]]
        g, area = grad_lambda(v, np.array([[0, 1, 2]]))
    g, area = g[0], area[0]
    t = np.array([g[0] @ g[0], g[0] @ g[1], g[1] @ g[1]]) / 5.0
    rho = v[:, 1]
    T = local_eps_matrix(v, [(0, 1), (0, 2), (1, 2)]) / area
    gold = _read_appb()
    pos = {"T11": (0, 0), "T12": (0, 1), "T13": (0, 2), "T23": (1, 2), "T33": (2, 2)}
    for name, (i, j) in pos.items():
        printed = sum(t[k] * (gold[name][k] @ rho) for k in range(3))
        assert T[i, j] == pytest.approx(printed, rel=1e-12)
        assert T[j, i] == pytest.approx(printed, rel=1e-12)
    garbled = sum(t[k] * (gold["T22_printed"][k] @ rho) for k in range(3))
    corrected = t[0] * (rho[0] + rho[1] / 2 + rho[2]) + t[1] * (4 * rho[0] / 3 + rho[1] / 2 + 2 * rho[2] / 3) \
        + t[2] * (rho[0] / 2 + rho[1] / 6 + rho[2] / 6)
    assert T[1, 1] == pytest.approx(corrected, rel=1e-12)
    assert abs(T[1, 1] - garbled) > 1e-3 * abs(T[1, 1])


def _duffy_rule(n):
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1), 0.5 * w
    pts, wts = [], []
    for xu, wu in zip(x, w):
        for xv, wv in zip(x, w):
            l1, l2 = xu, (1 - xu) * xv
            pts.append((1 - l1 - l2, l1, l2))
            wts.append(wu * wv * (1 - xu) * 2.0)   # times area later
    return np.array(pts), np.array(wts)


def test_local_eps_against_independent_quadrature():
    """int_T rho W1_k . W1_l by a product Gauss rule (exact for cubics)."""
    rng = np.random.default_rng(11)
    v = np.array([[0.0, 0.2], [1.0, 0.5], [0.3, 1.1]]) + rng.uniform(0, 0.1, (3, 2))
    loc = [(0, 1), (1, 2), (2, 0)]
    T = local_eps_matrix(v, loc)
    A = 0.5 * ((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
    # independent gradients: solve the affine map lam(r)
    Mx = np.array([[1, v[i, 0], v[i, 1]] for i in range(3)])
    coef = np.linalg.inv(Mx)          # lam_i = coef[0,i] + coef[1,i] z + coef[2,i] rho
    grads = coef[1:, :].T             # (3, 2)
    lam, w = _duffy_rule(5)
    Q = np.zeros((3, 3))
    for L, wt in zip(lam, w):
        rho = L @ v[:, 1]
        W = [L[a] * grads[b] - L[b] * grads[a] for a, b in loc]
        for k in range(3):
            for l in range(3):
                Q[k, l] += wt * A * rho * W[k] @ W[l]
    np.testing.assert_allclose(T, Q, rtol=1e-12, atol=1e-14 * abs(Q).max())


def test_constant_field_energy_identity(c1):
    """Edge values of a uniform E0 make E^T [*eps] E = eps0 |E0|^2 int rho dA exactly."""
    m, topo, A, H = c1
    e0 = np.array([3.0e5, -1.7e5])
    E = synth.uniform_field_dofs(topo.nodes, topo.edges, e0[0], e0[1])
    int_rho = np.sum(topo.area * topo.nodes[topo.tris][..., 1].mean(axis=1))
    assert E @ (A @ E) == pytest.approx(EPS0 * (e0 @ e0) * int_rho, rel=1e-12)


def test_eps_hodge_spd_five_per_row(c1):
    m, topo, A, H = c1
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-14 * abs(Ad).max())
    np.linalg.cholesky(Ad)
    interior = topo.edge_tag == 0
    assert np.all(np.diff(A.indptr)[interior] == 5)   # App. B: 5 non-zeros per interior row


def test_mu_hodge_closed_form(c1):
    """W2 = 1/Area from its App. B definition; [*mu^-1] = mean(rho)/(mu0 Area)."""
    m, topo, A, H = c1
    np.testing.assert_allclose(whitney2_value(topo.nodes, topo.tris), 1.0 / topo.area, rtol=1e-12)
    mu0 = 1.0 / (EPS0 * 299792458.0 ** 2)
    np.testing.assert_allclose(H, topo.nodes[topo.tris][..., 1].mean(axis=1) / (mu0 * topo.area), rtol=1e-12)


# ---------------------------------------------------------------------- SPAI
def test_spai_full_pattern_is_exact_inverse():
    m = synth.tiny_mesh("eight")
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    M = spai(A, topo.edge_free, level=12, drop_tol=0.0)
    idx = np.flatnonzero(topo.edge_free)
    Ai = np.linalg.inv(A.toarray()[np.ix_(idx, idx)])
    np.testing.assert_allclose(M.toarray()[np.ix_(idx, idx)], Ai, rtol=1e-9, atol=1e-9 * abs(Ai).max())


def test_spai_columns_solve_least_squares(c1):
    """Before the symmetric average, column k of the scaled M is the
    minimiser of ||A^(:,J_k) m - e_k||_2 (compared with scipy.linalg.lstsq,
    and the residual satisfies the normal equations)."""
    import scipy.sparse as sp
    from oracle.spai import spai_pattern
    m, topo, A, H = c1
    idx = np.flatnonzero(topo.edge_free)
    Af = A[idx][:, idx]
    s = 1.0 / np.sqrt(Af.diagonal())
    Ah = (sp.diags(s) @ Af @ sp.diags(s)).tocsc()
    P = spai_pattern(Ah.tocsr(), 2)
    M = spai(A, topo.edge_free, level=2, drop_tol=0.0, symmetric=False)
    Mh = (sp.diags(1 / s) @ M[idx][:, idx] @ sp.diags(1 / s)).tocsc()
    rng = np.random.default_rng(0)
    for k in rng.choice(len(idx), 25, replace=False):
        J = P.indices[P.indptr[k]:P.indptr[k + 1]]
        Ad = Ah[:, J].toarray()
        e = np.zeros(len(idx)); e[k] = 1.0
        mk = scipy.linalg.lstsq(Ad, e)[0]
        assert abs(Ad.T @ (Ad @ mk - e)).max() < 1e-10
        col = Mh[:, k].toarray().ravel()
        np.testing.assert_allclose(col[J], mk, rtol=1e-9, atol=1e-12 * abs(mk).max())
        assert np.all(np.delete(col, J) == 0)


def test_spai_level3_quality_and_spd(c1):
    m, topo, A, H = c1
    res = []
    for level in (1, 2, 3):
        M = spai(A, topo.edge_free, level=level, drop_tol=1e-3)
        res.append(spai_residuals(A, M, topo.edge_free)[0])
    assert res[0] > res[1] > res[2]
    idx = np.flatnonzero(topo.edge_free)
    Md = M.toarray()[np.ix_(idx, idx)]
    assert np.allclose(Md, Md.T, atol=1e-14 * abs(Md).max())
    assert np.linalg.eigvalsh(Md).min() > 0
    nnz_row = M.nnz / len(idx)
    assert 15 < nnz_row < 25


def test_cfl_matches_dense_eigenvalue(c1):
    m, topo, A, H = c1
    M = spai(A, topo.edge_free, level=1, drop_tol=1e-3)
    dt, lam = cfl_dt(topo, H, M, iters=2000)
    from oracle.cfl import curl_curl
    idx = np.flatnonzero(topo.edge_free)
    K = curl_curl(topo, H).toarray()[np.ix_(idx, idx)]
    Md = M.toarray()[np.ix_(idx, idx)]
    # generalized symmetric problem K v = lam M^-1 v
    ev = scipy.linalg.eigh(K, np.linalg.inv(Md), eigvals_only=True)
    assert lam == pytest.approx(ev.max(), rel=1e-6)


# ------------------------------------------------------------- paper Table 1
def test_table1_analytic_frequencies():
    """Table 1's analytic f_a are c/(2 pi) sqrt((x_0n/a)^2 + (p pi/h)^2) for
    a = 0.5 m, h = 1 m.  Three rows carry mislabelled (n, p): printed
    (0,3,1) at 0.879 is (0,3,2), printed (0,3,1) at 0.917 is (0,2,5),
    printed (0,2,5) at 0.929 is (0,1,6)."""
    c = 299792458.0
    x = scipy.special.jn_zeros(0, 3)
    relabel = {0.879: (3, 2), 0.917: (2, 5), 0.929: (1, 6)}
    for line in open(os.path.join(GOLDEN, "table1_cavity_modes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        m_, n, p, fa, err = line.split()
        fa = float(fa)
        n, p = relabel.get(fa, (int(n), int(p)))
        f = c / (2 * np.pi) * np.hypot(x[n - 1] / 0.5, p * np.pi / 1.0) / 1e9
        assert abs(f - fa) < 1.0e-3


def test_spai_rows_are_the_rows_of_the_spai():
    """Rows of the SPAI computed alone, from only the column problems they
    need, equal the rows of the whole SPAI (to the rounding of the
    averaging order); conductor edges are refused."""
    import scipy.sparse as sp
    from oracle.spai import spai, spai_rows
    from synth import configs
    m = configs.cavity_mesh()
    topo = build_topology(m.nodes, m.tris, m.seg, m.tag)
    A = hodge_eps(topo)
    M = sp.csr_matrix(spai(A, topo.edge_free, 3, 1e-3))
    rows = np.random.default_rng(3).choice(np.flatnonzero(topo.edge_free), 40, replace=False)
    R = spai_rows(A, topo.edge_free, rows, 3, 1e-3)
    assert R.shape == (40, topo.n1)
    assert abs(R - M[rows]).max() <= 1e-15 * abs(M).max()
    assert R.nnz == M[rows].nnz
    with pytest.raises(ValueError):
        spai_rows(A, topo.edge_free, np.flatnonzero(~topo.edge_free)[:1])
