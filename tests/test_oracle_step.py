"""Pins of the oracle's time step: field leapfrog, gather, push, scatter,
charge conservation and the discrete Gauss law.

References used: the exact dispersion of the leapfrog on a discrete
eigenmode; the discrete energy it conserves; the analytic TM010 frequency
(the paper's Table 1 accuracy level); closed forms of the Boris rotation and
of a gyro-orbit about the axis; the pairing property of Whitney forms; an
independent quadrature of the current line integral; and the exact
identities of Sec. 3.4 (DCE, DGL invariance).
"""

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle.pic import OracleSim, boris, move
from oracle.cfl import curl_curl

C = 299792458.0
QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS


def _c1_sim(dt=None, level=3):
    m = synth.rect_mesh(0.0, 0.02, 0.01, 0.49e-3, seed=0)
    return m, OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=dt, spai_level=level)


@pytest.fixture(scope="module")
def c1():
    return _c1_sim()


# ------------------------------------------------------------------- fields
def test_leapfrog_eigenmode_phase_is_exact():
    """Source-free, E^n = cos(n theta) v for a generalised eigenpair
    K v = lam M^-1 v when B^{-1/2} = (dt/2) C v, with sin(theta/2) = dt sqrt(lam)/2."""
    m = synth.rect_mesh(0.0, 0.006, 0.004, 0.8e-3, seed=4)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, spai_level=2)
    idx = np.flatnonzero(sim.topo.edge_free)
    K = curl_curl(sim.topo, sim.H).toarray()[np.ix_(idx, idx)]
    Minv = np.linalg.inv(sim.M.toarray()[np.ix_(idx, idx)])
    lam, V = scipy.linalg.eigh(K, Minv)
    j = int(np.searchsorted(lam, 1e-6 * lam.max())) + 3       # a low non-static mode
    v = np.zeros(sim.topo.n1)
    v[idx] = V[:, j]
    sim.set_fields(v, 0.5 * sim.dt * (sim.topo.C @ v))
    theta = 2 * np.arcsin(sim.dt * np.sqrt(lam[j]) / 2)
    w = np.zeros(sim.topo.n1)
    w[idx] = Minv @ V[:, j]
    vv = v @ w
    for n in range(1, 301):
        sim.step(1)
        if n % 50 == 0:
            assert (sim.E @ w) / vv == pytest.approx(np.cos(n * theta), abs=1e-10)


def test_source_free_discrete_energy_is_conserved(c1):
    """1/2 E^n M^-1 E^n + 1/2 B^{n+1/2} H B^{n-1/2} is invariant for the
    leapfrog pair (full_d_dfl)/(full_d_dal) without sources."""
    m, sim0 = c1
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    E0, B0, _ = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, 0.01, 1e6, sim.dt)
    sim.set_fields(E0, B0)

    def energy():
        Bh = sim.B - sim.dt * (sim.topo.C @ sim.E)
        return 0.5 * sim.E @ sim.eps_a(sim.E) + 0.5 * Bh @ (sim.H * sim.B)

    W0 = energy()
    for _ in range(10):
        sim.step(50)
        assert energy() == pytest.approx(W0, rel=1e-11)


def test_tm010_frequency(c1):
    """C1 cavity (a = 1 cm): the field solver's TM010 frequency is within
    2e-3 of c x 2.4048/(2 pi a) (Table 1's TM010 error is 8.3e-4)."""
    m, sim0 = c1
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    E0, B0, omega = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, 0.01, 1e6, sim.dt)
    sim.set_fields(E0, B0)
    ref = sim.E.copy()
    proj = []
    for _ in range(1000):
        proj.append(sim.E @ ref / (ref @ ref))
        sim.step(1)
    proj = np.array(proj)
    i = np.flatnonzero(np.sign(proj[1:]) != np.sign(proj[:-1]))
    tz = (i + proj[i] / (proj[i] - proj[i + 1])) * sim.dt
    f = 1.0 / (2 * np.mean(np.diff(tz)))
    assert abs(f / (omega / (2 * np.pi)) - 1) < 2e-3


# ------------------------------------------------------------------- gather
def test_whitney_reproduces_uniform_field(c1):
    m, sim = c1
    e0 = (2.5e5, -4.0e5)
    sim.E = synth.uniform_field_dofs(sim.topo.nodes, sim.topo.edges, *e0)
    rng = np.random.default_rng(3)
    tri = rng.integers(0, sim.topo.n2, 200)
    lam = rng.dirichlet([1, 1, 1], 200)
    pts = np.einsum("ij,ijk->ik", lam, sim.topo.nodes[sim.topo.tris[tri]])
    out = sim.sample(tri, pts[:, 0], pts[:, 1])
    np.testing.assert_allclose(out[:, 0], e0[0], rtol=1e-10)
    np.testing.assert_allclose(out[:, 1], e0[1], rtol=1e-10)


def test_whitney_pairing_with_edges(c1):
    """<edge_i, w1_j> = delta_ij (eq. paring, App. A) along every edge of a face."""
    m, sim = c1
    tp = sim.topo
    x, w = np.polynomial.legendre.leggauss(4)
    x, w = 0.5 * (x + 1), 0.5 * w
    rng = np.random.default_rng(5)
    for t in rng.integers(0, tp.n2, 20):
        for j in tp.tri_edges[t]:
            sim.E = np.zeros(tp.n1)
            sim.E[j] = 1.0
            for i in tp.tri_edges[t]:
                a, b = tp.nodes[tp.edges[i, 0]], tp.nodes[tp.edges[i, 1]]
                pts = a + x[:, None] * (b - a)
                f = sim.sample(np.full(len(x), t), pts[:, 0], pts[:, 1])
                val = np.sum(w * (f[:, 0] * (b - a)[0] + f[:, 1] * (b - a)[1]))
                assert val == pytest.approx(1.0 if i == j else 0.0, abs=1e-12)


# --------------------------------------------------------------------- push
def test_boris_uniform_electric_field():
    u0 = np.array([1.0e7, -2.0e6, 3.0e7])
    E = np.array([4.0e5, 0.0, -7.0e5])
    k = QE / ME * 1e-13 / 2
    u1 = boris(u0, E, np.zeros(3), k)
    np.testing.assert_allclose(u1, u0 + 2 * k * E, rtol=1e-14)


def test_boris_uniform_magnetic_rotation():
    """E = 0: |u| is kept and u turns by 2 atan(|q| B dt / (2 gamma m)) per step."""
    u0 = np.array([2.0e8, 1.0e8, 5.0e7])
    B = np.array([0.0, 0.0, 1.5])
    dt = 2e-12
    g = np.sqrt(1 + u0 @ u0 / C ** 2)
    u1 = boris(u0, np.zeros(3), B, QE / ME * dt / 2)
    assert np.linalg.norm(u1) == pytest.approx(np.linalg.norm(u0), rel=1e-14)
    ang = np.arctan2(u0[0] * u1[1] - u0[1] * u1[0], u0[0] * u1[0] + u0[1] * u1[1])
    assert abs(ang) == pytest.approx(2 * np.arctan(abs(QE) * 1.5 * dt / (2 * g * ME)), rel=1e-12)
    assert u1[2] == u0[2]


@pytest.mark.parametrize("kev", [5.0, 500.0])
def test_gyro_orbit_about_the_axis(kev):
    """Uniform B_z, E = 0, guiding centre on the axis: the discrete Boris
    orbit is a regular polygon inscribed in a circle of radius
    R = |v| dt / (2 sin(theta/2)), so the axisymmetric push must keep
    rho = R and (u_rho, u_phi) = |u| (sin(theta/2), cos(theta/2)) in the
    local frame at every step."""
    Bz, dt = 1.0, 1e-12
    g, beta = synth.gamma_beta_from_kev(kev)
    v = beta * C
    theta = 2 * np.arctan(abs(QE) * Bz * dt / (2 * g * ME))
    R = v * dt / (2 * np.sin(theta / 2))
    un = g * v
    u = np.array([un * np.sin(theta / 2), un * np.cos(theta / 2), 0.0])
    z, rho = 0.0, R
    for _ in range(500):
        u = boris(u, np.zeros(3), np.array([0.0, 0.0, Bz]), QE / ME * dt / 2)
        z, rho, u = move(z, rho, u, dt)
        assert rho == pytest.approx(R, rel=1e-10)
        np.testing.assert_allclose(u[:2], [un * np.sin(theta / 2), un * np.cos(theta / 2)], rtol=1e-9)
    assert z == 0.0


# ------------------------------------------------------------------ scatter
def _bary_independent(nodes, tris, t, p):
    v = nodes[tris[t]]
    Mx = np.array([[1, v[i, 0], v[i, 1]] for i in range(3)])
    return np.array([1.0, p[0], p[1]]) @ np.linalg.inv(Mx)


def _locate_independent(nodes, tris, p):
    for t in range(len(tris)):
        lam = _bary_independent(nodes, tris, t, p)
        if lam.min() >= -1e-12:
            return t
    raise AssertionError


def test_current_equals_line_integral_across_faces(c1):
    """J_e = (q/2 pi/dt) int W1_e . dr along a straight path crossing many
    faces, against a fine midpoint quadrature with independently computed
    barycentric coordinates."""
    m, sim0 = c1
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=1e-12, M=sim0.M)
    tp = sim.topo
    sp_ = sim.add_species(QE, ME, 1.0)
    p0 = np.array([0.0071, 0.0043])
    p1 = np.array([0.0102, 0.0021])          # ~6 edge lengths away
    sim.inject(sp_, p0[None, :], np.zeros((1, 3)))
    J = np.zeros(tp.n1)
    nseg = sim.walk_only(0, p1[0], p1[1], J)
    assert nseg >= 5
    assert sim.ptri[0] == _locate_independent(tp.nodes, tp.tris, p1)
    coef = QE / (2 * np.pi) / sim.dt
    # independent breakpoints: intersections of the path with every mesh edge
    d = p1 - p0
    cuts = [0.0, 1.0]
    for a, b in tp.nodes[tp.edges]:
        e = b - a
        den = d[0] * (-e[1]) - d[1] * (-e[0])
        if den == 0:
            continue
        rhs = a - p0
        s_ = (rhs[0] * (-e[1]) - rhs[1] * (-e[0])) / den
        r_ = (d[0] * rhs[1] - d[1] * rhs[0]) / den
        if 0 < s_ < 1 and 0 <= r_ <= 1:
            cuts.append(s_)
    cuts = np.unique(cuts)
    gx, gw = np.polynomial.legendre.leggauss(2)
    ref = np.zeros(tp.n1)
    for s0, s1 in zip(cuts[:-1], cuts[1:]):
        t = _locate_independent(tp.nodes, tp.tris, p0 + 0.5 * (s0 + s1) * d)
        v = tp.nodes[tp.tris[t]]
        inv = np.linalg.inv(np.array([[1, v[i, 0], v[i, 1]] for i in range(3)]))
        grads = inv[1:, :].T
        for xg, wg in zip(gx, gw):
            s = s0 + (s1 - s0) * 0.5 * (xg + 1)
            lam = _bary_independent(tp.nodes, tp.tris, t, p0 + s * d)
            for k in range(3):
                e = tp.tri_edges[t, k]
                a = int(np.where(tp.tris[t] == tp.edges[e, 0])[0][0])
                b = int(np.where(tp.tris[t] == tp.edges[e, 1])[0][0])
                W = lam[a] * grads[b] - lam[b] * grads[a]
                ref[e] += 0.5 * wg * (s1 - s0) * (W @ d)
    ref *= coef
    assert len(cuts) - 1 == nseg
    np.testing.assert_allclose(J, ref, rtol=0, atol=1e-12 * abs(ref).max())


def test_dce_per_particle_and_gauss_invariance(c1):
    """Eq. (DCE) per step (rounding level, and the paper's normalised
    residual below 1e-10), and eq. (DGL_RSD_REL):
    the Gauss residual of every free node stays at its initial value to
    rounding (relative to the size of the summed terms) over 1000 steps, for
    both D^n and the brute-force M^-1 E^n of the E-form state."""
    m, sim0 = c1
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=sim0.dt, M=sim0.M)
    E0, B0, _ = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, 0.01, 1e6, sim.dt)
    sim.set_fields(E0, B0)
    sp_ = sim.add_species(QE, ME, 1.0e4)
    zr, u = synth.disk_beam(3000, 0.002, 0.0, 0.02, 0.5, seed=1)
    sim.inject(sp_, zr, u)
    free = sim.topo.node_free
    absD = abs(sim.topo.Ddiv)
    Q0 = sim.charge()
    g0 = sim.gauss_residual()
    qscale = np.abs(Q0).max()
    Qp = Q0
    for n in range(1000):
        sim.step(1)
        Q = sim.charge()
        divJ = sim.dt * (sim.topo.Ddiv @ sim.J)
        dce = (Q - Qp) + divJ
        assert np.abs(dce).max() <= 1e-13 * qscale
        # normalised residual of Sec. 5.1.1: 1 + dQ/(dt div J), below the
        # paper's 1e-10 peak level wherever the denominator is not tiny
        big = np.abs(divJ) > 1e-3 * max(np.abs(divJ).max(), 1e-300)
        if big.any():
            assert np.abs(1 + (Q - Qp)[big] / divJ[big]).max() < 1e-10
        Qp = Q
        if n % 100 == 99:
            scale = (absD @ np.abs(sim.D)).max()
            assert np.abs((sim.gauss_residual() - g0)[free]).max() <= 1e-13 * scale
            gE = sim.topo.Ddiv @ sim.eps_a(sim.E) - Q
            assert np.abs((gE - g0)[free]).max() <= 1e-11 * scale
    assert sim.stats[1] > 0          # particles reached the end plates and were absorbed
    assert sim.stats[2] == 0


def test_tiny_mesh_one_step_by_hand():
    """Two-triangle mesh, one particle, uniform E_z, no B: after one step
    u = q E dt / m exactly; the position moves by v dt along z; the current
    of the straight piece equals (q/2pi/dt)(lam_t^0 lam_h^1 - lam_h^0 lam_t^1)
    with barycentric coordinates taken from the affine map by hand."""
    m = synth.tiny_mesh("two")             # square [0,1] x [1,2], rho >= 1
    m.tag[:] = synth.BC_OPEN                 # free field boundary: the uniform E survives
    dt = 1e-12
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=dt, spai_level=1)
    ez = 1.0e4
    E0 = synth.uniform_field_dofs(sim.topo.nodes, sim.topo.edges, ez, 0.0)
    sim.set_fields(E0, np.zeros(2))
    sp_ = sim.add_species(QE, ME, 1.0)
    p0 = np.array([0.6, 1.2])                 # inside face 0 = (0,1,2): z > rho - 1
    sim.inject(sp_, p0[None, :], np.zeros((1, 3)))
    sim.step(1)
    uz = QE / ME * ez * dt
    assert sim.pu[0, 2] == pytest.approx(uz, rel=1e-14)
    g = np.sqrt(1 + (uz / C) ** 2)
    p1 = p0 + np.array([uz / g * dt, 0.0])
    assert sim.pz[0] == pytest.approx(p1[0], abs=1e-15) and sim.prho[0] == pytest.approx(p1[1], abs=1e-15)
    # face 0 nodes (0,0,1),(1,1,1),(2,1,2) in (z, rho): lam0 = 1 - z, lam1 = z - rho + 1, lam2 = rho - 1
    lam = lambda p: np.array([1 - p[0], p[0] - p[1] + 1, p[1] - 1])
    l0, l1 = lam(p0), lam(p1)
    coef = QE / (2 * np.pi) / dt
    idx = {tuple(e): i for i, e in enumerate(sim.topo.edges)}
    for (a, b) in [(0, 1), (1, 2), (0, 2)]:
        assert sim.J[idx[(a, b)]] == pytest.approx(coef * (l0[a] * l1[b] - l0[b] * l1[a]), rel=1e-12)
    assert sim.J[idx[(2, 3)]] == 0.0 and sim.J[idx[(0, 3)]] == 0.0
