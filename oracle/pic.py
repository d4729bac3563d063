"""Driver of the FP64 oracle: setup in numpy/scipy, per-step loop in C.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State is kept in the E-form of eqs. (full_d_dfl)/(full_d_dal): E^n on
edges, B^{n-1/2} on faces, particles with global (z, rho), their triangle
and u = gamma v.  D^n = [*eps]_a E^n is carried beside it for the discrete
Gauss law check of Sec. 3.5.2 ([*eps]_a = M^-1).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.spatial

from .topology import build_topology, AXIS
from .hodge import hodge_eps, hodge_mu_inv, EPS0, C_LIGHT
from .spai import spai
from .cfl import cfl_dt

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_step.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_pic.so")
TWO_PI = 2.0 * np.pi


_LIB_OMP = os.path.join(_HERE, "_build", "liboracle_pic_omp.so")


def build_oracle(force: bool = False, openmp: bool = False) -> str:
    """Compile pic_step.c with gcc, FP64 without value-changing
    optimisations: -O3 single thread, or -O3 -fopenmp for timing (particles
    split statically over the threads, per-thread buffers added in thread
    order)."""
    lib = _LIB_OMP if openmp else _LIB
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        tmp = lib + f".tmp{os.getpid()}"
        flags = ["-fopenmp"] if openmp else []
        subprocess.run(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fno-fast-math", *flags,
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, lib)
    return lib


_lib = None


def use_openmp(on: bool = True):
    """Selects the OpenMP build of the step for this process (timing of the
    oracle on several cores); must precede the first step."""
    global _OPENMP
    if _lib is not None and bool(on) != _OPENMP:
        raise RuntimeError("the oracle library is already loaded")
    _OPENMP = bool(on)


_OPENMP = False


def _load():
    global _lib
    if _lib is None:
        # ORACLE_PIC_LIBRARY: another build of pic_step.c (the sanitizer test's)
        alt = os.environ.get("ORACLE_PIC_LIBRARY")
        _lib = C.CDLL(alt if alt else build_oracle(openmp=_OPENMP))
        vp = C.c_void_p
        _lib.oracle_step.argtypes = [vp, vp, C.c_double, C.c_double, C.c_int, C.c_int64, vp, vp, vp] + [vp] * 9
        _lib.oracle_step.restype = None
        _lib.oracle_charge.argtypes = [vp, vp, vp, vp]
        _lib.oracle_sample.argtypes = [vp, C.c_int64, vp, vp, vp, vp, vp, vp]
        _lib.oracle_walk_only.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_double, C.c_double, vp, vp, vp]
        _lib.oracle_walk_only.restype = C.c_int
        _lib.oracle_boris.argtypes = [vp, vp, vp, C.c_double]
        _lib.oracle_vay.argtypes = [vp, vp, vp, C.c_double]
        _lib.oracle_move.argtypes = [C.c_double, C.c_double, vp, C.c_double, vp, vp]
        _lib.oracle_threads.restype = C.c_int
    return _lib


def oracle_threads() -> int:
    """Threads of the loaded oracle step (1 for the serial build)."""
    return int(_load().oracle_threads())


class _OMesh(C.Structure):
    _fields_ = [("n0", C.c_int64), ("n1", C.c_int64), ("n2", C.c_int64)] + \
               [(n, C.c_void_p) for n in ("nodes", "tris", "edges", "tri_edges", "tri_signs", "tri_nbr",
                                          "edge_tag", "edge_free", "H", "m_ptr", "m_col", "m_val")]


class _OParticles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(n, C.c_void_p) for n in
                                     ("z", "rho", "tri", "u", "alive", "species", "sp_qm", "sp_qw")]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class _OPml(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in ("face", "beta", "Az", "Ar", "h", "q", "eprev")]


def pml_sigma(topo, z_left, z_right, sigma_max, order):
    """Conductivity of the absorbing layers on each face (at its centroid):
    sigma_max (depth / thickness)^order beyond z_left (towards smaller z) and
    beyond z_right, 0 in between."""
    zc = topo.nodes[topo.tris][:, :, 0].mean(axis=1)
    z0, z1 = topo.nodes[:, 0].min(), topo.nodes[:, 0].max()
    sig = np.zeros(topo.n2)
    if z_left is not None and z_left > z0:
        m = zc < z_left
        sig[m] = sigma_max * ((z_left - zc[m]) / (z_left - z0)) ** order
    if z_right is not None and z_right < z1:
        m = zc > z_right
        sig[m] = sigma_max * ((zc[m] - z_right) / (z1 - z_right)) ** order
    return sig


class OracleSim:
    """Plain FP64 simulation of one meridian device."""

    def __init__(self, nodes, tris, seg, tag, dt=None, bz=0.0, spai_level=3, drop_tol=1e-3,
                 cfl_fraction=0.5, M=None, pml=None):
        """pml: optional dict(z_left, z_right, sigma_max, order) of the
        stretched-coordinate absorbing layers at the two ends (the time step
        is fixed first, without the layers; M is then the SPAI of the
        stretched Hodge)."""
        t0 = time.perf_counter()
        self.topo = build_topology(nodes, tris, seg, tag)
        self.A = hodge_eps(self.topo)
        self.H = hodge_mu_inv(self.topo)
        if pml is not None and dt is None:
            if M is not None:
                raise ValueError("with absorbing layers and a given M, give dt too")
            M0 = sp.csr_matrix(spai(self.A, self.topo.edge_free, spai_level, drop_tol))
            dt = cfl_fraction * cfl_dt(self.topo, self.H, M0)[0]
        self.pml = None
        self._pml_c = None
        self.K = self.A
        if pml is not None:
            from .hodge import pml_parts
            sig = pml_sigma(self.topo, pml.get("z_left"), pml.get("z_right"), pml["sigma_max"], pml.get("order", 3))
            faces = np.flatnonzero(sig > 0).astype(np.int64)
            beta = sig[faces] * dt / (2.0 * EPS0)
            Az, Ar = pml_parts(self.topo, faces)
            rows, cols, vals = [], [], []
            for i, t in enumerate(faces):
                ed = self.topo.tri_edges[t]
                dK = beta[i] * Ar[i] + (1.0 / (1.0 + beta[i]) - 1.0) * Az[i]
                for k in range(3):
                    for l in range(3):
                        rows.append(ed[k]); cols.append(ed[l]); vals.append(dK[k, l])
            self.K = (self.A + sp.csr_matrix((vals, (rows, cols)), shape=self.A.shape)).tocsr()
            self.pml = dict(face=faces, beta=np.ascontiguousarray(beta), Az=np.ascontiguousarray(Az.reshape(-1, 9)),
                            Ar=np.ascontiguousarray(Ar.reshape(-1, 9)), h=np.zeros(len(faces)),
                            q=np.zeros((len(faces), 3)), eprev=np.zeros((len(faces), 3)), sigma=sig)
        self.M = M if M is not None else spai(self.K, self.topo.edge_free, spai_level, drop_tol)
        self.M = sp.csr_matrix(self.M)
        self.M.sort_indices()
        self.dt_cfl, self.lam_max = cfl_dt(self.topo, self.H, self.M)
        self.dt = float(dt) if dt is not None else cfl_fraction * self.dt_cfl
        if self.pml is not None:
            if self.dt > self.dt_cfl:
                raise ValueError(f"dt {self.dt:.3e} above the stability limit {self.dt_cfl:.3e} of the layered scheme")
            P = self.pml
            self._pml_c = _OPml(len(P["face"]), *[_p(P[k]) for k in ("face", "beta", "Az", "Ar", "h", "q", "eprev")])
        self.bz = float(bz)
        self.pusher = 0                    # 0 relativistic Boris, 1 Vay
        self.sources = []                  # magnetic point sources: (face, amplitude, t0, sigma, omega)
        self.probe = None                  # (face, z, rho) of the field probe
        self.probe_signal = []             # (E_z, E_rho) at the probe at t^n, one per step
        self.setup_seconds = time.perf_counter() - t0
        tp = self.topo
        n0, n1, n2 = tp.n0, tp.n1, tp.n2
        self.E = np.zeros(n1)
        self.B = np.zeros(n2)
        self.D = np.zeros(n1)
        self.J = np.zeros(n1)
        self.Qres = np.zeros(n0)
        self._Bh = np.zeros(n2)
        self._rhs = np.zeros(n1)
        self.stats = np.zeros(3, dtype=np.int64)
        self.n_step = 0
        # energies of every step's starting time level n when log_energies is
        # set: (n, W_E, W_B, W_K, W_E_exact) per radian [J/rad] with
        # W_E = 1/2 E^n [*eps]_a E^n, W_B = 1/2 B^{n+1/2} H B^{n-1/2},
        # W_K = 1/2 (K^{n-1/2} + K^{n+1/2}) and W_E_exact = 1/2 E^n [*eps] E^n
        # (the exact Hodge); see oracle_step
        self.log_energies = False
        self.energy_log = []
        self._energy = np.zeros(4)
        # contiguous arrays handed to C
        self._arr = dict(
            nodes=np.ascontiguousarray(tp.nodes, dtype=np.float64),
            tris=np.ascontiguousarray(tp.tris, dtype=np.int64),
            edges=np.ascontiguousarray(tp.edges, dtype=np.int64),
            tri_edges=np.ascontiguousarray(tp.tri_edges, dtype=np.int64),
            tri_signs=np.ascontiguousarray(tp.tri_signs, dtype=np.int64),
            tri_nbr=np.ascontiguousarray(tp.tri_nbr, dtype=np.int64),
            edge_tag=np.ascontiguousarray(tp.edge_tag, dtype=np.int64),
            edge_free=np.ascontiguousarray(tp.edge_free, dtype=np.uint8),
            H=np.ascontiguousarray(self.H, dtype=np.float64),
            m_ptr=np.ascontiguousarray(self.M.indptr, dtype=np.int64),
            m_col=np.ascontiguousarray(self.M.indices, dtype=np.int64),
            m_val=np.ascontiguousarray(self.M.data, dtype=np.float64),
        )
        self._mesh = _OMesh(n0, n1, n2, *[_p(self._arr[k]) for k in (
            "nodes", "tris", "edges", "tri_edges", "tri_signs", "tri_nbr", "edge_tag", "edge_free",
            "H", "m_ptr", "m_col", "m_val")])
        # particles
        self.sp_qm = np.zeros(0)
        self.sp_qw = np.zeros(0)
        self.sp_m = np.zeros(0)
        self.sp_w = np.zeros(0)
        self.pz = np.zeros(0)
        self.prho = np.zeros(0)
        self.ptri = np.zeros(0, dtype=np.int64)
        self.pu = np.zeros((0, 3))
        self.palive = np.zeros(0, dtype=np.int8)
        self.pspecies = np.zeros(0, dtype=np.int64)
        self._tree = None
        self._Msolve = None
        self._emit = None          # (Emitter, species, per_step, seed, u_mean, u_spread)

    # ---------------------------------------------------------------- fields
    def set_fields(self, E0, B_mhalf):
        free = self.topo.edge_free
        self.E = np.where(free, np.asarray(E0, dtype=np.float64), 0.0)
        self.B = np.asarray(B_mhalf, dtype=np.float64).copy()
        self.D = self.eps_a(self.E)
        if self.pml is not None:
            # layer state of fields at rest: h = H B, q = A_z e, e^{-1} = e^0
            P = self.pml
            P["h"][:] = self.H[P["face"]] * self.B[P["face"]]
            ed = self.topo.tri_edges[P["face"]]
            P["eprev"][:] = self.E[ed]
            P["q"][:] = np.einsum("ikl,il->ik", P["Az"].reshape(-1, 3, 3), self.E[ed])

    def eps_a(self, E):
        """[*eps]_a E = M^-1 E on free edges (sparse direct solve)."""
        idx = np.flatnonzero(self.topo.edge_free)
        if self._Msolve is None:
            self._Msolve = spla.splu(self.M[idx][:, idx].tocsc())
        D = np.zeros(self.topo.n1)
        D[idx] = self._Msolve.solve(np.asarray(E)[idx])
        return D

    # ------------------------------------------------------------- particles
    def add_species(self, q, m, weight):
        self.sp_qm = np.append(self.sp_qm, q / m)
        self.sp_qw = np.append(self.sp_qw, q * weight)
        self.sp_m = np.append(self.sp_m, m)
        self.sp_w = np.append(self.sp_w, float(weight))
        return len(self.sp_qm) - 1

    def locate(self, zr):
        """Containing triangle of each point: the face among the nearest
        centroids whose smallest barycentric coordinate is largest.  The 8
        nearest centroids are tried first and the 24 nearest only for points
        none of those contains (a point inside a face has no larger smallest
        coordinate in any other face, so the wider search finds the same
        face)."""
        tp = self.topo
        if self._tree is None:
            self._tree = scipy.spatial.cKDTree(tp.nodes[tp.tris].mean(axis=1))
        zr = np.asarray(zr, dtype=np.float64).reshape(-1, 2)
        out = np.empty(len(zr), dtype=np.int64)

        def nearest(ids, k):
            """Best of the k nearest centroids; ids of points none contains."""
            miss = []
            for a in range(0, len(ids), 65536):      # bounded memory
                sel = ids[a:a + 65536]
                z = zr[sel]
                _, cand = self._tree.query(z, k=min(k, tp.n2))
                cand = np.asarray(cand).reshape(len(z), -1)
                minlam = _bary_many(tp.nodes[tp.tris[cand]], z[:, None, :]).min(axis=-1)
                out[sel] = cand[np.arange(len(z)), np.argmax(minlam, axis=1)]
                miss.extend(sel[minlam.max(axis=1) < -1e-12])
            return np.asarray(miss, dtype=np.int64)

        bad = nearest(nearest(np.arange(len(zr)), 8), 24)
        for i in bad:                        # far from any centroid: scan all faces
            ml = _bary_many(tp.nodes[tp.tris], zr[i][None, :]).min(axis=-1)
            if ml.max() < -1e-9:
                raise ValueError(f"point {zr[i]} is outside the mesh")
            out[i] = int(np.argmax(ml))
        return out.astype(np.int64)

    def inject(self, species, zr, u):
        zr = np.asarray(zr, dtype=np.float64).reshape(-1, 2)
        u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
        tri = self.locate(zr)
        n = len(zr)
        self.pz = np.concatenate([self.pz, zr[:, 0]])
        self.prho = np.concatenate([self.prho, zr[:, 1]])
        self.ptri = np.concatenate([self.ptri, tri])
        self.pu = np.concatenate([self.pu, u], axis=0)
        self.palive = np.concatenate([self.palive, np.ones(n, dtype=np.int8)])
        self.pspecies = np.concatenate([self.pspecies, np.full(n, species, dtype=np.int64)])

    def _parts(self):
        self.pz = np.ascontiguousarray(self.pz)
        self.prho = np.ascontiguousarray(self.prho)
        self.ptri = np.ascontiguousarray(self.ptri, dtype=np.int64)
        self.pu = np.ascontiguousarray(self.pu)
        self.palive = np.ascontiguousarray(self.palive)
        self.pspecies = np.ascontiguousarray(self.pspecies)
        self.sp_qm = np.ascontiguousarray(self.sp_qm)
        self.sp_qw = np.ascontiguousarray(self.sp_qw)
        return _OParticles(len(self.pz), _p(self.pz), _p(self.prho), _p(self.ptri), _p(self.pu),
                           _p(self.palive), _p(self.pspecies), _p(self.sp_qm), _p(self.sp_qw))

    def set_injector(self, species, per_step, u_mean, u_spread, seed):
        """Continuous emission at the start of every step (see oracle.inject)."""
        from .inject import Emitter
        if per_step == 0:
            self._emit = None
            return
        self._emit = (Emitter(self.topo), int(species), int(per_step), int(seed),
                      np.asarray(u_mean, dtype=np.float64), float(u_spread))

    def _inject_step(self):
        em, sp_, k, seed, um, us = self._emit
        z, rho, face, u, ta, hb, wa = em.emit(self.n_step, k, seed, um, us)
        q_ring = self.sp_qw[sp_] / (2.0 * np.pi)
        np.subtract.at(self.Qres, ta, q_ring * wa)
        np.subtract.at(self.Qres, hb, q_ring * (1.0 - wa))
        self.pz = np.concatenate([self.pz, z])
        self.prho = np.concatenate([self.prho, rho])
        self.ptri = np.concatenate([self.ptri, face])
        self.pu = np.concatenate([self.pu, u], axis=0)
        self.palive = np.concatenate([self.palive, np.ones(k, dtype=np.int8)])
        self.pspecies = np.concatenate([self.pspecies, np.full(k, sp_, dtype=np.int64)])

    # ------------------------------------------------------------------ step
    def add_point_source(self, z, rho, amplitude, t0, sigma, omega):
        """Magnetic point source of Sec. 4.1 at (z, rho): the magnetic current
        M(t) = amplitude exp(-((t - t0) / (2 sigma))^2) cos(omega (t - t0))
        drives the flux of the face holding the point."""
        face = int(self.locate(np.array([[z, rho]]))[0])
        self.sources.append((face, float(amplitude), float(t0), float(sigma), float(omega)))

    def set_probe(self, z, rho):
        """Record (E_z, E_rho) at (z, rho) at the start of every step (t^n)."""
        self.probe = (int(self.locate(np.array([[z, rho]]))[0]), float(z), float(rho))
        self.probe_signal = []

    def _source_values(self):
        t = self.n_step * self.dt
        return np.array([a * np.exp(-((t - t0) / (2.0 * sg)) ** 2) * np.cos(w * (t - t0))
                         for (_, a, t0, sg, w) in self.sources], dtype=np.float64)

    def step(self, n=1):
        lib = _load()
        P = self._parts()
        src_face = np.array([f for (f, *_r) in self.sources], dtype=np.int64)
        for _ in range(n):
            if self._emit is not None:
                self._inject_step()
                P = self._parts()
            if self.probe is not None:
                f, z, r = self.probe
                e = self.sample(np.array([f]), np.array([z]), np.array([r]))[0]
                self.probe_signal.append((e[0], e[1]))
            src_val = self._source_values()
            log = self.log_energies
            we_exact = 0.5 * self.E @ (self.A @ self.E) if log else 0.0
            lib.oracle_step(C.byref(self._mesh), C.byref(P), self.dt, self.bz, int(self.pusher),
                            len(src_face), _p(src_face), _p(src_val),
                            None if self._pml_c is None else C.byref(self._pml_c),
                            _p(self.E), _p(self.B), _p(self.D), _p(self.J), _p(self.Qres),
                            _p(self._Bh), _p(self._rhs), _p(self.stats), _p(self._energy) if log else None)
            if log:
                e = self._energy
                self.energy_log.append((self.n_step, float(e[0]), float(e[1]), float(e[2]), float(we_exact)))
            self.n_step += 1

    # ----------------------------------------------------------- diagnostics
    def charge(self):
        """Q^n per node, eq. (charge), including absorbed wall charge."""
        lib = _load()
        P = self._parts()
        Q = np.zeros(self.topo.n0)
        lib.oracle_charge(C.byref(self._mesh), C.byref(P), _p(self.Qres), _p(Q))
        return Q

    def gauss_residual(self, D=None):
        """res^n = D~div [*eps]_a E^n - Q^n (Sec. 3.5.2), on every node."""
        D = self.D if D is None else D
        return self.topo.Ddiv @ D - self.charge()

    def kinetic_energy(self):
        """sum over live particles of (m w c^2 / 2 pi)(gamma - 1) [J/rad] at
        the momenta held now (u^{n-1/2} after n steps)."""
        a = self.palive.astype(bool)
        w2 = (self.pu[a] ** 2).sum(axis=1) / C_LIGHT ** 2
        sp_ = self.pspecies[a]
        return float(np.sum(self.sp_w[sp_] * self.sp_m[sp_] * (w2 / (np.sqrt(1.0 + w2) + 1.0)))
                     * C_LIGHT ** 2 / TWO_PI)

    def sample(self, tri, z, rho):
        lib = _load()
        tri = np.ascontiguousarray(tri, dtype=np.int64)
        z = np.ascontiguousarray(z, dtype=np.float64)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.zeros((len(tri), 3))
        lib.oracle_sample(C.byref(self._mesh), len(tri), _p(tri), _p(z), _p(rho), _p(self.E), _p(self.B), _p(out))
        return out

    def walk_only(self, p, z_end, rho_end, J):
        lib = _load()
        P = self._parts()
        return lib.oracle_walk_only(C.byref(self._mesh), C.byref(P), int(p), float(z_end), float(rho_end),
                                    self.dt, _p(J), _p(self.Qres), _p(self.stats))

    def particles(self):
        a = self.palive.astype(bool)
        return (np.stack([self.pz[a], self.prho[a]], axis=1), self.pu[a].copy(), self.pspecies[a].copy())


def _bary_many(v, r):
    """Barycentric coordinates of points r (..., 2) in triangles v (..., 3, 2)."""
    A = 0.5 * ((v[..., 1, 0] - v[..., 0, 0]) * (v[..., 2, 1] - v[..., 0, 1])
               - (v[..., 2, 0] - v[..., 0, 0]) * (v[..., 1, 1] - v[..., 0, 1]))
    out = []
    for i in range(3):
        pj, pk = v[..., (i + 1) % 3, :], v[..., (i + 2) % 3, :]
        out.append(0.5 * ((pj[..., 0] - r[..., 0]) * (pk[..., 1] - r[..., 1])
                          - (pk[..., 0] - r[..., 0]) * (pj[..., 1] - r[..., 1])) / A)
    return np.stack(out, axis=-1)


def _bary_np(v, r):
    """Barycentric coordinates of point r in triangle with vertices v (3, 2)."""
    lam = np.empty(3)
    A = 0.5 * ((v[1, 0] - v[0, 0]) * (v[2, 1] - v[0, 1]) - (v[2, 0] - v[0, 0]) * (v[1, 1] - v[0, 1]))
    for i in range(3):
        pj, pk = v[(i + 1) % 3], v[(i + 2) % 3]
        lam[i] = 0.5 * ((pj[0] - r[0]) * (pk[1] - r[1]) - (pk[0] - r[0]) * (pj[1] - r[1])) / A
    return lam


def boris(u, E, B, k):
    """Python handle on the oracle's Boris rotation (u is modified copy)."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib.oracle_boris(_p(u), _p(E), _p(B), float(k))
    return u


def vay(u, E, B, k):
    """Python handle on the oracle's Vay pusher (u is modified copy)."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lib.oracle_vay(_p(u), _p(E), _p(B), float(k))
    return u


def move(z, rho, u, dt):
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    zn = C.c_double()
    rn = C.c_double()
    lib.oracle_move(float(z), float(rho), _p(u), float(dt), C.byref(zn), C.byref(rn))
    return zn.value, rn.value, u
