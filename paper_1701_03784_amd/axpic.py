"""Thin Python binding of the axpic C ABI (include/axpic.h).

Argument marshalling only: numpy arrays are handed to the library as host
pointers; every step of the simulation runs in the library's HIP kernels.
PyTorch, when present, supplies the HIP stream (and, optionally, device
memory through the allocator callback).  The binding refuses to run
without the built library: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libaxpic.so")

AXP_OK = 0
ERRORS = {-1: "AXP_E_ARG", -2: "AXP_E_MESH", -3: "AXP_E_SPAI", -4: "AXP_E_UNSTABLE", -5: "AXP_E_OOM",
          -6: "AXP_E_HIP", -7: "AXP_E_WALK", -8: "AXP_E_FIXED_OVERFLOW", -9: "AXP_E_NAN", -10: "AXP_E_STATE"}
BC_PEC, BC_AXIS, BC_EMITTER, BC_OPEN = 1, 2, 3, 4
PREC_PLAIN_FP64, PREC_MIXED = 0, 1
PUSH_BORIS, PUSH_VAY = 0, 1
SPAI_PLAIN, SPAI_LEARNED, SPAI_LEARNED_REJECTED, SPAI_LEARNED_REVERTED = 0, 1, 2, 3
SPAI_FEATURES = 16

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class AxpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [("device", C.c_int32), ("hip_stream", C.c_void_p), ("precision", C.c_int32),
                ("dt", C.c_double), ("cfl_fraction", C.c_double), ("spai_level", C.c_int32),
                ("spai_drop_tol", C.c_double), ("sort_period", C.c_int32), ("diag_every", C.c_int32),
                ("max_walk", C.c_int32), ("use_graph", C.c_int32), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p), ("pusher", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_edges", C.c_int64), ("n_faces", C.c_int64),
                ("n_free_edges", C.c_int64), ("n_free_nodes", C.c_int64), ("spai_nnz", C.c_int64),
                ("spai_fro_residual", C.c_double), ("spai_max_col_residual", C.c_double),
                ("dt", C.c_double), ("dt_cfl", C.c_double), ("setup_seconds", C.c_double),
                ("particle_capacity", C.c_int64), ("n_particles", C.c_int64), ("step", C.c_int64),
                ("precision", C.c_int32), ("n_species", C.c_int32), ("spai_mode", C.c_int32), ("pad_", C.c_int32),
                ("spai_fallback_columns", C.c_int64), ("spai_pred_resid_mean", C.c_double),
                ("spai_kept_resid_mean", C.c_double), ("spai_energy_drift", C.c_double), ("spai_seconds", C.c_double),
                ("n_layer_faces", C.c_int64), ("spai_guard_trip_step", C.c_int64), ("spai_run_drift", C.c_double),
                ("spai_feature_seconds", C.c_double), ("spai_infer_seconds", C.c_double),
                ("spai_solve_seconds", C.c_double), ("sort_period", C.c_int32), ("window_lead", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_live", C.c_int64), ("n_absorbed", C.c_int64),
                ("walk_overflow", C.c_int64), ("nan_count", C.c_int64), ("fixed_overflow", C.c_int64),
                ("dce_max_abs", C.c_int64), ("dce_max_rel", C.c_double), ("gauss_max_drift", C.c_double),
                ("gauss_max_abs", C.c_double), ("gauss_scale", C.c_double), ("W_E", C.c_double),
                ("W_B", C.c_double), ("W_K", C.c_double), ("Q_total", C.c_double),
                ("energy_step", C.c_int64), ("n_evals", C.c_int64), ("W_E_now", C.c_double)]


class Energy(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_live", C.c_int64), ("W_E", C.c_double), ("W_B", C.c_double),
                ("W_K", C.c_double), ("Q_total", C.c_double)]


EXPORTS = ["axp_config_default", "axp_create", "axp_set_mesh", "axp_set_boundary", "axp_build",
           "axp_info_get", "axp_get_edges", "axp_get_spai", "axp_set_fields", "axp_set_electrostatic", "axp_set_layers", "axp_add_point_source",
           "axp_clear_point_sources", "axp_set_probe", "axp_get_probe", "axp_set_external_bz",
           "axp_add_species", "axp_inject", "axp_set_injector", "axp_step", "axp_sync", "axp_diag_get",
           "axp_get_energies",
           "axp_get_fields", "axp_get_sources", "axp_get_particles", "axp_save", "axp_load",
           "axp_last_error", "axp_destroy", "axp_batch_create", "axp_batch_step", "axp_batch_sync",
           "axp_batch_destroy", "axp_set_timing", "axp_get_timing", "axp_autotune", "axp_batch_autotune",
           "axp_batch_set_timing", "axp_batch_get_timing", "axp_batch_info", "axp_batch_last_error",
           "axp_mlp_create", "axp_mlp_n_params", "axp_mlp_set_params", "axp_mlp_get_params", "axp_mlp_forward",
           "axp_mlp_loss_grad", "axp_mlp_loss_grad_noalloc", "axp_mlp_adam_step", "axp_mlp_info", "axp_mlp_save", "axp_mlp_load",
           "axp_mlp_last_error", "axp_mlp_destroy", "axp_set_spai_model", "axp_set_spai_run_guard", "axp_spai_pairs",
           "axp_spai_model_load", "axp_spai_model_train"]
PHASES = ["face", "particles", "edge", "spmv", "sort", "diag", "inject", "walk"]

_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libaxpic.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1701_03784_amd.build.build()")
    try:
        # PyTorch carries its own HIP runtime; load it first so that the
        # library binds to the same one (one HIP runtime per process)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "axp_config_default": (None, [C.POINTER(Config)]),
        "axp_create": (i32, [C.POINTER(Config), C.POINTER(vp)]),
        "axp_set_mesh": (i32, [vp, i32, vp, i32, vp]),
        "axp_set_boundary": (i32, [vp, i32, vp, vp]),
        "axp_build": (i32, [vp]),
        "axp_info_get": (i32, [vp, C.POINTER(Info)]),
        "axp_get_edges": (i32, [vp, vp]),
        "axp_get_spai": (i32, [vp, i64, C.POINTER(i64), vp, vp, vp]),
        "axp_set_fields": (i32, [vp, vp, vp]),
        "axp_set_electrostatic": (i32, [vp, vp, i32, vp]),
        "axp_set_layers": (i32, [vp, i32, dbl, dbl, dbl, i32]),
        "axp_add_point_source": (i32, [vp, dbl, dbl, dbl, dbl, dbl, dbl]),
        "axp_clear_point_sources": (i32, [vp]),
        "axp_set_probe": (i32, [vp, dbl, dbl, i64]),
        "axp_get_probe": (i32, [vp, i64, C.POINTER(i64), vp]),
        "axp_set_external_bz": (i32, [vp, dbl]),
        "axp_add_species": (i32, [vp, dbl, dbl, i64, C.POINTER(i32)]),
        "axp_inject": (i32, [vp, i32, i64, vp, vp]),
        "axp_set_injector": (i32, [vp, i32, i64, vp, dbl, C.c_uint64]),
        "axp_step": (i32, [vp, i32]),
        "axp_sync": (i32, [vp]),
        "axp_diag_get": (i32, [vp, C.POINTER(Diag)]),
        "axp_get_energies": (i32, [vp, i64, C.POINTER(i64), C.POINTER(Energy)]),
        "axp_get_fields": (i32, [vp, vp, vp]),
        "axp_get_sources": (i32, [vp, vp, vp, vp]),
        "axp_get_particles": (i32, [vp, i64, C.POINTER(i64), vp, vp, vp]),
        "axp_save": (i32, [vp, C.c_char_p]),
        "axp_load": (i32, [vp, C.c_char_p]),
        "axp_last_error": (C.c_char_p, [vp]),
        "axp_destroy": (None, [vp]),
        "axp_batch_create": (i32, [vp, i32, C.POINTER(vp)]),
        "axp_batch_step": (i32, [vp, i32]),
        "axp_batch_sync": (i32, [vp]),
        "axp_batch_destroy": (None, [vp]),
        "axp_set_timing": (i32, [vp, i32]),
        "axp_get_timing": (i32, [vp, vp, vp]),
        "axp_autotune": (i32, [vp, i32, C.POINTER(i32)]),
        "axp_batch_autotune": (i32, [vp, i32, C.POINTER(i32)]),
        "axp_batch_set_timing": (i32, [vp, i32]),
        "axp_batch_get_timing": (i32, [vp, vp, vp]),
        "axp_batch_info": (i32, [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]),
        "axp_batch_last_error": (C.c_char_p, [vp]),
        "axp_mlp_create": (i32, [i32, vp, i32, i32, i32, i32, C.c_uint64, C.POINTER(vp)]),
        "axp_mlp_n_params": (i64, [vp]),
        "axp_mlp_set_params": (i32, [vp, vp]),
        "axp_mlp_get_params": (i32, [vp, vp]),
        "axp_mlp_forward": (i32, [vp, vp, i64, vp]),
        "axp_mlp_loss_grad": (i32, [vp, vp, vp, vp, i64, C.POINTER(dbl), vp]),
        "axp_mlp_loss_grad_noalloc": (i32, [vp, vp, vp, vp, i64, vp, vp]),
        "axp_mlp_adam_step": (i32, [vp, dbl, dbl, dbl, dbl]),
        "axp_mlp_info": (i32, [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(i64)]),
        "axp_mlp_save": (i32, [vp, C.c_char_p]),
        "axp_mlp_load": (i32, [i32, vp, C.c_char_p, C.POINTER(vp)]),
        "axp_mlp_last_error": (C.c_char_p, [vp]),
        "axp_mlp_destroy": (None, [vp]),
        "axp_set_spai_model": (i32, [vp, vp, dbl, dbl, i32]),
        "axp_set_spai_run_guard": (i32, [vp, dbl]),
        "axp_spai_pairs": (i32, [vp, i64, C.POINTER(i64), vp, vp, vp]),
        "axp_spai_model_load": (i32, [vp, C.c_char_p]),
        "axp_spai_model_train": (i32, [C.c_char_p, C.c_char_p, C.c_uint64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, user):
        self.live.pop(int(ptr) if ptr else 0, None)


def current_torch_stream(device=0):
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream(device).cuda_stream
    except Exception:
        pass
    return None


class Ctx:
    """One simulated device (mesh + fields + particles) on one GPU."""

    def __init__(self, precision=PREC_MIXED, dt=0.0, cfl_fraction=0.5, spai_level=3, spai_drop_tol=1e-3,
                 sort_period=4, diag_every=0, max_walk=64, use_graph=1, device=0, stream=None,
                 torch_memory=False, pusher=PUSH_BORIS):
        self.lib = load_library()
        cfg = Config()
        self.lib.axp_config_default(C.byref(cfg))
        cfg.device, cfg.precision, cfg.dt, cfg.cfl_fraction = device, precision, dt, cfl_fraction
        cfg.spai_level, cfg.spai_drop_tol, cfg.sort_period = spai_level, spai_drop_tol, sort_period
        cfg.diag_every, cfg.max_walk, cfg.use_graph = diag_every, max_walk, use_graph
        cfg.pusher = pusher
        cfg.hip_stream = stream if stream is not None else current_torch_stream(device)
        self._allocator = None
        if torch_memory:
            self._allocator = TorchAllocator(device)
            cfg.alloc, cfg.free = self._allocator.alloc_cb, self._allocator.free_cb
        self.cfg = cfg
        h = C.c_void_p()
        self._check(self.lib.axp_create(C.byref(cfg), C.byref(h)), None)
        self.h = h

    def _check(self, st, h="self"):
        if st != AXP_OK:
            msg = ""
            if h is not None and getattr(self, "h", None):
                msg = (self.lib.axp_last_error(self.h) or b"").decode()
            raise AxpError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.axp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup
    def set_mesh(self, nodes, tris):
        self._nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        self._tris = np.ascontiguousarray(tris, dtype=np.int32)
        self._check(self.lib.axp_set_mesh(self.h, len(self._nodes), _ptr(self._nodes), len(self._tris), _ptr(self._tris)))

    def set_boundary(self, seg, tag):
        seg = np.ascontiguousarray(seg, dtype=np.int32)
        tag = np.ascontiguousarray(tag, dtype=np.uint8)
        self._check(self.lib.axp_set_boundary(self.h, len(seg), _ptr(seg), _ptr(tag)))

    def build(self):
        self._check(self.lib.axp_build(self.h))

    def info(self):
        i = Info()
        self._check(self.lib.axp_info_get(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def get_edges(self):
        n = self.info()["n_edges"]
        e = np.zeros((n, 2), dtype=np.int32)
        self._check(self.lib.axp_get_edges(self.h, _ptr(e)))
        return e

    def get_spai(self):
        import scipy.sparse as sp
        n = self.info()["n_edges"]
        nnz = C.c_int64()
        rowptr = np.zeros(n + 1, dtype=np.int64)
        self.lib.axp_get_spai(self.h, 0, C.byref(nnz), _ptr(rowptr), None, None)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._check(self.lib.axp_get_spai(self.h, nnz.value, C.byref(nnz), _ptr(rowptr), _ptr(col), _ptr(val)))
        return sp.csr_matrix((val, col, rowptr), shape=(n, n))

    def set_fields(self, E0, B_mhalf):
        E0 = np.ascontiguousarray(E0, dtype=np.float64)
        B = np.ascontiguousarray(B_mhalf, dtype=np.float64)
        self._check(self.lib.axp_set_fields(self.h, _ptr(E0), _ptr(B)))

    def set_electrostatic(self, phi_conductor=None, with_charge=False):
        """Gauss-consistent electrostatic fields (axp_set_electrostatic);
        returns the nodal potential."""
        n0 = self.info()["n_nodes"]
        phi = np.zeros(n0)
        pc = None if phi_conductor is None else np.ascontiguousarray(phi_conductor, dtype=np.float64)
        self._check(self.lib.axp_set_electrostatic(self.h, None if pc is None else _ptr(pc), int(bool(with_charge)),
                                                   _ptr(phi)))
        return phi

    def add_point_source(self, z, rho, amplitude, t0, sigma, omega):
        """Magnetic point source with a Gaussian-modulated pulse (axp_add_point_source)."""
        self._check(self.lib.axp_add_point_source(self.h, float(z), float(rho), float(amplitude), float(t0),
                                                  float(sigma), float(omega)))

    def clear_point_sources(self):
        self._check(self.lib.axp_clear_point_sources(self.h))

    def set_probe(self, z, rho, capacity):
        """Record E at (z, rho) at the start of each of the next `capacity` steps."""
        self._check(self.lib.axp_set_probe(self.h, float(z), float(rho), int(capacity)))

    def get_probe(self):
        """(n, 2) array of (E_z, E_rho) recorded so far."""
        n = C.c_int64()
        self._check(self.lib.axp_get_probe(self.h, 0, C.byref(n), None))
        out = np.zeros((n.value, 2))
        if n.value:
            self._check(self.lib.axp_get_probe(self.h, n.value, C.byref(n), _ptr(out)))
        return out

    def set_external_bz(self, bz):
        self._check(self.lib.axp_set_external_bz(self.h, float(bz)))

    def add_species(self, q, m, weight):
        sid = C.c_int32()
        self._check(self.lib.axp_add_species(self.h, float(q), float(m), int(weight), C.byref(sid)))
        return sid.value

    def inject(self, species, zr, u):
        zr = np.ascontiguousarray(zr, dtype=np.float64).reshape(-1, 2)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1, 3)
        self._check(self.lib.axp_inject(self.h, int(species), len(zr), _ptr(zr), _ptr(u)))

    def set_injector(self, species, per_step, u_mean, u_spread, seed):
        um = np.ascontiguousarray(u_mean, dtype=np.float64)
        self._check(self.lib.axp_set_injector(self.h, int(species), int(per_step), _ptr(um), float(u_spread), int(seed)))

    # ---- run
    def step(self, n=1):
        self._check(self.lib.axp_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.axp_sync(self.h))

    def diag(self):
        d = Diag()
        self._check(self.lib.axp_diag_get(self.h, C.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def energies(self, capacity=4096):
        """Energy records of the diagnostic steps not yet returned, oldest
        first: a structured array (step, n_live, W_E, W_B, W_K, Q_total)."""
        buf = (Energy * max(1, int(capacity)))()
        n = C.c_int64()
        self._check(self.lib.axp_get_energies(self.h, int(capacity), C.byref(n), buf))
        dt = np.dtype([(k, np.int64 if t is C.c_int64 else np.float64) for k, t in Energy._fields_])
        out = np.zeros(n.value, dtype=dt)
        for i in range(n.value):
            for k, _ in Energy._fields_:
                out[i][k] = getattr(buf[i], k)
        return out

    def set_timing(self, on=True):
        self._check(self.lib.axp_set_timing(self.h, 1 if on else 0))

    def save(self, path):
        self._check(self.lib.axp_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(self.lib.axp_load(self.h, str(path).encode()))

    def set_spai_model(self, net, row_tol=0.01, energy_drift_tol=1e-6, iters=3):
        """Learned SPAI for the next build (net: Mlp or None)."""
        self._spai_model = net
        self._check(self.lib.axp_set_spai_model(self.h, net.h if net is not None else None, float(row_tol),
                                                float(energy_drift_tol), int(iters)))

    def set_spai_run_guard(self, drift_tol):
        """Arms (drift_tol >= 0) or disarms (< 0) the run-time energy guard
        of the learned SPAI (axp_set_spai_run_guard)."""
        self._check(self.lib.axp_set_spai_run_guard(self.h, float(drift_tol)))

    def spai_model_load(self, path):
        """Learned SPAI for the next build from a saved network file
        (axp_spai_model_load; the context owns the loaded network)."""
        self._check(self.lib.axp_spai_model_load(self.h, str(path).encode()))

    def spai_pairs(self):
        """(X[n][16] float32, y[n] float32, kj[n][2] int32) of the built context."""
        n = C.c_int64()
        self._check(self.lib.axp_spai_pairs(self.h, 0, C.byref(n), None, None, None))
        X = np.zeros((n.value, SPAI_FEATURES), dtype=np.float32)
        y = np.zeros(n.value, dtype=np.float32)
        kj = np.zeros((n.value, 2), dtype=np.int32)
        self._check(self.lib.axp_spai_pairs(self.h, n.value, C.byref(n), _ptr(X), _ptr(y), _ptr(kj)))
        return X, y, kj

    def autotune(self, trial_steps=16):
        """Chooses the sort period, then the particle kernel's window lead, by
        timing real steps (or from the AXP_AUTOTUNE_CACHE file); returns the
        period (info() has both)."""
        sp = C.c_int32()
        self._check(self.lib.axp_autotune(self.h, int(trial_steps), C.byref(sp)))
        return sp.value

    def get_timing(self):
        """{phase: (total device ms, launches)} since set_timing(True)."""
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int64)
        self._check(self.lib.axp_get_timing(self.h, _ptr(ms), _ptr(n)))
        return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(PHASES)}

    # ---- read-back
    def get_fields(self):
        i = self.info()
        E = np.zeros(i["n_edges"])
        B = np.zeros(i["n_faces"])
        self._check(self.lib.axp_get_fields(self.h, _ptr(E), _ptr(B)))
        return E, B

    def get_sources(self):
        i = self.info()
        D = np.zeros(i["n_edges"])
        J = np.zeros(i["n_edges"])
        Q = np.zeros(i["n_nodes"])
        self._check(self.lib.axp_get_sources(self.h, _ptr(D), _ptr(J), _ptr(Q)))
        return D, J, Q

    def get_particles(self):
        n = C.c_int64()
        self.lib.axp_get_particles(self.h, 0, C.byref(n), None, None, None)
        cap = n.value
        zr = np.zeros((cap, 2))
        u = np.zeros((cap, 3))
        sp = np.zeros(cap, dtype=np.int32)
        self._check(self.lib.axp_get_particles(self.h, cap, C.byref(n), _ptr(zr), _ptr(u), _ptr(sp)))
        return zr[:n.value], u[:n.value], sp[:n.value]


def write_mesh(path, mesh):
    """Writes a mesh (synth.Mesh-like: nodes, tris, seg, tag) in the text
    format axp_spai_model_train reads."""
    nodes = np.asarray(mesh.nodes, dtype=np.float64)
    tris = np.asarray(mesh.tris, dtype=np.int64)
    seg = np.asarray(mesh.seg, dtype=np.int64)
    tag = np.asarray(mesh.tag, dtype=np.int64)
    with open(path, "w") as f:
        f.write(f"axpic-mesh 1\n{len(nodes)} {len(tris)} {len(seg)}\n")
        np.savetxt(f, nodes, fmt="%.17g")
        np.savetxt(f, tris, fmt="%d")
        np.savetxt(f, np.column_stack([seg, tag]), fmt="%d")


def spai_model_train(mesh_list, out_model, seed=0):
    """Trains and saves a learned-SPAI network natively (axp_spai_model_train):
    mesh_list is a text file naming one write_mesh file per line."""
    lib = load_library()
    st = lib.axp_spai_model_train(str(mesh_list).encode(), str(out_model).encode(), int(seed))
    if st != AXP_OK:
        raise AxpError(st, "axp_spai_model_train")


def make_ctx(mesh, spai_model=None, spai_row_tol=0.01, spai_energy_tol=1e-6, spai_iters=3, layers=None, **kw):
    """Context with mesh and boundary set and built (mesh: synth.Mesh-like).
    layers: optional dict(z_left=None, z_right=None, sigma_max, order=3) of
    absorbing layers (axp_set_layers)."""
    c = Ctx(**kw)
    c.set_mesh(mesh.nodes, mesh.tris)
    c.set_boundary(mesh.seg, mesh.tag)
    if layers is not None:
        zl, zr = layers.get("z_left"), layers.get("z_right")
        sides = (1 if zl is not None else 0) | (2 if zr is not None else 0)
        c._check(c.lib.axp_set_layers(c.h, sides, float(zl or 0.0), float(zr or 0.0), float(layers["sigma_max"]),
                                      int(layers.get("order", 3))))
    if spai_model is not None:
        c.set_spai_model(spai_model, spai_row_tol, spai_energy_tol, spai_iters)
    c.build()
    return c


DEFAULT_SPAI_MODEL = os.path.join(_HERE, "spai_mlp_l3.bin")


def default_spai_model(device=0, stream=None):
    """The network trained by train_spai.py on 48 seeded rippled-wall tubes
    (level-3 pattern, 16 -> 64 -> 64 -> 1)."""
    return Mlp.load(DEFAULT_SPAI_MODEL, device=device, stream=stream)


def _dptr(t):
    """Device address of a contiguous torch tensor (device memory plumbing)."""
    return C.c_void_p(t.data_ptr())


def _check_dev(name, t, device, shape, dtype="float32"):
    """Rejects what the network kernels cannot read: host or other-device
    tensors, other dtypes (float32 unless stated), non-contiguous views,
    wrong shapes."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: a torch tensor is required")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{name}: must live on cuda:{device} (got {t.device})")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name}: {dtype} required (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")


class Mlp:
    """The learned-SPAI network (axp_mlp_*): its kernels run on the device."""

    def __init__(self, n_hidden=64, n_layers=2, spai_level=3, seed=0, device=0, stream=None, _handle=None):
        self.lib = load_library()
        self.device = int(device)
        if _handle is not None:
            self.h = _handle
        else:
            h = C.c_void_p()
            st = self.lib.axp_mlp_create(device, stream if stream is not None else current_torch_stream(device),
                                         SPAI_FEATURES, n_hidden, n_layers, spai_level, int(seed), C.byref(h))
            if st != AXP_OK:
                raise AxpError(st, "axp_mlp_create")
            self.h = h

    @classmethod
    def load(cls, path, device=0, stream=None):
        lib = load_library()
        h = C.c_void_p()
        st = lib.axp_mlp_load(device, stream if stream is not None else current_torch_stream(device),
                              str(path).encode(), C.byref(h))
        if st != AXP_OK:
            raise AxpError(st, f"axp_mlp_load {path}")
        return cls(_handle=h, device=device)

    def _check(self, st):
        if st != AXP_OK:
            raise AxpError(st, (self.lib.axp_mlp_last_error(self.h) or b"").decode())

    def n_params(self):
        return int(self.lib.axp_mlp_n_params(self.h))

    def info(self):
        v = [C.c_int32() for _ in range(4)] + [C.c_int64()]
        self._check(self.lib.axp_mlp_info(self.h, *[C.byref(x) for x in v]))
        return dict(zip(["n_in", "n_hidden", "n_layers", "spai_level", "adam_steps"], [x.value for x in v]))

    def get_params(self):
        p = np.zeros(self.n_params(), dtype=np.float32)
        self._check(self.lib.axp_mlp_get_params(self.h, _ptr(p)))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params()
        self._check(self.lib.axp_mlp_set_params(self.h, _ptr(p)))

    def _n_in(self):
        return self.info()["n_in"]

    def forward(self, X, y_out):
        """X (n, n_in), y_out (n,): contiguous float32 torch tensors on the
        network's device (ValueError otherwise, before any launch)."""
        _check_dev("X", X, self.device, None)
        _check_dev("y_out", y_out, self.device, None)
        n = int(X.shape[0]) if X.dim() == 2 else -1
        _check_dev("X", X, self.device, (n, self._n_in()))
        _check_dev("y_out", y_out, self.device, (n,))
        self._check(self.lib.axp_mlp_forward(self.h, _dptr(X), n, _dptr(y_out)))

    def loss_grad(self, X, y, w, want_grad=False):
        """X (n, n_in), y and w (n,): contiguous float32 tensors on the
        network's device (ValueError otherwise, before any launch)."""
        for name, t in (("X", X), ("y", y), ("w", w)):
            _check_dev(name, t, self.device, None)
        n = int(X.shape[0]) if X.dim() == 2 else -1
        _check_dev("X", X, self.device, (n, self._n_in()))
        _check_dev("y", y, self.device, (n,))
        _check_dev("w", w, self.device, (n,))
        loss = C.c_double()
        g = np.zeros(self.n_params(), dtype=np.float32) if want_grad else None
        self._check(self.lib.axp_mlp_loss_grad(self.h, _dptr(X), _dptr(y), _dptr(w), n, C.byref(loss),
                                               _ptr(g)))
        return (loss.value, g) if want_grad else loss.value

    def loss_grad_noalloc(self, X, y, w, loss_out, grad_out):
        """Allocation-free loss and gradient (axp_mlp_loss_grad_noalloc):
        X (n, n_in), y and w (n,) float32, loss_out (2,) float64 and
        grad_out (n_params,) float32, all contiguous on the network's device.
        Enqueued on the network's stream; nothing is synchronised."""
        for name, t in (("X", X), ("y", y), ("w", w), ("grad_out", grad_out)):
            _check_dev(name, t, self.device, None)
        _check_dev("loss_out", loss_out, self.device, (2,), dtype="float64")
        n = int(X.shape[0]) if X.dim() == 2 else -1
        _check_dev("X", X, self.device, (n, self._n_in()))
        _check_dev("y", y, self.device, (n,))
        _check_dev("w", w, self.device, (n,))
        _check_dev("grad_out", grad_out, self.device, (self.n_params(),))
        self._check(self.lib.axp_mlp_loss_grad_noalloc(self.h, _dptr(X), _dptr(y), _dptr(w), n, _dptr(loss_out),
                                                       _dptr(grad_out)))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.lib.axp_mlp_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def save(self, path):
        self._check(self.lib.axp_mlp_save(self.h, str(path).encode()))

    def close(self):
        if getattr(self, "h", None):
            self.lib.axp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Pool of built contexts advanced together (axp_batch_*).  The member
    contexts must stay alive while the batch exists; their state is read
    back by sync()."""

    def __init__(self, ctxs):
        self.lib = load_library()
        self.ctxs = list(ctxs)
        arr = (C.c_void_p * len(self.ctxs))(*[c.h for c in self.ctxs])
        h = C.c_void_p()
        st = self.lib.axp_batch_create(arr, len(self.ctxs), C.byref(h))
        if st != AXP_OK:
            raise AxpError(st, (self.lib.axp_last_error(self.ctxs[0].h) or b"").decode())
        self.h = h

    def _check(self, st):
        if st != AXP_OK:
            raise AxpError(st, (self.lib.axp_batch_last_error(self.h) or b"").decode())

    def step(self, n=1):
        self._check(self.lib.axp_batch_step(self.h, int(n)))

    def sync(self):
        self._check(self.lib.axp_batch_sync(self.h))

    def autotune(self, trial_steps=16):
        sp = C.c_int32()
        self._check(self.lib.axp_batch_autotune(self.h, int(trial_steps), C.byref(sp)))
        return sp.value

    def set_timing(self, on=True):
        self._check(self.lib.axp_batch_set_timing(self.h, 1 if on else 0))

    def get_timing(self):
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int64)
        self._check(self.lib.axp_batch_get_timing(self.h, _ptr(ms), _ptr(n)))
        return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(PHASES)}

    def info(self):
        v = [C.c_int64() for _ in range(4)]
        self._check(self.lib.axp_batch_info(self.h, *[C.byref(x) for x in v]))
        return dict(zip(["n_faces", "n_edges", "n_particles", "step"], [x.value for x in v]))

    def close(self):
        if getattr(self, "h", None):
            self.lib.axp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
