"""Host-side checks of the C ABI: the library loads and exports every
function include/axpic.h declares; enum values match the binding.  No
compute calls (no GPU needed)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "axpic.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(axp_[a-z_]+)\s*\(", src)) - {"axp_alloc_fn", "axp_free_fn"})


def test_header_declares_the_interface():
    names = _declared()
    for n in ("axp_create", "axp_build", "axp_step", "axp_diag_get", "axp_inject", "axp_get_fields"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1701_03784_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = pkg.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing
    assert sorted(pkg.EXPORTS) == _declared()


def test_enum_values_match_binding():
    import paper_1701_03784_amd.axpic as ax
    import synth
    src = open(HEADER).read()
    val = dict((k, int(v)) for k, v in re.findall(r"(AXP_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    assert val["AXP_BC_PEC"] == ax.BC_PEC == synth.BC_PEC
    assert val["AXP_BC_AXIS"] == ax.BC_AXIS == synth.BC_AXIS
    assert val["AXP_BC_EMITTER"] == ax.BC_EMITTER == synth.BC_EMITTER
    assert val["AXP_BC_OPEN"] == ax.BC_OPEN == synth.BC_OPEN
    assert val["AXP_PREC_MIXED"] == ax.PREC_MIXED
    assert val["AXP_PUSH_BORIS"] == ax.PUSH_BORIS
    assert val["AXP_PUSH_VAY"] == ax.PUSH_VAY
    for k, v in ax.ERRORS.items():
        assert val[v] == k


def _c_layout():
    """sizeof/offsetof of the ABI structs as a C compiler lays them out."""
    import subprocess
    import tempfile
    fields = {"axp_config": ["device", "hip_stream", "precision", "dt", "cfl_fraction", "spai_level", "spai_drop_tol",
                             "sort_period", "diag_every", "max_walk", "use_graph", "alloc", "free", "alloc_user",
                             "pusher"],
              "axp_info": ["n_nodes", "n_edges", "n_faces", "n_free_edges", "n_free_nodes", "spai_nnz",
                           "spai_fro_residual", "spai_max_col_residual", "dt", "dt_cfl", "setup_seconds",
                           "particle_capacity", "n_particles", "step", "precision", "n_species", "spai_mode",
                           "spai_fallback_columns", "spai_pred_resid_mean", "spai_kept_resid_mean",
                           "spai_energy_drift", "spai_seconds", "n_layer_faces", "spai_guard_trip_step",
                           "spai_run_drift", "spai_feature_seconds", "spai_infer_seconds", "spai_solve_seconds",
                           "sort_period", "window_lead"],
              "axp_diag": ["step", "n_live", "n_absorbed", "walk_overflow", "nan_count", "fixed_overflow",
                           "dce_max_abs", "dce_max_rel", "gauss_max_drift", "gauss_max_abs", "gauss_scale", "W_E",
                           "W_B", "W_K", "Q_total", "energy_step", "n_evals", "W_E_now"],
              "axp_energy": ["step", "n_live", "W_E", "W_B", "W_K", "Q_total"]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} sizeof %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "probe.c"), os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        st, f, v = line.split()
        res[(st, f)] = int(v)
    return res, fields


def test_struct_layout_matches_c_compiler():
    import ctypes as C
    import paper_1701_03784_amd.axpic as ax
    lay, fields = _c_layout()
    for st, cls in (("axp_config", ax.Config), ("axp_info", ax.Info), ("axp_diag", ax.Diag),
                    ("axp_energy", ax.Energy)):
        assert C.sizeof(cls) == lay[(st, "sizeof")], st
        for f in fields[st]:
            assert getattr(cls, f).offset == lay[(st, f)], (st, f)


def test_spai_enum_values():
    import paper_1701_03784_amd.axpic as ax
    src = open(HEADER).read()
    val = dict((k, int(v)) for k, v in re.findall(r"(AXP_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    assert val["AXP_SPAI_PLAIN"] == ax.SPAI_PLAIN
    assert val["AXP_SPAI_LEARNED"] == ax.SPAI_LEARNED
    assert val["AXP_SPAI_LEARNED_REJECTED"] == ax.SPAI_LEARNED_REJECTED
    assert val["AXP_SPAI_LEARNED_REVERTED"] == ax.SPAI_LEARNED_REVERTED


def test_spai_model_train_rejects_bad_arguments_before_any_device_work(tmp_path):
    """axp_spai_model_train checks its arguments and the mesh list before it
    touches the device: NULL arguments and an unreadable or empty list give
    AXP_E_ARG (runs without a GPU)."""
    import paper_1701_03784_amd as pkg
    lib = pkg.load_library()
    assert lib.axp_spai_model_train(None, b"x.bin", 0) == -1
    assert lib.axp_spai_model_train(str(tmp_path / "no_such_list.txt").encode(), None, 0) == -1
    assert lib.axp_spai_model_train(str(tmp_path / "no_such_list.txt").encode(), b"x.bin", 0) == -1
    empty = tmp_path / "empty.txt"
    empty.write_text("# nothing but a comment\n\n")
    assert lib.axp_spai_model_train(str(empty).encode(), str(tmp_path / "x.bin").encode(), 0) == -1
    assert not (tmp_path / "x.bin").exists()


def test_network_binding_rejects_unreadable_tensors_before_any_launch():
    """Mlp.forward / loss_grad refuse host tensors, other dtypes and
    non-contiguous views with ValueError before anything reaches the library
    (the kernels read float4 rows from device memory)."""
    import torch
    import paper_1701_03784_amd.axpic as ax
    net = ax.Mlp.__new__(ax.Mlp)          # no device handle: any library call would fail differently
    net.lib, net.h, net.device = None, None, 0
    X = torch.zeros(8, 16)
    y = torch.zeros(8)
    with pytest.raises(ValueError, match="cuda:0"):
        net.forward(X, y)
    with pytest.raises(ValueError, match="cuda:0"):
        net.loss_grad(X, y, y)
    with pytest.raises(ValueError):
        net.forward(X.double(), y)
    with pytest.raises(ValueError):
        net.loss_grad(X.t(), y, y)
    with pytest.raises(ValueError, match="torch tensor"):
        net.forward(X.numpy(), y)
    net.h = None
