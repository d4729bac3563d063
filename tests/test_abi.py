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
    for k, v in ax.ERRORS.items():
        assert val[v] == k


def test_struct_sizes_match_header_layout():
    import ctypes as C
    import paper_1701_03784_amd.axpic as ax
    # axp_config: 4 int + pointer, see include/axpic.h (natural alignment)
    assert C.sizeof(ax.Config) == 96
    assert C.sizeof(ax.Diag) == 7 * 8 + 8 * 8
    assert C.sizeof(ax.Info) == 6 * 8 + 5 * 8 + 3 * 8 + 2 * 4
