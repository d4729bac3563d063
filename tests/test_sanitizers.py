"""The library's host code and the oracle's C step under the address and
undefined-behaviour sanitizers (CPU builds with g++/gcc; the GPU kernels are
not involved).

- host setup (topology, Hodge, plain and learned SPAI, stability limit,
  conjugate gradients, energy guard, point location, absorbing layers):
  tests/native/host_setup_check.cpp linked with csrc/host_setup.cpp, run on
  the cavity mesh and a short rippled tube;
- the oracle's step (push, walk, current, charge, emission, energies):
  oracle/pic_step.c built as a sanitized shared library and loaded by a
  child interpreter with the address-sanitizer runtime preloaded, on the
  cavity with a beam and on the 1 mm diode with emission.
Any sanitizer report fails the run (halt_on_error).
"""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import synth
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


pytestmark = pytest.mark.skipif(shutil.which("g++") is None or _runtime("libasan.so") is None,
                                reason="no g++ with the sanitizer runtimes")


def _write_mesh(path, m):
    with open(path, "wb") as f:
        np.array([len(m.nodes), len(m.tris), len(m.seg)], dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.nodes, dtype=np.float64).tofile(f)
        np.ascontiguousarray(m.tris, dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.seg, dtype=np.int32).tofile(f)
        np.ascontiguousarray(m.tag, dtype=np.uint8).tofile(f)


def test_host_setup_under_sanitizers(tmp_path):
    exe = tmp_path / "host_setup_check"
    cmd = ["g++", "-std=c++17", *SAN, "-pthread", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           os.path.join(ROOT, "tests", "native", "host_setup_check.cpp"),
           os.path.join(ROOT, "paper_1701_03784_amd", "csrc", "host_setup.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    for name, m in (("cavity", configs.cavity_mesh()),
                    ("tube", configs.bwo_mesh(seed=5, h=0.8e-3, n_periods=2, up=0.004, down=0.004))):
        p = tmp_path / f"{name}.mesh"
        _write_mesh(p, m)
        r = subprocess.run([str(exe), str(p)], capture_output=True, text=True, env=ENV, timeout=600)
        print(name, r.stdout.strip())
        assert r.returncode == 0, r.stdout + r.stderr[-4000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


ORACLE_RUN = r"""
import sys, numpy as np
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import synth
from synth import configs
from oracle.pic import OracleSim
QE, ME = synth.ELECTRON_CHARGE, synth.ELECTRON_MASS
m = configs.cavity_mesh()
sim = OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=configs.CAVITY_DT, bz=0.5)
E0, B0, _ = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, configs.CAVITY_A, 1e6, sim.dt)
sim.set_fields(E0, B0)
zr, u = configs.cavity_beam(500, seed=3)
sim.inject(sim.add_species(QE, ME, configs.CAVITY_WEIGHT), zr, u)
sim.log_energies = True
sim.step(40)
d = configs.diode_mesh(h=1.0e-3)
s2 = OracleSim(d.nodes, d.tris, d.seg, d.tag)
phi = configs.DIODE_VOLTS * d.nodes[:, 0] / configs.DIODE_GAP
e = s2.topo.edges
s2.set_fields(-(phi[e[:, 1]] - phi[e[:, 0]]), np.zeros(s2.topo.n2))
s2.set_injector(s2.add_species(QE, ME, 2000), 40, [0.0, 0.0, 5.9e5], 1e5, seed=7)
s2.step(60)
print("oracle ok", int(sim.palive.sum()), int(s2.palive.sum()), len(sim.energy_log))
"""


def test_oracle_step_under_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_pic_san.so"
    subprocess.run(["gcc", "-std=c99", *SAN, "-fPIC", "-shared", "-fno-fast-math", "-o", str(lib),
                    os.path.join(ROOT, "oracle", "pic_step.c"), "-lm"], check=True, capture_output=True)
    env = dict(ENV, ORACLE_PIC_LIBRARY=str(lib), LD_PRELOAD=_runtime("libasan.so"))
    code = ORACLE_RUN.format(root=ROOT, tests=os.path.join(ROOT, "tests"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout.strip())
    assert r.returncode == 0 and "oracle ok" in r.stdout, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
