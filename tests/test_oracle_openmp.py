"""The OpenMP form of the oracle step (used only to time the oracle on
several cores) computes what the serial form computes: with one thread bit
for bit, with four threads to the rounding of the current sums (the only
quantities summed across particles), and with the same particles."""

import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle.pic as op
op.use_openmp({omp})
import synth
from synth import configs
m = configs.cavity_mesh(h=0.8e-3)
sim = op.OracleSim(m.nodes, m.tris, m.seg, m.tag, dt=configs.CAVITY_DT)
E0, B0, _ = synth.tm010_fields(m.nodes, m.tris, sim.topo.edges, configs.CAVITY_A, 1e6, sim.dt)
sim.set_fields(E0, B0)
zr, u = configs.cavity_beam(3000, seed=2)
sim.inject(sim.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, configs.CAVITY_WEIGHT), zr, u)
sim.log_energies = True
sim.step(60)
np.savez({out!r}, E=sim.E, B=sim.B, D=sim.D, z=sim.pz, r=sim.prho, u=sim.pu, alive=sim.palive,
         Q=sim.Qres, W=np.array(sim.energy_log), stats=sim.stats)
"""


def _run(tmp_path, omp, threads):
    out = str(tmp_path / f"o_{int(omp)}_{threads}.npz")
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT, omp=omp, out=out)], check=True, env=env,
                   timeout=600)
    return np.load(out)


def test_openmp_oracle_matches_serial(tmp_path):
    a = _run(tmp_path, False, 1)
    b = _run(tmp_path, True, 1)
    c = _run(tmp_path, True, 4)
    for k in a.files:
        assert np.array_equal(a[k], b[k]), k          # one thread: the serial loop
    assert np.array_equal(a["alive"], c["alive"]) and np.array_equal(a["stats"], c["stats"])
    for k in ("E", "B", "D"):
        np.testing.assert_allclose(c[k], a[k], rtol=0, atol=1e-12 * np.abs(a[k]).max())
    for k in ("z", "r"):
        np.testing.assert_allclose(c[k], a[k], rtol=0, atol=1e-15)
    np.testing.assert_allclose(c["u"], a["u"], rtol=0, atol=1e-10 * np.abs(a["u"]).max())
    np.testing.assert_allclose(c["W"], a["W"], rtol=1e-12)
    np.testing.assert_allclose(c["Q"], a["Q"], rtol=0, atol=1e-12 * max(np.abs(a["Q"]).max(), 1e-30))
