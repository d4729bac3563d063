"""Pin of the cold test (band edges of one period closed by conductor
plates at symmetry planes): for a smooth cylinder (no ripple) the two
lowest TM0 modes of the cell are the edges of the TM01 passband,
c x_01 / (2 pi r0) (phase advance 0) and c/(2 pi) sqrt((x_01/r0)^2 +
(pi/d)^2) (phase advance pi); the oracle's probe spectrum peaks there
within the coarse mesh's dispersion error (0.5 %)."""

import numpy as np

import synth
from oracle.pic import OracleSim

C = 299792458.0
X01 = 2.404825557695773


def test_uniform_cell_band_edges():
    r0, d = 0.015, 0.0167
    m = synth.rippled_mesh(lambda z: np.full_like(np.asarray(z, float), r0), 0.0, d, 0.8e-3, seed=0, jitter=0.0)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    sim.add_point_source(d / 3.0, 0.6 * r0, 1.0, 0.3e-9, 0.04e-9, 2 * np.pi * 10e9)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(0.21 * d, 0.31 * r0)
    sim.step(int(12e-9 / sim.dt))
    sig = np.array(sim.probe_signal)[int(0.6e-9 / sim.dt):]
    nfft = 8 * len(sig)
    f = np.fft.rfftfreq(nfft, sim.dt)
    P = sum(np.abs(np.fft.rfft(np.hanning(len(sig)) * sig[:, k], nfft)) ** 2 for k in range(2))
    f0 = C / (2 * np.pi) * X01 / r0
    fp = C / (2 * np.pi) * np.hypot(X01 / r0, np.pi / d)
    # a peak is the maximum over +-6 bins of the unpadded transform (the Hann
    # window's main lobe and first sidelobes), above 1e-4 of the band's maximum
    W = 6 * 8
    band = (f > 0.5 * f0) & (f < 1.3 * fp)
    top = P[band].max()
    pk = [i for i in np.flatnonzero(band) if P[i] > 1e-4 * top and P[i] == P[max(0, i - W):i + W + 1].max()]
    assert len(pk) >= 2
    assert abs(f[pk[0]] / f0 - 1) < 5e-3
    assert abs(f[pk[1]] / fp - 1) < 5e-3
