"""Pin of the cold test (band edges of one period closed by conductor
plates at symmetry planes): for a smooth cylinder (no ripple) the two
lowest TM0 modes of the cell are the edges of the TM01 passband,
c x_01 / (2 pi r0) (phase advance 0) and c/(2 pi) sqrt((x_01/r0)^2 +
(pi/d)^2) (phase advance pi); the oracle's probe spectrum peaks there
within the coarse mesh's dispersion error (0.5 %).  Two periods between
the plates add the standing wave of phase advance pi/2 per period; for the
smooth guide all three lowest modes are the closed form
c/(2 pi) sqrt((x_01/r0)^2 + (k pi / (2 d))^2), k = 0, 1, 2."""

import numpy as np

import synth
from oracle.pic import OracleSim

C = 299792458.0
X01 = 2.404825557695773


R0, D = 0.015, 0.0167


def _ring(periods):
    """Probe spectrum peaks of `periods` smooth-guide periods rung for 12 ns."""
    m = synth.rippled_mesh(lambda z: np.full_like(np.asarray(z, float), R0), 0.0, periods * D, 0.8e-3,
                           seed=0, jitter=0.0)
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    sim.add_point_source(D / 3.0, 0.6 * R0, 1.0, 0.3e-9, 0.04e-9, 2 * np.pi * 10e9)
    sim.set_fields(np.zeros(sim.topo.n1), np.zeros(sim.topo.n2))
    sim.set_probe(0.21 * D, 0.31 * R0)
    sim.step(int(12e-9 / sim.dt))
    sig = np.array(sim.probe_signal)[int(0.6e-9 / sim.dt):]
    nfft = 8 * len(sig)
    f = np.fft.rfftfreq(nfft, sim.dt)
    P = sum(np.abs(np.fft.rfft(np.hanning(len(sig)) * sig[:, k], nfft)) ** 2 for k in range(2))
    # a peak is the maximum over +-6 bins of the unpadded transform (the Hann
    # window's main lobe and first sidelobes), above 1e-4 of the band's maximum
    W = 6 * 8
    band = (f > 0.5 * _closed(0.0)) & (f < 1.3 * _closed(np.pi))
    top = P[band].max()
    return f[[i for i in np.flatnonzero(band) if P[i] > 1e-4 * top and P[i] == P[max(0, i - W):i + W + 1].max()]]


def _closed(phase):
    return C / (2 * np.pi) * np.hypot(X01 / R0, phase / D)


def test_uniform_cell_band_edges():
    pk = _ring(1)
    assert len(pk) >= 2
    assert abs(pk[0] / _closed(0.0) - 1) < 5e-3
    assert abs(pk[1] / _closed(np.pi) - 1) < 5e-3


def test_two_periods_sample_the_dispersion_curve():
    pk = _ring(2)
    assert len(pk) >= 3
    for k in range(3):
        assert abs(pk[k] / _closed(k * np.pi / 2) - 1) < 3e-3
