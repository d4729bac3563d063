"""Cold test of the slow-wave structure: band edges of the TM01 passband
under mesh refinement (the cold test of Sec. 5 and the staircasing study of Sec. 5.1.2), run on the GPU.

    python -m paper_1701_03784_amd.cold_test [--amp 0.0025] [--period 0.0167] [--r0 0.015]
                                             [--h 0.4e-3 0.2e-3 0.1e-3] [--ns 60]
                                             [--mesh hex grid staircase] [--periods 1]

One period of the rippled wall R(z) = r0 + amp cos(2 pi z / d) is closed by
conductor plates at z = 0 and z = d.  Both plates lie at symmetry planes of
the wall (its extrema), so the modes of this cell are the Floquet modes of
the periodic structure with phase advance 0 and pi per period: the lowest
two TM0 modes are the two edges of the TM01 passband, the upper one the
pi point at which the backward-wave oscillator works.  A broadband
magnetic point source rings the cell; the probe's spectrum gives the mode
frequencies (Hann window, zero padding, parabolic peak refinement), on
successively refined meshes.  With amp = 0 the two edges are the closed
forms c/(2 pi) x_01/r0 and c/(2 pi) sqrt((x_01/r0)^2 + (pi/d)^2).

With N periods between the plates the closed structure's standing waves
have phase advance k pi / N per period (k = 0 .. N), so its lowest N + 1
modes sample the TM01 dispersion curve at those phases, without periodic
(Floquet) boundaries; for a smooth guide they are the closed form
c/(2 pi) sqrt((x_01/r0)^2 + (k pi / (N d))^2).

The staircasing study of Sec. 5.1.2 compares a wall that follows R(z) with
the step-cell wall a structured grid would impose: 'grid' and 'staircase'
meshes share their triangles and differ only at the wall, so the change of
the pi-point frequency between them is the staircasing error alone.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

C_LIGHT = 299792458.0
X01 = 2.404825557695773


def log(msg):
    print(f"[cold] {msg}", file=sys.stderr, flush=True)


MESH_KINDS = ("hex", "grid", "staircase")


def cell_mesh(r0, amp, d, h, seed=0, kind="hex", periods=1):
    """Mesh of the cell r <= r0 + amp cos(2 pi z / d), 0 <= z <= periods * d.

    kind 'hex': a regular (unjittered) hexagonal lattice mapped onto the wall;
    'grid': a checkerboard-split grid mapped onto the wall; 'staircase': the
    same grid with the wall rounded to whole grid rows per column (the
    step-cell wall of a structured grid, with vertical risers)."""
    import synth
    R = lambda z: r0 + amp * np.cos(2.0 * np.pi * np.asarray(z, dtype=np.float64) / d)
    L = periods * d
    if kind == "hex":
        return synth.rippled_mesh(R, 0.0, L, h, seed=seed, jitter=0.0)
    if kind in ("grid", "staircase"):
        return synth.grid_mesh(R, 0.0, L, h, staircase=kind == "staircase")
    raise ValueError(f"unknown mesh kind {kind!r}")


def lowest_peaks(signal, dt, f_lo, f_hi, count=2, pad=8, floor=1e-4):
    """The lowest `count` spectral peaks in (f_lo, f_hi) above floor x max."""
    w = np.hanning(len(signal))
    nfft = pad * len(signal)
    f = np.fft.rfftfreq(nfft, dt)
    P = sum(np.abs(np.fft.rfft(w * signal[:, k], nfft)) ** 2 for k in range(signal.shape[1]))
    band = (f > f_lo) & (f < f_hi)
    top = P[band].max()
    # a peak is the maximum over +-6 bins of the unpadded transform (the Hann
    # window's main lobe and first sidelobes), above floor x the band's maximum
    W = 6 * pad
    pk = [i for i in np.flatnonzero(band) if P[i] > floor * top and P[i] == P[max(0, i - W):i + W + 1].max()]
    out = []
    for i in pk[:count]:
        y0, y1, y2 = np.log(P[i - 1]), np.log(P[i]), np.log(P[i + 1])
        out.append(float(f[i] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (f[1] - f[0])))
    return out


def uniform_dispersion(r0, d, phase):
    """TM01 frequency of a smooth guide of radius r0 at phase advance `phase`
    per length d (the closed form the rippled wall's band bends away from)."""
    return C_LIGHT / (2 * np.pi) * np.hypot(X01 / r0, np.asarray(phase, dtype=np.float64) / d)


def cell_modes(ctx_factory, m, r0, d, ns, f_lo, f_hi, count=2, chunk=500_000):
    """The `count` lowest TM0 modes of a closed cell (mesh m) rung by a
    broadband magnetic point source and read at a probe in the first period.
    Returns (frequencies, faces, steps).  For `periods` periods between
    plates at symmetry planes the lowest periods + 1 modes are the TM01 band
    at phase advance k pi / periods, k = 0 .. periods."""
    c = ctx_factory(m)
    info = c.info()
    dt = info["dt"]
    c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
    c.add_point_source(d / 3.0, 0.6 * r0, 1.0, 0.3e-9, 0.04e-9, 2 * np.pi * 10e9)
    steps = int(ns * 1e-9 / dt)
    c.set_probe(0.21 * d, 0.31 * r0, steps)
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        c.step(n)
        done += n
        if done < steps:
            log(f"{info['n_faces']} faces: {done}/{steps} steps")
    sig = c.get_probe()
    c.close()
    n0 = int(0.6e-9 / dt)                       # after the pulse
    return lowest_peaks(sig[n0:], dt, f_lo, f_hi, count=count), info["n_faces"], steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--r0", type=float, default=0.015)
    ap.add_argument("--amp", type=float, default=0.0025)
    ap.add_argument("--period", type=float, default=0.0167)
    ap.add_argument("--h", type=float, nargs="+", default=[0.4e-3, 0.2e-3, 0.1e-3])
    ap.add_argument("--ns", type=float, default=60.0)
    ap.add_argument("--mesh", nargs="+", choices=MESH_KINDS, default=["hex"])
    ap.add_argument("--periods", type=int, default=1,
                    help="periods between the plates: the band at periods + 1 phase advances")
    args = ap.parse_args()
    import paper_1701_03784_amd as axp
    axp.load_library()
    r0, amp, d = args.r0, args.amp, args.period
    f0u = C_LIGHT / (2 * np.pi) * X01 / r0
    fpu = C_LIGHT / (2 * np.pi) * np.hypot(X01 / r0, np.pi / d)
    f_lo, f_hi = 0.5 * f0u, 1.3 * fpu
    factory = lambda m: axp.make_ctx(m)
    N = args.periods
    phases = np.pi * np.arange(N + 1) / N
    print(json.dumps({"uniform_guide_band_edges_GHz": [f0u / 1e9, fpu / 1e9], "r0": r0, "amp": amp, "period": d,
                      "periods": N, "phase_over_pi": list(phases / np.pi),
                      "uniform_guide_GHz": list(uniform_dispersion(r0, d, phases) / 1e9)}), flush=True)
    for kind in args.mesh:
        for h in args.h:
            t0 = time.perf_counter()
            m = cell_mesh(r0, amp, d, h, kind=kind, periods=N)
            peaks, faces, steps = cell_modes(factory, m, r0, d, args.ns, f_lo, f_hi, count=N + 1)
            line = {"mesh": kind, "h_mm": h * 1e3, "faces": faces, "steps": steps,
                    "f0_GHz": peaks[0] / 1e9 if len(peaks) > 0 else None,
                    "fpi_GHz": peaks[N] / 1e9 if len(peaks) > N else None,
                    "modes_GHz": [p / 1e9 for p in peaks],
                    "seconds": time.perf_counter() - t0}
            print(json.dumps(line), flush=True)
            log(json.dumps(line))


if __name__ == "__main__":
    main()
