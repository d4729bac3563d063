"""Hot test of the backward-wave oscillator (Sec. 5.1, synthetic geometry).

    python -m paper_1701_03784_amd.bwo_hot_test [--ns 40] [--h 0.19e-3] [--per-step 300]

The tube of the benchmark workload: a smooth-walled upstream drift of 2 cm,
ten periods of the rippled wall R = 1.5 + 0.25 sin(2 pi z / d) cm (d =
1.67 cm, raised-cosine ramps over half a period at both ends), and a 3 cm
downstream drift whose last 2 cm are an absorbing layer.  The upstream end
is a conductor plate whose annulus 9 mm <= rho <= 11 mm emits a 500 keV
electron beam of 1.5 kA every step; a 1 T axial field guides it.  The
backward wave the beam drives travels toward the cathode, reflects there,
and leaves through the layer.  A probe between beam and wall records E; the
spectrum of the last part of the record gives the oscillation frequency.

The frequency is set by the synchronism of the beam with the backward
(-1) spatial harmonic of the TM01 band: f = v phi / (2 pi d) for phase
advance phi per period in (pi, 2 pi), where the band runs back down, f(phi)
= f_band(2 pi - phi).  The band comes from the cold test (cold_test.py),
so the two runs check each other.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

QE, ME, C = 1.602176634e-19, 9.1093837015e-31, 299792458.0


def log(msg):
    print(f"[hot] {msg}", file=sys.stderr, flush=True)


def tube_mesh(h, r_in=0.009, r_out=0.011, seed=3):
    """The benchmark tube with an emitting annulus on the upstream plate."""
    import synth
    from synth import configs
    R, z1 = configs.bwo_radius_fn()
    L = z1 + 0.03

    def tag(side, z, rho):
        if side == "bottom":
            return synth.BC_AXIS
        if side == "left" and r_in <= rho <= r_out:
            return synth.BC_EMITTER
        return synth.BC_PEC

    return synth.rippled_mesh(R, 0.0, L, h, seed=seed, tags=tag, meta=dict(length=L, z_ripple_end=z1)), L


def synchronism(f_band, period, v):
    """Frequency where the beam line f = v phi / (2 pi d) meets the TM01
    band's backward branch f_band(2 pi - phi), phi in (pi, 2 pi); f_band is
    sampled at phase advances 0 .. pi (uniform) and interpolated linearly."""
    fb = np.asarray(f_band, dtype=np.float64)
    ph = np.linspace(0.0, np.pi, len(fb))
    phi = np.linspace(np.pi, 2 * np.pi, 4001)
    beam = v * phi / (2 * np.pi * period)
    band = np.interp(2 * np.pi - phi, ph, fb)
    i = int(np.argmax(beam >= band))
    if beam[i] < band[i]:
        return None
    t = (band[i - 1] - beam[i - 1]) / ((beam[i] - beam[i - 1]) - (band[i] - band[i - 1]))
    return float(beam[i - 1] + t * (beam[i] - beam[i - 1]))


def main():
    import synth
    from synth import configs
    from . import make_ctx
    ap = argparse.ArgumentParser()
    ap.add_argument("--ns", type=float, default=40.0)
    ap.add_argument("--h", type=float, default=0.19e-3)
    ap.add_argument("--per-step", type=int, default=300)
    ap.add_argument("--current", type=float, default=1500.0)
    ap.add_argument("--kev", type=float, default=500.0)
    ap.add_argument("--bz", type=float, default=configs.BWO_BZ)
    ap.add_argument("--probe", type=float, nargs=2, default=[0.10, 0.012])
    ap.add_argument("--period", type=float, default=0.0167, help="wall period of the tube (as built by synth)")
    ap.add_argument("--band-ghz", type=float, nargs="+", default=[7.5669, 7.8231, 8.5144, 9.4045, 9.9161],
                    help="TM01 band of the cell at phase advances 0 .. pi (cold test, four periods)")
    args = ap.parse_args()
    t0 = time.perf_counter()
    m, L = tube_mesh(args.h)
    c = make_ctx(m, sort_period=8, layers=dict(z_right=L - 0.02, sigma_max=3.66, order=3))
    info = c.info()
    dt = info["dt"]
    c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
    c.set_external_bz(args.bz)
    g, b = synth.gamma_beta_from_kev(args.kev)
    w = max(1, int(round(args.current * dt / (args.per_step * QE))))
    sp = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, w)
    c.set_injector(sp, args.per_step, [0.0, 0.0, g * b * C], 0.0, 5)
    steps = int(args.ns * 1e-9 / dt)
    c.set_probe(args.probe[0], args.probe[1], steps)
    f_sync = synchronism(np.array(args.band_ghz) * 1e9, args.period, b * C)
    head = {"faces": info["n_faces"], "edges": info["n_edges"], "layer_faces": info["n_layer_faces"], "dt": dt,
            "steps": steps, "weight": w, "per_step": args.per_step, "current_A": w * args.per_step * QE / dt,
            "beam_beta": b, "synchronism_GHz_cold_band": None if f_sync is None else f_sync / 1e9,
            "setup_s": time.perf_counter() - t0}
    print(json.dumps(head), flush=True)
    c.diag()
    worst_dce, chunk, done = 0, 20000, 0
    t1 = time.perf_counter()
    while done < steps:
        n = min(chunk, steps - done)
        c.step(n)
        done += n
        d = c.diag()
        worst_dce = max(worst_dce, d["dce_max_abs"])
        log(f"{done}/{steps} steps ({done * dt * 1e9:.2f} ns): live {d['n_live']}, absorbed {d['n_absorbed']}, "
            f"dce {d['dce_max_abs']}, W_E {d['W_E']:.3e} J/rad, {time.perf_counter() - t1:.0f} s")
    sig = c.get_probe()
    run_s = time.perf_counter() - t1
    d = c.diag()
    c.close()
    # envelope of |E| at the probe in 1 ns windows, and the spectrum of the last 40 % of the record
    win = max(1, int(1e-9 / dt))
    amp = np.sqrt((sig ** 2).sum(axis=1))
    env = [float(amp[i:i + win].max()) for i in range(0, len(amp) - win + 1, win)]
    tail = sig[int(0.6 * len(sig)):]
    nfft = 8 * len(tail)
    f = np.fft.rfftfreq(nfft, dt)
    P = sum(np.abs(np.fft.rfft(np.hanning(len(tail)) * tail[:, k], nfft)) ** 2 for k in range(2))
    band = (f > 2e9) & (f < 20e9)
    idx = np.flatnonzero(band)
    W = 6 * 8                                    # +-6 bins of the unpadded transform
    local = [i for i in idx if P[i] == P[max(0, i - W):i + W + 1].max()]
    lines = []
    for i in sorted(local, key=lambda i: -P[i])[:3]:
        y0, y1, y2 = np.log(P[i - 1]), np.log(P[i]), np.log(P[i + 1])
        fi = float(f[i] + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2) * (f[1] - f[0]))
        lines.append((fi, float(P[band][np.abs(f[band] - fi) < 0.2e9].sum() / P[band].sum())))
    f_peak, frac = lines[0]
    out = {"ns": steps * dt * 1e9, "run_s": run_s, "ms_per_step": run_s * 1e3 / steps, "live": d["n_live"],
           "absorbed": d["n_absorbed"], "dce_max_abs_worst": worst_dce, "walk_overflow": d["walk_overflow"],
           "nan_count": d["nan_count"], "f_peak_GHz": f_peak / 1e9, "power_within_200MHz": frac,
           "lines_GHz_and_power_fraction": [(fi / 1e9, fr) for fi, fr in lines],
           "envelope_V_per_m_per_ns": env}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
