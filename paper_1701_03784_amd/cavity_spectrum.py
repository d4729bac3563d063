"""The cavity validation of Sec. 4.1 run on the GPU.

    python -m paper_1701_03784_amd.cavity_spectrum [--steps 2000000] [--dt 1e-12] [--h 0.00854]
                                                   [--precision mixed|plain] [--out spectrum.json]

A PEC cylinder of radius a = 0.5 m and height h = 1 m (the meridian plane
meshed with about 15,800 faces at the default spacing), excited by the two
magnetic point sources of Sec. 4.1 (Gaussian-modulated pulses centred at
20 and 40 ns, sigma = 1 ns, carrier 0.5 GHz), with the field probe at
(z = 0.71 m, rho = 0.39 m) (the printed probe position lies outside the
cavity; its two coordinates are read swapped).  The probe signal of the
whole run goes through a Hann window and a zero-padded FFT; each TM0np
mode below 0.95 GHz is located as the spectral peak nearest its analytic
frequency c/(2 pi) sqrt((x_0n / a)^2 + (p pi / h)^2), refined by a
parabola through the logarithm of the three highest bins.  Prints one JSON
line per mode and a summary line.
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

C_LIGHT = 299792458.0
A_CAV, H_CAV = 0.5, 1.0
TG, SIG, WG = 40e-9, 1e-9, np.pi * 1e9
SOURCES = [(0.2, 0.37, 0.7, TG / 2), (0.7, 0.08, 0.5, TG)]      # (z, rho, amplitude, pulse centre)
PROBE = (0.71, 0.39)


def log(msg):
    print(f"[cavity] {msg}", file=sys.stderr, flush=True)


def analytic_modes(f_max=0.95e9):
    import scipy.special
    x = scipy.special.jn_zeros(0, 4)
    out = []
    for n in range(1, 5):
        for p in range(0, 12):
            f = C_LIGHT / (2 * np.pi) * np.hypot(x[n - 1] / A_CAV, p * np.pi / H_CAV)
            if f < f_max:
                out.append((f, n, p))
    return sorted(out)


def spectrum_peaks(signal, dt, modes, pad=4):
    """Peak frequency nearest each analytic mode frequency (within 0.5 %)."""
    w = np.hanning(len(signal))
    nfft = pad * len(signal)
    f = np.fft.rfftfreq(nfft, dt)
    P = sum(np.abs(np.fft.rfft(w * signal[:, k], nfft)) ** 2 for k in range(signal.shape[1]))
    peaks = np.flatnonzero((P[1:-1] > P[:-2]) & (P[1:-1] > P[2:])) + 1
    res = []
    for fa, n, p in modes:
        near = peaks[np.abs(f[peaks] / fa - 1.0) < 0.005]
        if len(near) == 0:
            res.append((fa, n, p, None, None))
            continue
        i = near[np.argmax(P[near])]
        y0, y1, y2 = np.log(P[i - 1]), np.log(P[i]), np.log(P[i + 1])
        d = 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)         # parabola vertex, in bins
        fs = f[i] + d * (f[1] - f[0])
        res.append((fa, n, p, fs, float(P[i] / P.max())))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2_000_000)
    ap.add_argument("--dt", type=float, default=1e-12)
    ap.add_argument("--h", type=float, default=0.00854)
    ap.add_argument("--precision", choices=["mixed", "plain"], default="mixed")
    ap.add_argument("--chunk", type=int, default=100_000)
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    import synth
    import paper_1701_03784_amd as axp
    axp.load_library()
    t0 = time.perf_counter()
    m = synth.rect_mesh(0.0, H_CAV, A_CAV, args.h, seed=0)
    prec = axp.PREC_PLAIN_FP64 if args.precision == "plain" else axp.PREC_MIXED
    c = axp.make_ctx(m, dt=args.dt, precision=prec)
    info = c.info()
    log(f"{info['n_nodes']} nodes, {info['n_edges']} edges, {info['n_faces']} faces; dt {info['dt']:.3e} s "
        f"(limit {info['dt_cfl']:.3e}); setup {time.perf_counter() - t0:.1f} s")
    c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
    for z, rho, a, tc in SOURCES:
        c.add_point_source(z, rho, a, tc, SIG, WG)
    c.set_probe(*PROBE, args.steps)
    t1 = time.perf_counter()
    done = 0
    while done < args.steps:
        k = min(args.chunk, args.steps - done)
        c.step(k)
        done += k
        c.sync()
        log(f"step {done} ({time.perf_counter() - t1:.1f} s)")
    run_s = time.perf_counter() - t1
    sig = c.get_probe()
    c.close()
    res = spectrum_peaks(sig, args.dt, analytic_modes())
    errs = []
    for fa, n, p, fs, rel in res:
        line = {"mode": [0, n, p], "f_a_GHz": fa / 1e9, "f_s_GHz": None if fs is None else fs / 1e9,
                "err_percent": None if fs is None else abs(fs - fa) / fa * 100, "peak_rel_power": rel}
        if fs is not None:
            errs.append(line["err_percent"])
        print(json.dumps(line), flush=True)
    summary = {"faces": info["n_faces"], "edges": info["n_edges"], "steps": args.steps, "dt": args.dt,
               "precision": args.precision, "run_seconds": run_s, "us_per_step": run_s / args.steps * 1e6,
               "record_s": args.steps * args.dt, "modes_found": len(errs), "modes": len(res),
               "max_err_percent": max(errs) if errs else None, "mean_err_percent": float(np.mean(errs)) if errs else None}
    print(json.dumps(summary), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": summary, "modes": [list(r) for r in res]}, f)


if __name__ == "__main__":
    main()
