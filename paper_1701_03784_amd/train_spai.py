"""Train and evaluate the learned-SPAI network.

    python -m paper_1701_03784_amd.train_spai --meshes 48 --out spai_mlp_l3.bin [--bwo-steps 20000]
    python -m paper_1701_03784_amd.train_spai --load spai_mlp_l3.bin --eval-meshes 64 [--faces-max 200000]

Training meshes are seeded rippled-wall tubes (random ripple amplitude,
period, taper and mesh size); every mesh's plain SPAI is computed by the
library and its pattern pairs become training samples (a random subset per
mesh).  The network is trained on the GPU by the library's kernels.  The
evaluation reports, on meshes not seen in training, the mean column residual
||e_k - A^ m_k|| of the network's columns and after the CGNR refinement, next
to the Jacobi starting guess refined the same way and to the plain SPAI; the
setup time of both constructions; and, on the rippled-wall BWO workload, a
run with the learned matrix next to one with the plain matrix (energy,
Gauss-law drift, continuity, field difference).
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(f"[train_spai] {msg}", file=sys.stderr, flush=True)


def random_tube(seed, faces_min, faces_max):
    from synth import configs
    rng = np.random.default_rng(seed)
    amp = float(rng.uniform(0.001, 0.004))
    period = float(rng.uniform(0.012, 0.020))
    taper = float(rng.uniform(0.0, 0.3))
    n_periods = int(rng.integers(2, 5))
    faces = float(rng.uniform(faces_min, faces_max))
    length = 0.008 + n_periods * period
    h = np.sqrt(4 * length * 0.015 / np.sqrt(3) / faces)
    return configs.bwo_mesh(seed=seed, h=h, amp=amp, period=period, n_periods=n_periods, taper=taper,
                            up=0.004, down=0.004)


def identity_network():
    """A network whose output is 1 on the diagonal pair (feature 0, d = 0) and
    0 elsewhere: the Jacobi starting guess, through the same construction."""
    from . import Mlp
    net = Mlp(n_hidden=32, n_layers=1, seed=0)
    p = np.zeros(net.n_params(), dtype=np.float32)
    a = 4.0
    p[0] = a                                   # hidden unit 0 = tanh(a * x0)
    off = 32 * 16 + 32                         # output layer weights
    p[off] = np.float32(1.0 / np.tanh(np.float32(a)))
    net.set_params(p)
    return net


def residual_study(net, ident, mesh, iters=3, row_tol=0.02):
    """Column residuals and setup times of the plain SPAI, the network's
    construction and the same construction from the Jacobi guess."""
    from . import make_ctx
    res = {"faces": mesh.n_tris}
    cp = make_ctx(mesh)
    ip = cp.info()
    res.update(plain_seconds=ip["spai_seconds"], plain_fro=ip["spai_fro_residual"], n_free=ip["n_free_edges"])
    cp.close()
    for name, model in (("learned", net), ("jacobi", ident)):
        c = make_ctx(mesh, spai_model=model, spai_row_tol=row_tol, spai_iters=iters)
        i = c.info()
        res[name] = {"seconds": i["spai_seconds"], "start_resid": i["spai_pred_resid_mean"],
                     "refined_resid_kept": i["spai_kept_resid_mean"], "fallback_columns": i["spai_fallback_columns"],
                     "fro": i["spai_fro_residual"], "energy_guard_drift": i["spai_energy_drift"],
                     "mode": i["spai_mode"]}
        c.close()
    return res


def bwo_runs(net, steps, particles, log_every):
    """The rippled-wall BWO workload with the learned and the plain SPAI."""
    import synth
    from synth import configs
    from . import make_ctx
    m = configs.bwo_mesh(seed=3)
    L = m.meta["length"]
    zr, u = configs.bwo_beam(particles, L, seed=3)
    out = {}
    fields = {}
    for name, model in (("learned", net), ("plain", None)):
        t0 = time.perf_counter()
        c = make_ctx(m, spai_model=model, spai_row_tol=0.02, spai_iters=3)
        info = c.info()
        c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
        c.set_external_bz(configs.BWO_BZ)
        sp = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, configs.bwo_weight(particles, L))
        c.inject(sp, zr, u)
        d0 = c.diag()
        e0 = d0["W_E"] + d0["W_B"] + d0["W_K"]
        worst_dce, worst_gauss = 0, 0.0
        t1 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(log_every, steps - done)
            c.step(k)
            done += k
            d = c.diag()
            worst_dce = max(worst_dce, d["dce_max_abs"])
            worst_gauss = max(worst_gauss, d["gauss_max_drift"] / max(d["gauss_scale"], 1e-300))
            log(f"{name}: step {done} live {d['n_live']} W {d['W_E'] + d['W_B'] + d['W_K']:.4e} "
                f"gauss drift/scale {worst_gauss:.2e} dce {worst_dce}")
        el = time.perf_counter() - t1
        E, B = c.get_fields()
        fields[name] = E
        out[name] = {"spai_mode": info["spai_mode"], "spai_seconds": info["spai_seconds"],
                     "setup_seconds": info["setup_seconds"], "fallback_columns": info["spai_fallback_columns"],
                     "energy_guard_drift": info["spai_energy_drift"], "dt_cfl": info["dt_cfl"],
                     "steps": steps, "run_seconds": el, "W_start": e0,
                     "W_end": d["W_E"] + d["W_B"] + d["W_K"], "max_gauss_drift_rel": worst_gauss,
                     "max_dce_abs": int(worst_dce), "n_live": d["n_live"], "n_absorbed": d["n_absorbed"],
                     "wall_seconds": time.perf_counter() - t0}
        c.close()
    out["E_rel_l2_learned_vs_plain"] = float(np.linalg.norm(fields["learned"] - fields["plain"]) /
                                             max(np.linalg.norm(fields["plain"]), 1e-300))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", type=int, default=48)
    ap.add_argument("--faces-min", type=float, default=10000)
    ap.add_argument("--faces-max", type=float, default=60000)
    ap.add_argument("--pairs-per-mesh", type=int, default=150000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--eval-meshes", type=int, default=8)
    ap.add_argument("--bwo-steps", type=int, default=0)
    ap.add_argument("--bwo-particles", type=int, default=8_000_000)
    ap.add_argument("--out", default="")
    ap.add_argument("--load", default="", help="evaluate a saved network instead of training one")
    args = ap.parse_args()

    import torch  # noqa: F401  (device buffers)
    from . import Mlp, load_library
    from .learned_spai import training_pairs, train
    load_library()
    if args.load:
        net = Mlp.load(args.load)
        training = {"loaded": args.load}
        log(f"network loaded from {args.load}")
    else:
        t0 = time.perf_counter()
        meshes = (random_tube(1000 + i, args.faces_min, args.faces_max) for i in range(args.meshes))
        X, y = training_pairs(meshes, max_pairs_per_mesh=args.pairs_per_mesh, seed=0, log=log)
        t_data = time.perf_counter() - t0
        n_pairs = int(len(y))
        log(f"{n_pairs} training pairs from {args.meshes} meshes in {t_data:.1f} s")
        net = Mlp(n_hidden=64, n_layers=2, seed=0)
        t1 = time.perf_counter()
        hist = train(net, X, y, epochs=args.epochs, batch=4096, lr=3e-3, lr_final=1e-4,
                     log=lambda s: log(s) if s.endswith("9") or s.startswith("epoch 0") else None)
        t_train = time.perf_counter() - t1
        log(f"trained in {t_train:.1f} s: loss {hist[0]:.3e} -> {hist[-1]:.3e}")
        if args.out:
            net.save(args.out)
        del X, y
        training = {"meshes": args.meshes, "faces": [args.faces_min, args.faces_max], "pairs": n_pairs,
                    "data_seconds": t_data, "train_seconds": t_train, "loss_first_epoch": hist[0],
                    "loss_last_epoch": hist[-1], "epochs": args.epochs}
    evals = []
    ident = identity_network()
    for i in range(args.eval_meshes):
        res = residual_study(net, ident, random_tube(2000 + i, args.faces_min, args.faces_max))
        log(f"unseen mesh {i}: {json.dumps(res)}")
        evals.append(res)
    summary = {"training": training, "unseen": evals}
    if args.bwo_steps:
        summary["bwo"] = bwo_runs(net, args.bwo_steps, args.bwo_particles, max(100, args.bwo_steps // 10))
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
