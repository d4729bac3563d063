"""Throughput benchmark of the axisymmetric EM-PIC step on one MI355X.

Workload (default): rippled-wall BWO slow-wave tube, ~208k faces, 8M
macro-electrons of a 500 keV annular beam, B_z = 1 T, mixed precision,
dt = 0.5 x the leapfrog stability limit.  Inputs are seeded and synthetic.

Prints one JSON line: particle-steps/s of the whole step (value), the field
kernels' HBM rate, the dominant kernel's roofline (HIP-event time of the
particle kernel on the library's stream) and the FP64 CPU oracle timed on a
bounded slice of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SRC = os.path.join(ROOT, "paper_1701_03784_amd", "csrc", "kernels_mixed.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_particles_bwo_traffic.txt")


def particle_bytes(n_live, n_faces):
    """Algorithmic bytes of one k_particles launch (gather, push, walk and
    current): 24 B of particle state read and written per particle (48 B),
    plus once per face the gather tile (32 B), the geometry used by the push
    (rho of the nodes and the scaled barycentric gradients, 32 B) and the
    three fixed-point side currents (24 B)."""
    return 48.0 * n_live + 88.0 * n_faces


def kernel_source_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_particles launch from the committed counter summary, if it
    was taken on the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def field_bytes(n_edges, n_faces, spai_nnz_padded):
    """Bytes the three field kernels must move once per step:
    face pass 144 B/face + 4 B/edge; edge pass 44 B/edge + 32 B/face;
    SpMV 8 B per stored matrix entry + 8 B/edge."""
    return (144.0 * n_faces + 4.0 * n_edges) + (44.0 * n_edges + 32.0 * n_faces) + \
        (8.0 * spai_nnz_padded + 8.0 * n_edges)


def setup_bwo(n_particles, seed=3, sort_period=4, precision=None, use_graph=1, pusher=0, diag_every=0):
    import synth
    from synth import configs
    import paper_1701_03784_amd as axp
    t0 = time.perf_counter()
    m = configs.bwo_mesh(seed=seed)
    L = m.meta["length"]
    log(f"mesh: {m.n_nodes} nodes, {m.n_tris} faces ({time.perf_counter() - t0:.1f} s)")
    kw = {} if precision is None else {"precision": precision}
    c = axp.make_ctx(m, sort_period=sort_period, use_graph=use_graph, pusher=pusher, diag_every=diag_every, **kw)
    info = c.info()
    log(f"built: {info['n_edges']} edges, SPAI nnz {info['spai_nnz']}, dt {info['dt']:.3e} s "
        f"(limit {info['dt_cfl']:.3e}), setup {info['setup_seconds']:.1f} s")
    c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
    c.set_external_bz(configs.BWO_BZ)
    w = configs.bwo_weight(n_particles, L)
    sp = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, w)
    zr, u = configs.bwo_beam(n_particles, L, seed=seed)
    t1 = time.perf_counter()
    c.inject(sp, zr, u)
    log(f"injected {n_particles} particles (weight {w}) in {time.perf_counter() - t1:.1f} s")
    desc = (f"bwo: rippled-wall tube R=1.5+0.25 sin cm, 10 periods of 1.67 cm + drifts, {m.n_tris} faces, "
            f"{info['n_edges']} edges; {n_particles} macro-electrons, 500 keV annular beam, B_z=1 T; "
            f"SPAI level 3 ({info['spai_nnz']} nnz); dt=0.5 CFL")
    return c, m, info, desc


def plain_leg(n_particles, steps, warmup, use_graph):
    """The same workload on the FP64 GPU step: the same kernel structure in
    FP64, one instance, sort period autotuned the same way; launched eagerly
    (the reference point of the speedups) or replayed from graphs."""
    import paper_1701_03784_amd as axp
    c, m, info, _ = setup_bwo(n_particles, precision=axp.PREC_PLAIN_FP64, use_graph=use_graph)
    sp = c.autotune(16)
    log(f"fp64 step: autotuned sort period {sp}")
    c.step(warmup)
    c.sync()
    steps = max(2 * sp, steps // (2 * sp) * (2 * sp))
    t0 = time.perf_counter()
    c.step(steps)
    c.sync()
    el = time.perf_counter() - t0
    d = c.diag()
    c.close()
    return {"value": d["n_live"] * steps / el, "unit": "particle-steps/s", "ms_per_step": el * 1e3 / steps,
            "steps": steps, "precision": "plain fp64", "particles": int(d["n_live"]), "sort_period": sp,
            "graphs": bool(use_graph)}


def vay_leg(n_particles, steps, warmup):
    """The headline workload with Vay's pusher in place of the Boris push
    (mixed precision, graphs, sort period autotuned)."""
    import paper_1701_03784_amd as axp
    c, m, info, _ = setup_bwo(n_particles, pusher=axp.PUSH_VAY)
    sp = c.autotune(16)
    c.step(warmup)
    c.sync()
    steps = max(2 * sp, steps // (2 * sp) * (2 * sp))
    t0 = time.perf_counter()
    c.step(steps)
    c.sync()
    el = time.perf_counter() - t0
    d = c.diag()
    c.close()
    return {"value": d["n_live"] * steps / el, "unit": "particle-steps/s", "ms_per_step": el * 1e3 / steps,
            "steps": steps, "precision": "mixed", "pusher": "vay", "particles": int(d["n_live"]), "sort_period": sp,
            "graphs": True}


def batched_leg(n_variants, steps, per_face=25, seed_note=""):
    """Batched sweep: members 0..n-1 of the seeded BWO variant family (ripple
    amplitude, period, taper, beam voltage; 20k-300k faces), ~25 particles
    per face each, pooled into one batch, sort schedule autotuned, steps
    replayed from graphs."""
    import synth
    from synth import configs
    import paper_1701_03784_amd as axp
    t0 = time.perf_counter()
    ctxs = []
    n_faces = n_part = 0
    for i in range(n_variants):
        m, p = configs.variant_mesh(i)
        c = axp.make_ctx(m, sort_period=4)
        info = c.info()
        c.set_fields(np.zeros(info["n_edges"]), np.zeros(info["n_faces"]))
        c.set_external_bz(configs.BWO_BZ)
        L = m.meta["length"]
        n = per_face * m.n_tris
        sp = c.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, configs.bwo_weight(n, L, kev=p["kev"]))
        r_out = min(0.011, 0.015 - p["amp"] - 0.001)       # keep the beam 1 mm inside the ripple minimum
        zr, u = configs.bwo_beam(n, L, kev=p["kev"], seed=p["seed"], r_in=r_out - 0.002, r_out=r_out)
        c.inject(sp, zr, u)
        n_faces += m.n_tris
        n_part += n
        ctxs.append(c)
        log(f"batch member {i}: {m.n_tris} faces, {n} particles, {p['kev']:.0f} keV")
    b = axp.Batch(ctxs)
    log(f"batch of {n_variants}: {n_faces} faces, {n_part} particles, setup {time.perf_counter() - t0:.1f} s")
    sp_best = b.autotune(trial_steps=16)
    log(f"autotuned sort period {sp_best}")
    b.step(2 * sp_best)
    b.sync()
    steps = max(2 * sp_best, steps // (2 * sp_best) * (2 * sp_best))
    t1 = time.perf_counter()
    b.step(steps)
    b.sync()
    el = time.perf_counter() - t1
    live = sum(c.info()["n_particles"] for c in ctxs)
    n_edges = b.info()["n_edges"]
    b.close()
    for c in ctxs:
        c.close()
    return {"value": live * steps / el, "unit": "particle-steps/s", "ms_per_step": el * 1e3 / steps,
            "steps": steps, "variants": n_variants, "faces": n_faces, "particles": int(live),
            "sort_period": sp_best, "graphs": True,
            "field_dof_steps_per_s": (n_faces + n_edges) * steps / el}


def cpu_baseline(target_seconds=15.0):
    """FP64 oracle on a bounded slice of the BWO workload: one ripple period
    of the same profile and mesh size, the same beam density."""
    from synth import configs
    import synth
    from oracle.pic import OracleSim
    m = configs.bwo_mesh(seed=3, n_periods=1, up=0.0, down=0.0)
    full_area = 0.217 * 0.015
    area = m.signed_areas().sum()
    n = int(8_000_000 * area / full_area)
    t0 = time.perf_counter()
    sim = OracleSim(m.nodes, m.tris, m.seg, m.tag)
    setup = time.perf_counter() - t0
    sim.bz = configs.BWO_BZ
    L = m.meta["length"]
    zr, u = configs.bwo_beam(n, L, seed=3)
    sp = sim.add_species(synth.ELECTRON_CHARGE, synth.ELECTRON_MASS, configs.bwo_weight(n, L))
    sim.inject(sp, zr, u)
    sim.step(1)
    steps, el = 0, 0.0
    while el < target_seconds and steps < 400:
        t1 = time.perf_counter()
        sim.step(1)
        el += time.perf_counter() - t1
        steps += 1
    live = int(sim.palive.sum())
    rate = live * steps / el
    return {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one ripple period of the bwo profile (1.67 cm, {m.n_tris} faces, h=0.19 mm) with "
                      f"{live} particles at the full beam density, {steps} steps timed "
                      f"({el:.1f} s) after {setup:.1f} s of oracle setup; single thread FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=8_000_000)
    ap.add_argument("--sort-period", type=int, default=0, help="0: chosen by the library's autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-steps", type=int, default=20, help="timed steps of the FP64 leg (0: skip)")
    ap.add_argument("--vay-steps", type=int, default=32, help="timed steps of the Vay-pusher leg (0: skip)")
    ap.add_argument("--batch-variants", type=int, default=8, help="members of the batched sweep (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=48)
    ap.add_argument("--diag-every", type=int, default=0,
                    help="diagnostic steps (nodal charge, Gauss and continuity residuals, energies) every this many steps")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the workload is measured at N=1; the multi-GPU path "
              "(z-slab decomposition, independent batch members per GPU) is a design, not implemented",
              file=sys.stderr)
        sys.exit(2)

    import paper_1701_03784_amd as axp
    axp.load_library()
    c, m, info, desc = setup_bwo(args.particles, sort_period=max(1, args.sort_period), diag_every=args.diag_every)
    sort_period = args.sort_period
    if sort_period == 0:
        sort_period = c.autotune(16)
        log(f"autotuned sort period {sort_period} (steps so far {c.info()['step']})")
    c.step(args.warmup)
    c.sync()
    log(f"warmup {args.warmup} steps done")
    # timed region: the production mode, steps replayed from graphs
    t0 = time.perf_counter()
    c.step(args.steps)
    c.sync()
    el = time.perf_counter() - t0
    d_timed = c.diag()
    # kernel durations: the next args.steps steps with HIP events around every
    # phase (eager launches: HIP cannot time event records inside a graph)
    c.set_timing(True)
    c.sync()
    t1 = time.perf_counter()
    c.step(args.steps)
    c.sync()
    el_events = time.perf_counter() - t1
    tim = c.get_timing()
    d = c.diag()
    n_live = d_timed["n_live"]
    n1, n2 = info["n_edges"], info["n_faces"]
    ms_step = el * 1e3 / args.steps
    value = n_live * args.steps / el
    part_ms, part_n = tim["particles"]
    part_avg_s = part_ms / part_n / 1e3
    pb = particle_bytes(n_live, n2)
    achieved = pb / part_avg_s / 1e9
    nnz_pad = info["spai_nnz"] * 1.15
    fb = field_bytes(n1, n2, nnz_pad)
    field_ms = sum(tim[k][0] for k in ("face", "edge", "spmv")) / args.steps
    walk_ms, walk_n = tim["walk"]
    field_gbs = fb / (field_ms / 1e3) / 1e9
    per_phase = {k: round(v[0] / max(1, v[1]) * 1e3, 2) for k, v in tim.items() if v[1]}
    log(f"{args.steps} steps in {el:.3f} s: {ms_step:.3f} ms/step; per-launch us {per_phase}")
    log(f"diag: live {n_live} absorbed {d['n_absorbed']} overflow {d['walk_overflow']} nan {d['nan_count']}")

    if args.copy_probe_mib:
        import torch
        a = torch.empty(args.copy_probe_mib * 2 ** 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB x3")

    c.close()
    plain = plain_graph = batched = None
    if args.plain_steps > 0:
        log("plain FP64 leg (eager) ...")
        plain = plain_leg(args.particles, args.plain_steps, 4, use_graph=0)
        log(f"plain: {plain['value']:.3e} particle-steps/s ({plain['ms_per_step']:.3f} ms/step)")
        log("plain FP64 leg (graphs) ...")
        plain_graph = plain_leg(args.particles, args.plain_steps, 4, use_graph=1)
        log(f"plain, graphs: {plain_graph['value']:.3e} particle-steps/s ({plain_graph['ms_per_step']:.3f} ms/step)")
    vay = None
    if args.vay_steps > 0:
        log("Vay pusher leg ...")
        vay = vay_leg(args.particles, args.vay_steps, 4)
        log(f"vay: {vay['value']:.3e} particle-steps/s ({vay['ms_per_step']:.3f} ms/step)")
    if args.batch_variants > 0:
        log("batched leg ...")
        batched = batched_leg(args.batch_variants, args.batch_steps)
        log(f"batched: {batched['value']:.3e} particle-steps/s ({batched['ms_per_step']:.3f} ms/step)")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.3e} particle-steps/s")

    out = {
        "metric": "particle-steps/s + field HBM GB/s at 1 GPU; batched-mixed vs plain at fixed error",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i64",
        "data": "synthetic (seeded mesh, beam and fields)",
        "config": {"workload": desc, "faces": n2, "edges": n1, "particles": int(n_live),
                   "precision": "mixed", "sort_period": sort_period},
        "field_dof_steps_per_s": (n1 + n2) * args.steps / el,
        "timing": "value and ms_per_step: wall clock of the timed steps, replayed from HIP graphs; kernel durations "
                  "(phase_us_*, roofline): HIP events around every phase over the same number of steps right after, "
                  f"launched eagerly ({el_events * 1e3 / args.steps:.4f} ms/step with the events)",
        "field_hbm_gbs": field_gbs,
        "phase_us_per_launch": per_phase,
        "phase_us_per_step": {k: round(v[0] / args.steps * 1e3, 2) for k, v in tim.items() if v[1]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_particles", "bytes_per_launch": pb,
                     "avg_launch_us": part_avg_s * 1e6,
                     "kernel_source_sha256_16": kernel_source_hash()},
        "cpu_baseline": cpu,
        "plain_fp64": plain,
        "plain_fp64_graphs": plain_graph,
        "pusher_vay": vay,
        "batched_mixed": batched,
        "speedup_mixed_vs_plain": (value / plain["value"]) if plain else None,
        "speedup_batched_mixed_vs_plain": (batched["value"] / plain["value"]) if (plain and batched) else None,
        "speedup_mixed_vs_plain_graphs": (value / plain_graph["value"]) if plain_graph else None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
