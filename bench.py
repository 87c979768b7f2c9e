"""Throughput of the level-set grain-growth step on one MI355X.

Prints ONE JSON line: grain-voxel updates per second of the batched mixed
(FP32) step on the 3D 256^3 / 8000-grain lognormal workload, the plain FP64
path on the same inputs, the roofline of the dominant kernel (HIP events on
the library's stream, algorithmic bytes), and the FP64 CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
SOURCES = [os.path.join(ROOT, "paper_1701_06658_amd", "csrc", f) for f in ("gg_kernels.hpp", "gg_lib.hip")]
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes per grain voxel of one launch, by kernel class, in units of
# the stored value size s (plus fixed extra bytes): every stencil kernel reads
# its input box values once and writes its output box values once.
ALG_BYTES = {
    "conv_xy": (2, 0), "conv_z": (2, 0), "compare": (2, 0),
    "reinit_xy": (2, 0), "reinit_z": (2, 0),
}
# with the predictor correction the xy pass (its epilogue) also reads phi and the
# ID-field, the corrector writes the ID-field and the re-initialization carries
# it over
ALG_BYTES_PHYS = {
    "conv_xy": (3, 4), "conv_z": (2, 0), "compare": (2, 4),
    "reinit_xy": (2, 8), "reinit_z": (2, 0),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def euclid_sweeps(dim, W):
    """Jacobi sweep count of the Euclidean re-initialization variant (the
    library's rule): ceil(sqrt(dim) W) + 1, rounded up to an even count."""
    K = int(math.ceil(math.sqrt(dim) * W)) + 1
    return K + (K & 1)


def run_gpu(cfg, precision, steps, warmup, copy_probe=False, redistance="taxicab", autotune=False):
    import paper_1701_06658_amd as gg
    phys = {}
    if cfg.get("physics") == "anisotropic":
        phys = dict(physics=gg.PHYS_MISORIENTATION, quat=cfg["quat"], theta_c_deg=cfg["theta_c_deg"])
    elif cfg.get("physics") == "magnetic":
        phys = dict(physics=gg.PHYS_BULK, energy=cfg["energy"], voxel_m=cfg["h_phys"],
                    gamma_max=cfg["gamma_max"])
    t0 = time.perf_counter()
    sim = gg.Simulation(cfg["labels"], cfg["W"], G=cfg["G"], precision=precision, redistance=redistance, **phys)
    sim.sync()
    log(f"[bench] {precision}: created in {time.perf_counter() - t0:.2f} s")
    tuned = None
    if autotune:
        # the tuner's steps (one per candidate tiling) are warm-up steps
        tuned = sim.autotune(cfg["dt"], 1)
        log(f"[bench] {precision}: autotuned LDS budgets {tuned}")
    if warmup:
        sim.step(cfg["dt"], warmup)
    sim.sync()
    gv0 = sim.stats()["total_grain_voxels"]
    sim.profile(True)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(cfg["dt"], steps)
    sim.sync()
    dt = time.perf_counter() - t0
    st = sim.stats()
    kt = sim.kernel_times()
    sim.profile(False)
    gv = st["total_grain_voxels"] - gv0
    out = dict(value=gv / dt, ms_per_step=1e3 * dt / steps, grain_voxels=gv, alive=st["alive"],
               superposition=st["superposition"], kernels=kt, physics=bool(phys),
               sweeps=euclid_sweeps(cfg["dim"], cfg["W"]) if redistance == "euclid" else 0, tuned=tuned)
    log(f"[bench] {precision}: {steps} steps in {dt:.3f} s, {out['value']:.3e} gv/s, "
        f"alive {st['alive']}")
    if copy_probe:
        # one state download after the timed steps: k_convert reads every stored
        # value once (4 or 8 B) and writes it as a double; its byte counters
        # calibrate the profiler
        _, v = sim.values()
        s = 4 if precision == "fp32" else 8
        out["copy_probe"] = dict(kernel="k_convert", values=int(v.size), read_bytes=int(v.size) * s,
                                 write_bytes=int(v.size) * 8)
    sim.close()
    return out


def run_coarsen(cfg, precision, warmup, n_new):
    """One gg_coarsen of the workload after `warmup` steps: wall time with the
    stream synchronised on both sides, and the grain voxels before and after."""
    import paper_1701_06658_amd as gg
    sim = gg.Simulation(cfg["labels"], cfg["W"], G=cfg["G"], precision=precision)
    sim.step(cfg["dt"], max(warmup, 1))
    sim.sync()
    before = sim.stats()["grain_voxels"]
    nn = (n_new, n_new, n_new) if cfg["dim"] == 3 else (n_new, n_new, 1)
    t0 = time.perf_counter()
    sim.coarsen(nn)
    sim.sync()
    ms = 1e3 * (time.perf_counter() - t0)
    # one step on the new grid: its grain voxels are the coarsened layout's
    sim.step(cfg["sigma"] ** 2 / (2.0 * n_new ** 2), 1)
    after = sim.stats()["grain_voxels"]
    alive = sim.alive_count()
    sim.close()
    log(f"[bench] coarsen {cfg['n'][0]} -> {n_new}: {ms:.2f} ms, {before} -> {after} grain voxels")
    return dict(n_new=n_new, ms=ms, grain_voxels_before=before, grain_voxels_after=after, alive_after=alive,
                gv_per_s=(before + after) / (ms * 1e-3))


def source_digest():
    """SHA-256 of the kernel sources: a recorded counter figure applies only to them."""
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, precision, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>_<workload>_<precision>.md), or None when the
    summary is missing or was taken from other kernel sources."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}_{precision}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256") != source_digest():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(res, s_bytes):
    table = dict(ALG_BYTES_PHYS if res["physics"] else ALG_BYTES)
    if res["sweeps"]:
        # each Jacobi sweep of the Euclidean variant reads and writes every value
        # once; one timed span holds all sweeps of a step
        table["reinit_sweep"] = (2 * res["sweeps"], 0)
    best = None
    per = {}
    for name, (mult, extra) in table.items():
        k = res["kernels"][name]
        if not k["launches"] or k["ms"] <= 0:
            continue
        bytes_alg = (mult * s_bytes + extra) * k["voxels"]
        avg_ms = k["ms"] / k["launches"]
        gbs = bytes_alg / (k["ms"] * 1e-3) / 1e9
        per[name] = dict(avg_ms=avg_ms, gbs=gbs, bytes_per_launch=bytes_alg / k["launches"], launches=k["launches"])
        if best is None or k["ms"] > res["kernels"][best]["ms"]:
            best = name
    r = per[best]
    return dict(bound="hbm", kernel=best, achieved=r["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=r["gbs"] / HBM_PEAK_GBS, traffic=None,
                avg_launch_ms=r["avg_ms"], alg_bytes_per_launch=r["bytes_per_launch"], launches=r["launches"],
                per_kernel={k: round(v["gbs"], 1) for k, v in per.items()})


def cpu_baseline(index, threads=None):
    """FP64 oracle on a bounded sample: one step of a density-matched cut of the
    workload (128^3 on all host threads; 64^3 on one thread)."""
    from oracle import Oracle, num_threads, set_num_threads
    from synth import make_config
    N = None if index == 1 else (64 if threads == 1 else 128)
    G = None if index == 1 else int(round({2: 1000, 3: 1000, 4: 781, 5: 781}[index] * (N / 128) ** 3))
    all_threads = num_threads()
    if threads:
        set_num_threads(threads)
    try:
        c = make_config(index, N=N, G=G)
        o = Oracle(c["labels"], c["W"], G=c["G"])
        gv = 0
        for k in range(c["G"]):
            alive, lo, ext = o.box(k)
            if alive:
                gv += int(ext[0]) * int(ext[1]) * int(ext[2])
        used = num_threads()
        t0 = time.perf_counter()
        o.step(c["dt"])
        dt = time.perf_counter() - t0
        o.close()
    finally:
        set_num_threads(all_threads)
    return dict(value=gv / dt, unit="grain-voxel updates/s", cores=used, kind="oracle",
                sample=f"1 FP64 oracle step of a density-matched {c['N']}^{c['dim']} cut with "
                       f"{c['G']} grains of workload {index} ({gv} grain voxels, {dt:.2f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", default=None, help="fp32 (mixed) or fp64 (plain)")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the tiling's LDS budgets with gg_autotune before the warm-up steps")
    ap.add_argument("--coarsen", type=int, default=0, metavar="N_NEW",
                    help="also time one grid coarsening of the workload onto N_NEW voxels per axis")
    ap.add_argument("--redistance", default="taxicab", choices=["taxicab", "euclid"],
                    help="re-initialization scheme: the method's taxicab one or the Euclidean variant")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run the library's state download once: a plain "
                         "streaming kernel of known size (reference for profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    from synth import make_config
    t0 = time.perf_counter()
    cfg = make_config(args.config)
    log(f"[bench] inputs {cfg['name']}: {cfg['G']} grains in {time.perf_counter() - t0:.1f} s")
    precision = args.precision or cfg["precision"]
    main_res = run_gpu(cfg, precision, args.steps, args.warmup, copy_probe=args.copy_probe,
                       redistance=args.redistance, autotune=args.autotune)
    s_bytes = 4 if precision == "fp32" else 8
    line = {
        "metric": "grain-voxel updates/s per step (mixed batched vs FP64 plain) + %HBM roofline",
        "value": main_res["value"],
        "unit": "grain-voxel updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": list(cfg["n"]), "grains": cfg["G"],
                   "sigma_voxels": cfg["sigma"], "band_voxels": cfg["W"],
                   "precision": precision, "redistance": args.redistance, "alive_after": main_res["alive"],
                   "superposition": round(main_res["superposition"], 3)},
        "roofline": roofline(main_res, s_bytes),
    }
    rl = line["roofline"]
    workload = ("3d256_8000g" if args.config == 3 else f"config{args.config}") + (
        "_euclid" if args.redistance == "euclid" else "")
    rl["traffic"] = recorded_traffic(rl["kernel"], precision, workload)
    if not args.no_plain and precision != "fp64":
        plain = run_gpu(cfg, "fp64", args.steps, args.warmup, redistance=args.redistance, autotune=args.autotune)
        line["plain_fp64"] = dict(value=plain["value"], ms_per_step=plain["ms_per_step"],
                                  roofline=roofline(plain, 8), mixed_speedup=main_res["value"] / plain["value"])
    if args.autotune:
        line["tuning"] = {"lds_bytes": main_res["tuned"][0], "small_class_bytes": main_res["tuned"][1]}
    if args.copy_probe:
        line["copy_probe"] = main_res["copy_probe"]
    if args.coarsen:
        line["coarsen"] = run_coarsen(cfg, precision, args.warmup, args.coarsen)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.config)
        line["cpu_baseline_1thread"] = cpu_baseline(args.config, threads=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
