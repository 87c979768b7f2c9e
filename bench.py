"""Throughput of the level-set grain-growth step on one MI355X.

Prints ONE JSON line: grain-voxel updates per second of the batched mixed
(FP32) step on the 3D 256^3 / 8000-grain lognormal workload (captured HIP
graphs, no per-kernel timing in the timed region), the plain FP64 path on the
same inputs, the roofline of the dominant kernel (per-kernel HIP events of a
second, profiled run of the same steps; algorithmic bytes), the whole step
against the HBM roofline on the step's algorithmic bytes, a measured streaming
copy beside the published peak, and the FP64 CPU oracle timed on a bounded
sample of the same workload.

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
SOURCES = [os.path.join(ROOT, "paper_1701_06658_amd", "csrc", f)
           for f in ("gg_kernels.hpp", "gg_march.hpp", "gg_closest.hpp", "gg_lib.hip")]
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes per grain voxel of one launch, by kernel class, in units of
# the stored value size s (plus fixed extra bytes): every sweep reads its input
# box values once and writes its output box values once.  With the predictor
# correction the corrector writes the ID-field and the predictor reads it (the
# re-initialization's carrying of the ID-field to the new boxes is not counted:
# it is this design's, not the method's).
ALG_BYTES = {"predict": (2, 0), "compare": (2, 0), "reinit": (2, 0)}
ALG_BYTES_PHYS = {"predict": (2, 4), "compare": (2, 4), "reinit": (2, 0)}
# closest-point weights: read phi and the ID-field, write the weight
ALG_BYTES_CLOSEST = (2, 4)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def euclid_sweeps(dim, W):
    """Jacobi sweep count of the Euclidean re-initialization variant (the
    library's rule): ceil(sqrt(dim) W) + 1, rounded up to an even count."""
    K = int(math.ceil(math.sqrt(dim) * W)) + 1
    return K + (K & 1)


def step_alg_bytes(s_bytes, physics):
    """Algorithmic bytes per grain voxel of a whole step: three sweeps, each
    reading and writing the box values once (+ the ID-field written by the
    corrector and read by the predictor with the correction)."""
    return 6 * s_bytes + (8 if physics else 0)


def _phys(cfg):
    import paper_1701_06658_amd as gg
    if cfg.get("physics") == "anisotropic":
        return dict(physics=gg.PHYS_MISORIENTATION, quat=cfg["quat"], theta_c_deg=cfg["theta_c_deg"])
    if cfg.get("physics") == "magnetic":
        return dict(physics=gg.PHYS_BULK, energy=cfg["energy"], voxel_m=cfg["h_phys"], gamma_max=cfg["gamma_max"])
    return {}


CLOSEST = False  # --closest-point: correction weights from the closest boundary point


def make_sim(cfg, precision, redistance, batched, order_size=True):
    import paper_1701_06658_amd as gg
    return gg.Simulation(cfg["labels"], cfg["W"], G=cfg["G"], precision=precision, redistance=redistance,
                         batched=batched, order_size=order_size, closest_point=CLOSEST, **_phys(cfg))


def run_gpu(cfg, precision, steps, warmup, redistance="taxicab", batched=True, order_size=True,
            autotune=False, copy_probe=False):
    """Timed run: warm-up steps, then `steps` steps between stream
    synchronisations, with no per-kernel timing."""
    t0 = time.perf_counter()
    sim = make_sim(cfg, precision, redistance, batched, order_size)
    sim.sync()
    log(f"[bench] {precision} batched={batched}: created in {time.perf_counter() - t0:.2f} s")
    tuned = None
    if autotune:
        # the tuner's steps (one per candidate schedule) are warm-up steps
        tuned = sim.autotune(cfg["dt"], 1)
        log(f"[bench] {precision}: autotuned schedule {tuned}")
    if warmup:
        sim.step(cfg["dt"], warmup)
    sim.sync()
    gv0 = sim.stats()["total_grain_voxels"]
    t0 = time.perf_counter()
    sim.step(cfg["dt"], steps)
    sim.sync()
    dt = time.perf_counter() - t0
    st = sim.stats()
    gv = st["total_grain_voxels"] - gv0
    out = dict(value=gv / dt, ms_per_step=1e3 * dt / steps, device_ms_per_step=st["last_step_ms"],
               grain_voxels=gv, alive=st["alive"], superposition=st["superposition"], tuned=tuned)
    log(f"[bench] {precision} batched={batched}: {steps} steps in {dt:.4f} s, {out['value']:.3e} gv/s, "
        f"alive {st['alive']}")
    if copy_probe:
        # one state download after the timed steps: k_convert reads every stored
        # value once (4 or 8 B) and writes it as a double; its byte counters
        # calibrate the profiler
        _, v = sim.values()
        s = 4 if precision == "fp32" else 8
        out["copy_probe"] = dict(kernel="k_convert", values=int(v.size), read_bytes=int(v.size) * s,
                                 write_bytes=int(v.size) * 8, steps_all=warmup + steps,
                                 grain_voxels_all=int(st["total_grain_voxels"]))
    sim.close()
    return out


def run_profiled(cfg, precision, steps, warmup, redistance="taxicab", order_size=True):
    """The same steps again on a fresh simulation with per-kernel HIP events
    (plain launches)."""
    sim = make_sim(cfg, precision, redistance, False, order_size)
    if warmup:
        sim.step(cfg["dt"], warmup)
    sim.profile(True)
    sim.step(cfg["dt"], steps)
    kt = sim.kernel_times()
    sim.profile(False)
    sim.close()
    return kt


def source_digest():
    """SHA-256 of the kernel sources: a recorded counter figure applies only to them."""
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, precision, workload):
    """Counter-measured HBM bytes per grain voxel of `kernel` from the committed
    summary profiles/traffic_<kernel>_<workload>_<precision>.md, or None when
    the summary is missing or was taken from other kernel sources."""
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
        return float(fields["hbm_bytes_per_gv"])
    except (KeyError, ValueError):
        return None


def recorded_error_vs_oracle(precision="fp32"):
    """The mixed path's error against the FP64 oracle over trajectories, per
    result (first divergence step, largest band |dphi|, ownership mismatch
    share, worst volume error, alive-count difference), from the committed
    summary profiles/error_vs_oracle_<precision>.md of the GPU test
    tests/test_gpu_mixed_trajectory.py; source_match tells whether it was
    taken from the current kernel sources.  None when there is no summary."""
    path = os.path.join(PROFILES, f"error_vs_oracle_{precision}.md")
    if not os.path.exists(path):
        return None
    work, digest = {}, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("- source_sha256:"):
                digest = line.split(":", 1)[1].strip().strip("`")
            elif line.startswith("- {"):
                rec = json.loads(line[2:])
                rec.pop("per_step", None)
                work[rec.pop("workload")] = rec
    return dict(workloads=work, source_match=digest == source_digest(),
                test="tests/test_gpu_mixed_trajectory.py")


def roofline(kt, s_bytes, physics, sweeps=0, workload=None, precision=None):
    """Per-kernel achieved GB/s of algorithmic bytes (HIP-event span times)
    and the dominant kernel's roofline entry."""
    table = dict(ALG_BYTES_PHYS if physics else ALG_BYTES)
    if CLOSEST:
        table["closest"] = ALG_BYTES_CLOSEST
    if sweeps:
        # each Jacobi sweep of the Euclidean variant reads and writes every value
        # once; one timed span holds all sweeps of a step
        table["reinit_sweep"] = (2 * sweeps, 0)
    best = None
    per = {}
    for name, (mult, extra) in table.items():
        k = kt[name]
        if not k["launches"] or k["ms"] <= 0 or not k["voxels"]:
            continue
        bpv = mult * s_bytes + extra
        bytes_alg = bpv * k["voxels"]
        avg_ms = k["ms"] / k["launches"]
        gbs = bytes_alg / (k["ms"] * 1e-3) / 1e9
        rec = recorded_traffic(name, precision, workload) if workload else None
        per[name] = dict(avg_ms=avg_ms, gbs=gbs, bytes_per_launch=bytes_alg / k["launches"],
                         launches=k["launches"], voxels_per_launch=k["voxels"] / k["launches"],
                         alg_bytes_per_gv=bpv, traffic_bytes_per_gv=rec,
                         traffic_over_algorithmic=(rec / bpv) if rec else None)
        if best is None or k["ms"] > kt[best]["ms"]:
            best = name
    r = per[best]
    traffic = r["traffic_bytes_per_gv"] * r["voxels_per_launch"] if r["traffic_bytes_per_gv"] else None
    return dict(bound="hbm", kernel=best, achieved=r["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=r["gbs"] / HBM_PEAK_GBS, traffic=traffic,
                traffic_over_algorithmic=r["traffic_over_algorithmic"],
                avg_launch_ms=r["avg_ms"], alg_bytes_per_launch=r["bytes_per_launch"], launches=r["launches"],
                per_kernel={k: dict(GBs=round(v["gbs"], 1), avg_ms=round(v["avg_ms"], 5),
                                    traffic_over_algorithmic=v["traffic_over_algorithmic"])
                            for k, v in per.items()})


def copy_peak(nbytes=2 << 30, reps=20):
    """Measured streaming copy on the device (read + write bytes per second of
    a device-to-device copy of `nbytes` by PyTorch), beside the published HBM
    peak.  Runs in a process of its own: PyTorch brings its own HIP runtime."""
    import subprocess
    code = f"""
import json, torch
a = torch.empty({nbytes} // 4, dtype=torch.float32, device="cuda")
b = torch.empty_like(a)
a.fill_(1.0)
for _ in range(3):
    b.copy_(a)
torch.cuda.synchronize()
e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
e0.record()
for _ in range({reps}):
    b.copy_(a)
e1.record()
torch.cuda.synchronize()
print(json.dumps(e0.elapsed_time(e1) / {reps}))
"""
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
        ms = float(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None
    return dict(GBs=2.0 * nbytes / (ms * 1e-3) / 1e9, bytes=nbytes, kind="PyTorch device-to-device copy")


def cpu_baseline(index, threads=None, steps=None):
    """FP64 oracle on a bounded sample: `steps` steps (4 on all host threads, 3
    on one) of a density-matched cut of the workload (128^3 on all host
    threads; 64^3 on one thread), about 10 s of host time on an MI355X node."""
    from oracle import ORACLE_CFLAGS, Oracle, num_threads, set_num_threads
    from synth import make_config
    N = None if index == 1 else (64 if threads == 1 else 128)
    G = None if index == 1 else int(round({2: 1000, 3: 1000, 4: 781, 5: 781}[index] * (N / 128) ** 3))
    steps = steps or (3 if threads == 1 else 4)
    all_threads = num_threads()
    if threads:
        set_num_threads(threads)
    try:
        c = make_config(index, N=N, G=G)
        o = Oracle(c["labels"], c["W"], G=c["G"])
        used = num_threads()
        gv, dt = 0, 0.0
        for _ in range(steps):
            for k in range(c["G"]):
                alive, lo, ext = o.box(k)
                if alive:
                    gv += int(ext[0]) * int(ext[1]) * int(ext[2])
            t0 = time.perf_counter()
            o.step(c["dt"])
            dt += time.perf_counter() - t0
        o.close()
    finally:
        set_num_threads(all_threads)
    return dict(value=gv / dt, unit="grain-voxel updates/s", cores=used, kind="oracle",
                sample=f"{steps} FP64 oracle steps of a density-matched {c['N']}^{c['dim']} cut with "
                       f"{c['G']} grains of workload {index} ({gv} grain voxels, {dt:.2f} s); "
                       f"gcc {' '.join(ORACLE_CFLAGS)}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--precision", default=None, help="fp32 (mixed) or fp64 (plain)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain-launch runs (FP32 and the FP64 comparison)")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled per-kernel run")
    ap.add_argument("--order-id", action="store_true",
                    help="per-grain kernels in grain-id order (default: largest box first)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose the launch schedule with gg_autotune before the warm-up steps")
    ap.add_argument("--redistance", default="taxicab", choices=["taxicab", "euclid"],
                    help="re-initialization scheme: the method's taxicab one or the Euclidean variant")
    ap.add_argument("--closest-point", action="store_true",
                    help="correction weights from the closest grain-boundary point (workloads with the "
                         "misorientation weights: --config 4)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the streaming-copy measurement")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed steps, run the library's state download once: a plain "
                         "streaming kernel of known size (reference for profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    from synth import make_config
    global CLOSEST
    CLOSEST = args.closest_point
    t0 = time.perf_counter()
    cfg = make_config(args.config)
    log(f"[bench] inputs {cfg['name']}: {cfg['G']} grains in {time.perf_counter() - t0:.1f} s")
    precision = args.precision or cfg["precision"]
    physics = bool(_phys(cfg))
    main_res = run_gpu(cfg, precision, args.steps, args.warmup, redistance=args.redistance, batched=True,
                       order_size=not args.order_id, autotune=args.autotune, copy_probe=args.copy_probe)
    s_bytes = 4 if precision == "fp32" else 8
    workload = ("3d256_8000g" if args.config == 3 else f"config{args.config}") + (
        "_euclid" if args.redistance == "euclid" else "") + ("_closest" if CLOSEST else "")
    bpg = step_alg_bytes(s_bytes, physics)
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
                   "precision": precision, "redistance": args.redistance, "batched": True,
                   "order_size": not args.order_id, "closest_point": CLOSEST, "alive_after": main_res["alive"],
                   "superposition": round(main_res["superposition"], 3)},
        "step_roofline": {"alg_bytes_per_gv": bpg, "achieved": main_res["value"] * bpg / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": main_res["value"] * bpg / 1e9 / HBM_PEAK_GBS,
                          "device_ms_per_step": main_res["device_ms_per_step"]},
    }
    sweeps = euclid_sweeps(cfg["dim"], cfg["W"]) if args.redistance == "euclid" else 0
    if not args.no_profile:
        kt = run_profiled(cfg, precision, args.steps, args.warmup, redistance=args.redistance,
                          order_size=not args.order_id)
        line["roofline"] = roofline(kt, s_bytes, physics, sweeps, workload, precision)
        log(f"[bench] {precision} per kernel: " + json.dumps({k: dict(ms=round(v["ms"], 3), launches=v["launches"])
                                                              for k, v in kt.items()}))
    if not args.no_plain:
        plain32 = run_gpu(cfg, precision, args.steps, args.warmup, redistance=args.redistance, batched=False,
                          order_size=not args.order_id)
        line["plain_launches"] = dict(value=plain32["value"], ms_per_step=plain32["ms_per_step"],
                                      batched_speedup=main_res["value"] / plain32["value"])
    if not args.no_plain and precision != "fp64":
        plain = run_gpu(cfg, "fp64", args.steps, args.warmup, redistance=args.redistance, batched=False,
                        order_size=not args.order_id)
        line["plain_fp64"] = dict(value=plain["value"], ms_per_step=plain["ms_per_step"],
                                  step_roofline_frac=plain["value"] * step_alg_bytes(8, physics) / 1e9 / HBM_PEAK_GBS,
                                  mixed_speedup=main_res["value"] / plain["value"])
        if not args.no_profile:
            kt64 = run_profiled(cfg, "fp64", args.steps, args.warmup, redistance=args.redistance,
                                order_size=not args.order_id)
            line["plain_fp64"]["roofline"] = roofline(kt64, 8, physics, sweeps, workload, "fp64")
    if args.autotune:
        line["tuning"] = main_res["tuned"]
    if precision == "fp32":
        line["error_vs_oracle"] = recorded_error_vs_oracle("fp32")
    if args.copy_probe:
        line["copy_probe"] = main_res["copy_probe"]
    if not args.no_copy:
        line["copy_peak"] = copy_peak()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.config)
        line["cpu_baseline_1thread"] = cpu_baseline(args.config, threads=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
