"""Benchmark of the co-scheduled physics + render step loop on one MI355X.

Workload (default): 1024 envs x 32 bodies (16 spheres, 16 cubes), one
128x128 RGB-D camera per env; one step = every env advanced one physics step
(4 substeps) and rendered once.  Reports env-steps/s co-scheduled (value)
next to the serialized loop, the dominant kernel's roofline, and the CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s (sim+render) co-scheduled vs serialized; p99 rollout latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def enqueue(w, schedule, n_envs, iters):
    half = n_envs // 2
    for _ in range(iters):
        if schedule == "serial":
            w.step()
            w.render()
        elif schedule == "interstep":
            w.render()   # renders S_t ...
            w.step()     # ... while S_t -> S_t+1 runs beside it
        elif schedule == "intertraj":
            w.step(0, half)
            w.render(half, n_envs)
            w.step(half, n_envs)
            w.render(0, half)
        else:
            raise ValueError(schedule)


def timed(torch, w, schedule, n_envs, steps, warmup, st0=None):
    if st0 is not None:
        w.load_state(st0)  # every measurement starts from the same scene state
    enqueue(w, schedule, n_envs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    enqueue(w, schedule, n_envs, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    w.wait()
    return dt


def kernel_times(torch, vuda, w, st0, reps=20):
    """Average duration of one physics launch and one raster launch, timed
    with HIP events on the stream the kernels run on (serialized mode),
    from the initial state."""
    w.cosched(0.0)
    w.load_state(st0)
    s = torch.cuda.ExternalStream(w.stream(vuda.PHASE_STEP))
    out = {}
    for name in ("physics", "raster"):
        fn = w.step if name == "physics" else w.render
        for _ in range(3):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(s)
            fn()
            b.record(s)
        torch.cuda.synchronize()
        out[name] = sum(a.elapsed_time(b) for a, b in ev) / reps * 1e-3  # seconds
    w.wait()
    return out


def cpu_baseline(scene_fn, n_envs, steps):
    import numpy as np  # noqa: F401
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    threads = max(1, min(16, cores))
    s = scene_fn(n_envs)
    st = s.state()
    t0 = time.perf_counter()
    status, _, _ = oracle.run_batch(s, st, steps, nthreads=threads, do_render=True)
    dt = time.perf_counter() - t0
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return dict(value=n_envs * steps / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n_envs} envs x {steps} steps of the same workload (seeded, same content), "
                       f"{threads} threads over whole envs, {dt:.1f} s, host {cpu_model}",
                status=int(status))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--envs", type=int, default=None, help="fewer envs (debug only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--splits", default="0.25,0.375,0.5,0.625,0.75")
    ap.add_argument("--profile", type=int, default=0,
                    help="only run this many serialized then co-scheduled steps (for rocprofv3)")
    ap.add_argument("--tune", default="", help="tuning knobs key=value,... (e.g. raster_threads=512)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the envs are independent and a multi-GPU run would "
              f"shard them with no exchange; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_01352_amd import scenegen as sg
    from paper_2605_01352_amd import vuda

    torch.cuda.init()
    cfg = args.config
    log(f"building scene c{cfg}")
    scene = sg.config_scene(cfg, n_envs=args.envs)
    n_envs = scene.n_envs
    w = vuda.World(scene)
    log(f"world: {n_envs} envs, {scene.n_bodies} bodies, {scene.n_cams} cameras, "
        f"{w.info()['arena_bytes'] / 2**20:.1f} MiB arena")

    st0 = scene.state()
    knob_ids = {"raster_threads": vuda.TUNE_RASTER_THREADS, "rec_cap": vuda.TUNE_REC_CAP,
                "phys_persistent": vuda.TUNE_PHYS_PERSISTENT,
                "raster_persistent": vuda.TUNE_RASTER_PERSISTENT, "graphs": vuda.TUNE_GRAPHS,
                "phys_prio": vuda.TUNE_PHYS_PRIORITY, "broadphase": vuda.TUNE_BROADPHASE}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        w.set_tuning(knob_ids[k], int(v))
    if args.profile:
        w.cosched(0.0)
        dt_s = timed(torch, w, "serial", n_envs, args.profile, 2, st0)
        w.cosched(2.0)
        dt_c = timed(torch, w, "interstep", n_envs, args.profile, 2, st0)
        log(f"profile run: serialized {dt_s / args.profile * 1e6:.1f} us/step, "
            f"co-scheduled {dt_c / args.profile * 1e6:.1f} us/step")
        w.close()
        return
    kt = kernel_times(torch, vuda, w, st0)
    log(f"kernel times: physics {kt['physics']*1e6:.1f} us, raster {kt['raster']*1e6:.1f} us")
    Ts, Tr = kt["physics"], kt["raster"]

    results = {}
    w.cosched(0.0)
    results["serialized"] = timed(torch, w, "serial", n_envs, args.steps, args.warmup, st0)
    log(f"serialized: {n_envs * args.steps / results['serialized']:.0f} env-steps/s")
    # co-scheduled candidates: unmasked streams and CU splits, both overlap patterns
    cands = [(2.0, sched) for sched in ("interstep", "intertraj")]
    cands += [(float(x), sched) for x in args.splits.split(",") for sched in ("interstep", "intertraj")]
    sweep = {}
    short = args.steps
    for split, sched in cands:
        w.cosched(split)
        dt = timed(torch, w, sched, n_envs, short, 5, st0)
        sweep[f"{sched}@{split:g}"] = n_envs * short / dt
        log(f"  {sched:9s} split {split:5g}: {n_envs * short / dt:.0f} env-steps/s")
    best = max(sweep, key=sweep.get)
    sched, split = best.split("@")
    split = float(split)
    w.cosched(split)
    dt = timed(torch, w, sched, n_envs, args.steps, args.warmup, st0)
    value = n_envs * args.steps / dt
    ser = n_envs * args.steps / results["serialized"]
    log(f"co-scheduled ({best}): {value:.0f} env-steps/s, {value / ser:.3f}x serialized, "
        f"bound {(Ts + Tr) / max(Ts, Tr):.3f}x")

    # roofline of the dominant kernel (algorithmic bytes per launch / duration)
    px = int((scene.cam_w.astype("int64") * scene.cam_h).sum())
    raster_bytes = 7 * px + 28 * int(sum(scene.counts()[e] * (scene.cam_off[e + 1] - scene.cam_off[e])
                                         for e in range(n_envs)))
    phys_bytes = 120 * scene.n_bodies
    if Tr >= Ts:
        dom, tb, td = "raster", raster_bytes, Tr
    else:
        dom, tb, td = "physics", phys_bytes, Ts
    ach = tb / td / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
            "bytes_per_launch": tb, "launch_us": round(td * 1e6, 2),
            "physics": {"launch_us": round(Ts * 1e6, 2), "bytes": phys_bytes,
                        "GBs": round(phys_bytes / Ts / 1e9, 2)},
            "raster": {"launch_us": round(Tr * 1e6, 2), "bytes": raster_bytes,
                       "GBs": round(raster_bytes / Tr / 1e9, 2)}}

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(lambda n: sg.config_scene(cfg, n_envs=n), min(512, n_envs), 100 if cfg <= 2 else 10)
        log(f"cpu baseline: {cpu['value']:.0f} env-steps/s on {cpu['cores']} threads")
    w.close()

    names = {1: "plain serialized loop: 16 envs x 8 spheres, 64x64 RGB-D",
             2: "co-scheduled: 1024 envs x 32 bodies (16 spheres / 16 cubes), 128x128 RGB-D, "
                "u8 RGB + u32 depth, FP32 state",
             3: "pipelined data-gen: 4096 envs x 64 bodies, 2 cameras 256x256",
             4: "uneven batching: 2048 envs, Poisson(24) bodies, {64,128,256}^2"}
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded sphere/cube drops standing in for ManiSkill3 scenes)",
        "config": {"workload": names.get(cfg, f"c{cfg}"), "envs": n_envs,
                   "bodies": int(scene.n_bodies), "cameras": int(scene.n_cams),
                   "schedule": sched, "cu_split": split, "parallelism": "single GPU"},
        "serialized": {"value": round(ser, 1), "ms_per_step": round(results["serialized"] / args.steps * 1e3, 4)},
        "speedup_vs_serialized": round(value / ser, 4),
        "overlap_bound": round((Ts + Tr) / max(Ts, Tr), 4),
        "sweep": {k: round(v, 1) for k, v in sweep.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
