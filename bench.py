"""Benchmark of the co-scheduled physics + render step loop on one MI355X.

Workload (default): 1024 envs x 32 bodies (16 spheres, 16 cubes), one
128x128 RGB-D camera per env; one step = every env advanced one physics step
(4 substeps) and rendered once.  Reports env-steps/s co-scheduled (value)
next to the serialized loop, the dominant kernel's roofline, and the CPU
oracle on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s (sim+render) co-scheduled vs serialized; p99 rollout latency"
HBM_PEAK_GBS = 8000.0
TUNED = "autotuned"  # the finalist that is the autotuner's choice
CSRC = os.path.join(ROOT, "paper_2605_01352_amd", "csrc")
KERNEL_SOURCES = {"raster_tiles": ["raster.hip", "vuda_internal.h"], "raster_setup": ["raster.hip", "vuda_internal.h"],
                  "raster_fused": ["raster.hip", "vuda_internal.h"], "physics": ["physics.hip", "vuda_internal.h"]}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_c{}.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def enqueue(w, schedule, n_envs, iters):
    if schedule == "pipelined":
        # tiles of S_t beside the setup of S_t+1 beside the step S_t+1 -> S_t+2
        from paper_2605_01352_amd import vuda
        w.run(vuda.SCHED_PIPELINED, iters)
        return
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


def timed(torch, w, schedule, n_envs, steps, warmup, st0=None, after_warmup=None):
    if st0 is not None:
        w.load_state(st0)  # every measurement starts from the same scene state
    enqueue(w, schedule, n_envs, warmup)
    torch.cuda.synchronize()
    if after_warmup is not None:
        after_warmup()
    t0 = time.perf_counter()
    enqueue(w, schedule, n_envs, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    w.wait()
    return dt


def launch_stats(vuda, w):
    """Average launch duration (s) and launch count per kernel since the last
    read, from the HIP events the library records around each launch on the
    stream the kernel runs on."""
    out = {}
    for name, k in (("physics", vuda.KERNEL_PHYSICS), ("raster_setup", vuda.KERNEL_RASTER_SETUP),
                    ("raster_tiles", vuda.KERNEL_RASTER_TILES), ("raster_fused", vuda.KERNEL_RASTER_FUSED)):
        t = w.kernel_times(k)
        n = max(1, t["launches"])
        out[name] = {"launches": t["launches"], "avg_s": t["total_ms"] * 1e-3 / n, "max_s": t["max_ms"] * 1e-3}
    return out


def phase_seconds(st, steps, presetup):
    """Per-step GPU time of the step phase and of the render phase: the
    raster setup belongs to the step with presetup, to the render without."""
    per = {k: v["avg_s"] * v["launches"] / steps for k, v in st.items()}
    if presetup:
        return per["physics"] + per["raster_setup"], per["raster_tiles"] + per["raster_fused"]
    return per["physics"], per["raster_setup"] + per["raster_tiles"] + per["raster_fused"]


def source_hash(kernel):
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(kernel, config):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current source of the kernel (else None).  Lines read:
    `traffic <kernel> c<config> src=<hash> fetch_kib=<f> write_kib=<w>
    fetch_factor=<a> write_factor=<b>`; bytes = 1024 (f a + w b)."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    want = source_hash(kernel)
    for line in lines:
        tok = line.strip().strip("`").split()
        if len(tok) < 3 or tok[0] != "traffic" or tok[1] != kernel or tok[2] != f"c{config}":
            continue
        kv = dict(t.split("=", 1) for t in tok[3:] if "=" in t)
        if kv.get("src") != want:
            return None
        return int(1024 * (float(kv["fetch_kib"]) * float(kv["fetch_factor"]) +
                           float(kv["write_kib"]) * float(kv["write_factor"])))
    return None


def copy_calibration(torch, mib):
    """A plain device copy of `mib` MiB (read + write of that many bytes), for
    scaling the HBM byte counters of a profiled run."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def copy_ceiling(torch, mib=1024, reps=5):
    """Practical HBM bandwidth: a device-to-device copy of `mib` MiB, median
    of `reps` (bytes read + bytes written per second)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del a, b
    t = sorted(ts)[len(ts) // 2]
    return 2.0 * n * 4 / t / 1e9


def device_info(torch):
    p = torch.cuda.get_device_properties(0)
    from paper_2605_01352_amd import build as vb
    with open(vb.MANIFEST) as f:
        built = json.load(f)["sources"]
    # one digest over the library's sources (the binding has checked that the
    # library was built from them)
    digest = hashlib.sha256("".join(f"{k}={built[k]};" for k in sorted(built)).encode()).hexdigest()[:16]
    return {"name": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "hbm_bytes": int(p.total_memory), "library_sources_sha256": digest}


VALU_PEAK_GINST = 256 * 4 * 2.4e9 / 4 / 1e9  # wave64 VALU instructions per second, 4 cycles each


def measured_valu(kernel, config):
    """Wave-VALU instructions per launch from the committed counter summary,
    if taken on the current source of the kernel.  Lines read: `valu <kernel>
    c<config> src=<hash> insts=<n>`."""
    try:
        lines = open(COUNTERS_FILE.format(config)).read().splitlines()
    except OSError:
        return None
    want = source_hash(kernel)
    for line in lines:
        tok = line.strip().strip("`").split()
        if len(tok) < 3 or tok[0] != "valu" or tok[1] != kernel or tok[2] != f"c{config}":
            continue
        kv = dict(t.split("=", 1) for t in tok[3:] if "=" in t)
        return float(kv["insts"]) if kv.get("src") == want else None
    return None


BF16_PEAK_TFLOPS = 2500.0


def policy_bench(torch, vuda, sg, scene, w, st0, steps, warmup, hidden, log):
    """The RL rollout loop with the MLP policy as a third phase: per
    iteration every env is rendered, acted on and stepped.  Serialized: one
    stream; co-scheduled: the envs in two halves, each half's act and step
    beside the other half's render.  Also the policy launch (layer 1 on MFMA
    and the head) against the bf16 MFMA roof."""
    n = scene.n_envs
    half = n // 2
    P = sg.policy_weights(2605, int(scene.cam_w[0]), int(scene.cam_h[0]), hidden, 32)
    w.set_policy(P)

    def loop(iters, cosched):
        for _ in range(iters):
            if cosched:
                w.render(0, half)
                w.act(0, half)
                w.step(0, half)
                w.render(half, n)
                w.act(half, n)
                w.step(half, n)
            else:
                w.render()
                w.act()
                w.step()

    out = {"hidden": hidden, "act_bodies": 32, "obs": int(4 * scene.cam_w[0] * scene.cam_h[0])}
    for name, split in (("serialized", 0.0), ("co_scheduled", 2.0)):
        w.cosched(split)
        w.load_state(st0)
        loop(warmup, split > 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loop(steps, split > 0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        w.wait()
        out[name] = round(n * steps / dt, 1)
        log(f"policy loop (hidden {hidden}, {name}): {n * steps / dt:.0f} env-steps/s")
    # the policy launch alone, all envs at once
    w.cosched(0.0)
    w.set_tuning(vuda.TUNE_TIMING, 1)
    w.render()
    w.act()
    w.wait()
    w.kernel_times(vuda.KERNEL_POLICY)
    for _ in range(20):
        w.act()
    w.wait()
    t = w.kernel_times(vuda.KERNEL_POLICY)
    w.set_tuning(vuda.TUNE_TIMING, 0)
    us = t["total_ms"] * 1e3 / max(1, t["launches"])
    flops = 2.0 * n * out["obs"] * hidden
    out["launch_us"] = round(us, 2)
    out["layer1_flops_per_launch"] = flops
    # layers 2 and 3 (float32), not counted in the roofline figure
    out["layers23_flops_per_launch"] = 2.0 * n * hidden * (hidden + 3 * 32)
    out["roofline"] = {"bound": "mfma", "achieved": round(flops / (us * 1e-6) / 1e12, 2),
                       "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(flops / (us * 1e-6) / 1e12 / BF16_PEAK_TFLOPS, 5)}
    log(f"policy launch (hidden {hidden}): {us:.1f} us, layer 1 {flops / (us * 1e-6) / 1e12:.1f} TFLOP/s "
        f"(bf16 MFMA)")
    w.set_policy(None)
    return out


def features_bench(torch, vuda, sg, scene, steps, log):
    """The optional features on the same workload, each in a world of its
    own: friction (mu = 0.5) in the physics kernel, half of the cubes made
    boxes (anisotropic extents and inertia) in the physics and setup
    kernels, with and without edge-edge contacts, near-plane clipping in the raster setup (cameras of this
    workload never cross the near plane, so only the cost of the cutting
    code shows), and the metric-depth fetch of every frame into device
    memory."""
    import dataclasses
    out = {}

    def kernel_avg(w, kernel, nsteps):
        w.set_tuning(vuda.TUNE_TIMING, 1)
        w.kernel_times(kernel)
        for _ in range(nsteps):
            w.step()
            w.render()
        w.wait()
        t = w.kernel_times(kernel)
        w.set_tuning(vuda.TUNE_TIMING, 0)
        return t["total_ms"] * 1e3 / max(1, t["launches"])

    boxes = sg.with_boxes(scene)
    for name, sc, kernel in (("physics_mu0", scene, vuda.KERNEL_PHYSICS),
                             ("physics_mu0.5", dataclasses.replace(scene, mu=0.5), vuda.KERNEL_PHYSICS),
                             ("physics_boxes", boxes, vuda.KERNEL_PHYSICS),
                             ("physics_boxes_edge", dataclasses.replace(boxes, edge_contacts=True),
                              vuda.KERNEL_PHYSICS),
                             ("setup", scene, vuda.KERNEL_RASTER_SETUP),
                             ("setup_boxes", boxes, vuda.KERNEL_RASTER_SETUP),
                             ("setup_near_clip", dataclasses.replace(scene, near_clip=True),
                              vuda.KERNEL_RASTER_SETUP)):
        with vuda.World(sc) as w:
            for _ in range(10):
                w.step()
                w.render()
            w.wait()
            out[name + "_us"] = round(kernel_avg(w, kernel, steps), 2)
    with vuda.World(scene) as w:
        w.step(nsteps=5)
        w.render()
        w.wait()
        n = w.fetch_bytes(vuda.FETCH_DEPTH_METRIC) // 4
        dev = torch.empty(n, dtype=torch.float32, device="cuda")
        w.fetch(vuda.FETCH_DEPTH_METRIC, out=dev)
        t0 = time.perf_counter()
        for _ in range(20):
            w.fetch(vuda.FETCH_DEPTH_METRIC, out=dev)
        dt = (time.perf_counter() - t0) / 20
        out["metric_depth_fetch_us"] = round(dt * 1e6, 1)
        out["metric_depth_GBs"] = round(8.0 * n / dt / 1e9, 1)  # 4 B read + 4 B written per pixel
    log(f"features: {out}")
    return out


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may use."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except Exception:
        allowed = os.cpu_count() or 1
    return model, os.cpu_count() or 1, allowed


def cpu_baseline(scene_fn, n_envs, steps, start_state=None):
    """The oracle (plain C, one env per thread at a time) on a bounded sample
    of the workload.  Threads: the CPU share one GPU of this machine may use
    (16), or fewer if the process may use fewer CPUs."""
    import oracle
    model, nproc, allowed = host_cpu()
    threads = max(1, min(16, allowed))
    s = scene_fn(n_envs)
    st = s.state() if start_state is None else {k: v.copy() for k, v in start_state.items()}
    t0 = time.perf_counter()
    status, _, _ = oracle.run_batch(s, st, steps, nthreads=threads, do_render=True)
    dt = time.perf_counter() - t0
    return dict(value=n_envs * steps / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n_envs} envs x {steps} steps of the same workload from the same mid-horizon state "
                       f"(seeded, same content), {threads} threads over whole envs, {dt:.1f} s; host: {model}, "
                       f"nproc {nproc}, {allowed} CPUs allowed to this process; 16 is the host CPU share of "
                       f"one GPU on this machine",
                host={"cpu_model": model, "nproc": nproc, "cpus_allowed": allowed, "threads": threads},
                seconds=round(dt, 2), status=int(status))


def divergence_report(vuda, sg, cfgs=((1, 16), (2, 32)), steps=100):
    """GPU and oracle each running free from the spawn for `steps` steps:
    the largest position difference over all bodies at each step (reported,
    not gated)."""
    import numpy as np
    import oracle
    out = {}
    for cfg, n in cfgs:
        scene = sg.config_scene(cfg, n_envs=n)
        st_o = scene.state()
        rows = []
        with vuda.World(scene) as w:
            for t in range(1, steps + 1):
                w.step()
                oracle.step_scene(scene, st_o)
                g = w.state()
                dp = np.linalg.norm(g["pos"].astype(np.float64) - st_o["pos"].astype(np.float64), axis=1)
                same = all(np.array_equal(g[k], st_o[k]) for k in ("pos", "vel", "quat", "omega"))
                rows.append((float(dp.max()), bool(same)))
        first = next((t for t, (_, sm) in enumerate(rows, 1) if not sm), None)
        out[f"c{cfg}[0:{n}]"] = {
            "max_dp_m": {str(t): float(f"{rows[t - 1][0]:.3e}") for t in (1, 10, 25, 50, 75, 100) if t <= steps},
            "max_dp_over_run_m": float(f"{max(m for m, _ in rows):.3e}"),
            "bit_equal_steps": sum(sm for _, sm in rows), "first_difference_step": first}
    return out


CONFIG_NAMES = {1: "plain serialized loop: 16 envs x 8 spheres, 64x64 RGB-D",
                2: "co-scheduled: 1024 envs x 32 bodies (16 spheres / 16 cubes), 128x128 RGB-D, "
                   "u8 RGB + u32 depth, FP32 state",
                3: "pipelined data-gen: 4096 envs x 64 bodies, 2 cameras 256x256",
                4: "uneven batching: 2048 envs, Poisson(24) bodies, {64,128,256}^2"}


def contact_stats(vuda, scene, st):
    """Contact pairs of one step from state st (a debug world loaded with
    it): pairs per substep, body-body and body-ground, summed over envs."""
    with vuda.World(scene, debug=True) as wd:
        wd.load_state(st)
        wd.step()
        wd.wait()
        cts = wd.contacts()
    S = scene.substeps
    tot = sum(len(p) for env in cts for p in env) / S
    body = sum(int((p[:, 1] != vuda.GROUND).sum()) for env in cts for p in env) / S
    return {"pairs_per_substep": round(tot, 1), "body_pairs_per_substep": round(body, 1),
            "ground_pairs_per_substep": round(tot - body, 1)}


def physics_leg(torch, vuda, scene, start, steps, log):
    """Physics launches alone on a config (one launch per step, each timed
    by its own event pair), from `start` steps past the spawn."""
    with vuda.World(scene) as w:
        w.step(nsteps=start)
        w.wait()
        w.set_tuning(vuda.TUNE_TIMING, 1)
        w.kernel_times(vuda.KERNEL_PHYSICS)
        for _ in range(steps):
            w.step()
        w.wait()
        t = w.kernel_times(vuda.KERNEL_PHYSICS)
        w.set_tuning(vuda.TUNE_TIMING, 0)
    us = t["total_ms"] * 1e3 / max(1, t["launches"])
    algo = 120 * scene.n_bodies
    out = {"envs": scene.n_envs, "bodies": int(scene.n_bodies), "from_step": start, "launches": t["launches"],
           "launch_us": round(us, 2), "max_launch_us": round(t["max_ms"] * 1e3, 2), "bytes_per_launch": algo,
           "roofline": {"bound": "hbm", "achieved": round(algo / (us * 1e-6) / 1e9, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(algo / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 5)}}
    log(f"physics leg {scene.name}: {us:.1f} us per launch ({out['roofline']['frac']:.4f} of the HBM roof)")
    return out


def uneven_c4_leg(torch, vuda, scene, start, steps, log):
    """The uneven config (Poisson body counts, mixed frame sizes) from `start`
    steps past the spawn: the serialized loop with default launches, the
    choice of vuda_autotune (schedule, CU split, persistent grids, graphs,
    tile size, raster path, ...) applied and timed, and the config's own
    launch plan -- one persistent launch per phase and graph-captured steps
    -- on the tuned split, with grids of the resident workgroups and with one
    (physics) and two (raster setup) workgroups per CU.  Medians of 3
    windows."""
    n = scene.n_envs
    with vuda.World(scene) as w:
        w.step(nsteps=start)
        w.wait()
        st0 = w.state()

        def med(sched):
            return sorted(timed(torch, w, sched, n, steps, 5, st0) for _ in range(3))[1]

        w.cosched(0.0)
        ser = n * steps / med("serial")
        w.load_state(st0)
        t0 = time.perf_counter()
        choice = w.autotune(steps=steps)
        t_tune = time.perf_counter() - t0
        sched = vuda.SCHED_NAMES[int(choice["schedule"])]
        tuned = n * steps / med(sched)
        # persistent grids of the workgroups the GPU holds at once (the
        # kernels' occupancy times the CU count), then of one and two per CU
        ncu = torch.cuda.get_device_properties(0).multi_processor_count
        plans = {}
        for name, pg, rg in (("resident", vuda.PERSISTENT_RESIDENT, vuda.PERSISTENT_RESIDENT),
                             ("per_cu_1_2", ncu, 2 * ncu)):
            for k, v in ((vuda.TUNE_PHYS_PERSISTENT, pg), (vuda.TUNE_RASTER_PERSISTENT, rg), (vuda.TUNE_GRAPHS, 1)):
                w.set_tuning(k, v)
            plans[name] = round(n * steps / med(sched), 1)
        plan = plans["resident"]
    out = {"envs": n, "bodies": int(scene.n_bodies), "from_step": start, "serialized": round(ser, 1),
           "autotuned": round(tuned, 1), "speedup_vs_serialized": round(tuned / ser, 4),
           "autotune_choice": {k: (round(v, 1) if isinstance(v, float) else v) for k, v in choice.items()},
           "autotune_seconds": round(t_tune, 2),
           "persistent_graphs_on_tuned_split": round(plan, 1), "persistent_graphs_grids": plans}
    log(f"c4: serialized {ser:.0f}, autotuned ({sched}@{choice['cu_split']:g}) {tuned:.0f} env-steps/s "
        f"({tuned / ser:.3f}x); persistent + graphs {plans}; choice {choice}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--start", type=int, default=-1,
                    help="steps advanced on the GPU before any timed window (default: half the horizon)")
    ap.add_argument("--windows", type=int, default=5, help="timed windows per mode; the median is reported")
    ap.add_argument("--gpu-warmup", type=float, default=3.0,
                    help="seconds of untimed serialized and co-scheduled iterations before any measurement")
    ap.add_argument("--envs", type=int, default=None, help="fewer envs (debug only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the physics leg at the 4096-env config")
    ap.add_argument("--no-c4", action="store_true", help="skip the autotuned leg at the uneven 2048-env config")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner leg at the bench config")
    ap.add_argument("--serve-seconds", type=float, default=120.0,
                    help="length of the continuous-batching serving run (0: skip)")
    ap.add_argument("--capacity-rates", default="100,150,200,300,400",
                    help="arrival rates of the serving capacity sweep, 10 s each (empty: skip)")
    ap.add_argument("--splits", default="0.25,0.375,0.5,0.625,0.75")
    ap.add_argument("--prios", default="3",
                    help="issue priorities of the step's waves tried on unmasked streams")
    ap.add_argument("--profile", type=int, default=0,
                    help="only run this many serialized then co-scheduled steps (for rocprofv3)")
    ap.add_argument("--physics-profile", type=int, default=0,
                    help="only run this many physics launches from the start state (for rocprofv3)")
    ap.add_argument("--profile-mode", default="interstep@2/p3",
                    help="the co-scheduled mode of --profile (schedule@split[/pPRIORITY])")
    ap.add_argument("--profile-serial", type=int, default=1,
                    help="with --profile: also run the serialized loop first (0: only the co-scheduled one)")
    ap.add_argument("--only", default="",
                    help="skip the sweep and time this co-scheduled mode, e.g. interstep@2")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--tune", default="", help="tuning knobs key=value,... (e.g. raster_threads=512)")
    ap.add_argument("--raster", default="auto", choices=["auto", "two", "fused"],
                    help="render path: setup + tile kernels, the fused kernel, or both measured (auto)")
    ap.add_argument("--fused-threads", type=int, default=512, help="workgroup size of the fused raster kernel")
    ap.add_argument("--policy-hidden", default="256,4096",
                    help="hidden sizes of the MLP policy loops measured after the main run (0: skip); "
                         "the profiling modes take the first")
    ap.add_argument("--policy-profile", type=int, default=0,
                    help="only render once and run this many policy launches (for rocprofv3)")
    ap.add_argument("--policy-loop", type=int, default=0,
                    help="only time the policy loop, this many steps per schedule (for rocprofv3)")
    args = ap.parse_args()
    hiddens = [int(h) for h in args.policy_hidden.split(",") if h.strip() and int(h) > 0]
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the envs are independent and a multi-GPU run would "
              f"shard them with no exchange; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    from paper_2605_01352_amd import scenegen as sg
    cfg = args.config
    _, _, allowed = host_cpu()
    workers = max(1, min(16, allowed))
    # scenes are built before anything touches the GPU
    log(f"building scene c{cfg}")
    scene = sg.config_scene(cfg, n_envs=args.envs, workers=workers)
    scene3 = None
    if cfg == 2 and not args.no_c3 and not args.profile and not args.policy_profile and not args.policy_loop \
            and not args.only and not args.physics_profile:
        t0 = time.perf_counter()
        scene3 = sg.config_scene(3, workers=workers)
        log(f"built scene c3 in {time.perf_counter() - t0:.1f} s")
    scene4 = None
    if scene3 is not None and not args.no_c4:
        scene4 = sg.config_scene(4, workers=workers)

    import torch
    from paper_2605_01352_amd import vuda

    torch.cuda.init()
    if args.copy_calib:
        copy_calibration(torch, args.copy_calib)
    n_envs = scene.n_envs
    horizon = sg.CONFIG_STEPS.get(cfg, 100)
    start = horizon // 2 if args.start < 0 else args.start
    w = vuda.World(scene)
    log(f"world: {n_envs} envs, {scene.n_bodies} bodies, {scene.n_cams} cameras, "
        f"{w.info()['arena_bytes'] / 2**20:.1f} MiB arena")
    knob_ids = {"raster_threads": vuda.TUNE_RASTER_THREADS, "rec_cap": vuda.TUNE_REC_CAP,
                "phys_persistent": vuda.TUNE_PHYS_PERSISTENT,
                "raster_persistent": vuda.TUNE_RASTER_PERSISTENT, "graphs": vuda.TUNE_GRAPHS,
                "phys_prio": vuda.TUNE_PHYS_PRIORITY, "broadphase": vuda.TUNE_BROADPHASE,
                "presetup": vuda.TUNE_PRESETUP, "policy_layered": vuda.TUNE_POLICY_LAYERED,
                "phys_pack": vuda.TUNE_PHYS_ENVS_PER_WAVE, "tile": vuda.TUNE_TILE_SIZE,
                "fused": vuda.TUNE_RASTER_FUSED, "fused_recs": vuda.TUNE_FUSED_LDS_RECORDS,
                "tile_waves": vuda.TUNE_TILE_WAVES, "tile_prio": vuda.TUNE_TILE_PRIORITY}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        w.set_tuning(knob_ids[k], int(v))
    # every timed window starts from the state `start` steps past the spawn
    # (bodies fallen and piled), reached on the GPU outside any window
    w.step(nsteps=start)
    w.wait()
    st0 = w.state()
    log(f"start state: {start} steps past the spawn")
    if args.policy_profile:
        w.set_policy(sg.policy_weights(2605, int(scene.cam_w[0]), int(scene.cam_h[0]), hiddens[0], 32))
        w.render()
        for _ in range(args.policy_profile):
            w.act()
        w.wait()
        log(f"policy profile run: {args.policy_profile} launches")
        w.close()
        return
    if args.policy_loop:
        policy_bench(torch, vuda, sg, scene, w, st0, args.policy_loop, 4, hiddens[0], log)
        w.close()
        return
    if args.physics_profile:
        for _ in range(args.physics_profile):
            w.step()
        w.wait()
        log(f"physics profile run: {args.physics_profile} launches from step {start}")
        w.close()
        return
    if args.profile:
        psched, rest = args.profile_mode.split("@")
        psplit, _, pprio = rest.partition("/p")
        if args.profile_serial:
            w.cosched(0.0)
            dt_s = timed(torch, w, "serial", n_envs, args.profile, 2, st0)
            log(f"profile run from step {start}: serialized {dt_s / args.profile * 1e6:.1f} us/step")
        w.cosched(float(psplit))
        if pprio:
            w.set_tuning(vuda.TUNE_PHYS_PRIORITY, int(pprio))
        dt_c = timed(torch, w, psched, n_envs, args.profile, 2, st0)
        log(f"profile run from step {start}: co-scheduled ({args.profile_mode}) "
            f"{dt_c / args.profile * 1e6:.1f} us/step")
        w.close()
        return

    def median_windows(sched):
        dts = sorted(timed(torch, w, sched, n_envs, args.steps, args.warmup, st0) for _ in range(max(1, args.windows)))
        return dts[len(dts) // 2], dts

    def kernel_run(sched):
        """The same window again with a HIP event pair around every launch:
        the per-kernel launch durations of that window.  The events cost
        throughput of their own, so the headline figures come from the runs
        without them."""
        w.set_tuning(vuda.TUNE_TIMING, 1)
        timed(torch, w, sched, n_envs, args.steps, args.warmup, st0,
              after_warmup=lambda: launch_stats(vuda, w))
        st = launch_stats(vuda, w)  # launches of the timed window
        w.set_tuning(vuda.TUNE_TIMING, 0)
        return st

    # render paths measured: the setup and tile kernels (setup workgroups of
    # t threads, tile workgroups of w waves), and the fused kernel (records
    # and bins in LDS)
    two_threads = w.get_tuning(vuda.TUNE_RASTER_THREADS)
    two_waves = w.get_tuning(vuda.TUNE_TILE_WAVES)
    path_knobs = {}
    if args.raster in ("auto", "two"):
        shapes = [(two_threads, two_waves)]
        if args.raster == "auto":
            shapes += [(t, wv) for t, wv in ((128, 4), (128, 2), (256, 2), (256, 4)) if (t, wv) != shapes[0]]
        for t, wv in shapes:
            path_knobs[f"t{t}w{wv}"] = {vuda.TUNE_RASTER_FUSED: 0, vuda.TUNE_RASTER_THREADS: t,
                                        vuda.TUNE_TILE_WAVES: wv}
    if args.raster in ("auto", "fused"):
        path_knobs["fused"] = {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_THREADS: args.fused_threads}
    paths = list(path_knobs)

    def set_path(path):
        for k, v in path_knobs[path].items():
            w.set_tuning(k, v)

    w.set_tuning(vuda.TUNE_TIMING, 0)
    # The first seconds of GPU work in a process run a few percent slower than
    # the rest (clocks and caches settle); both loops run untimed first, so
    # that neither side of the comparison is measured cold.
    t_end = time.perf_counter() + args.gpu_warmup
    while time.perf_counter() < t_end:
        for split, sched in ((0.0, vuda.SCHED_SERIAL), (2.0, vuda.SCHED_PIPELINED)):
            w.cosched(split)
            w.load_state(st0)
            w.run(sched, 50)
            w.wait()
    w.cosched(0.0)
    ser_paths = {}
    for path in paths:
        set_path(path)
        ser_paths[path] = median_windows("serial")
        log(f"serialized, raster {path}: {n_envs * args.steps / ser_paths[path][0]:.0f} env-steps/s")
    ser_path = min(ser_paths, key=lambda p: ser_paths[p][0])
    dt_ser, ser_windows = ser_paths[ser_path]
    set_path(ser_path)
    alone = kernel_run("serial")
    presetup = w.get_tuning(vuda.TUNE_PRESETUP) != 0
    Ts, Tr = phase_seconds(alone, args.steps, presetup)
    ser = n_envs * args.steps / dt_ser
    log(f"serialized ({ser_path} raster): {ser:.0f} env-steps/s (median of {len(ser_windows)} windows); per step "
        f"alone: step phase {Ts*1e6:.1f} us, render phase {Tr*1e6:.1f} us, bound {(Ts + Tr) / max(Ts, Tr):.3f}x "
        f"(physics {alone['physics']['avg_s']*1e6:.1f}, setup {alone['raster_setup']['avg_s']*1e6:.1f}, "
        f"tiles {alone['raster_tiles']['avg_s']*1e6:.1f}, fused {alone['raster_fused']['avg_s']*1e6:.1f} us "
        f"per launch)")
    # co-scheduled candidates: unmasked streams and CU splits, both overlap
    # patterns; on unmasked streams also raised issue priorities of the step's
    # waves (they share CUs with the render's)
    p0 = w.get_tuning(vuda.TUNE_PHYS_PRIORITY)
    prios = [int(p) for p in filter(None, args.prios.split(",")) if int(p) != p0]
    scheds = ("interstep", "intertraj", "pipelined")
    cands = [(2.0, sched, p0) for sched in scheds]
    cands += [(2.0, sched, p) for p in prios for sched in scheds]
    cands += [(float(x), sched, p0) for x in filter(None, args.splits.split(",")) for sched in scheds]
    cands = [c + (path, 0) for path in paths for c in cands]
    # the tile kernel's wave priority, on unmasked streams (its waves share CUs
    # with the step's)
    cands += [(sp, sc, pr, path, 1) for sp, sc, pr, path, _ in cands if sp == 2.0 and path != "fused"]
    if args.only:
        cands = []
    sweep = {}

    def name(sched, split, prio, path, tprio=0):
        return (f"{sched}@{split:g}" + (f"/p{prio}" if prio != p0 else "") + f"/{path}" +
                (f"/r{tprio}" if tprio else ""))

    def parse(nm):
        sched, rest = nm.split("@")
        tok = rest.split("/")
        prio, path, tprio = p0, paths[0], 0
        for t in tok[1:]:
            if t in path_knobs:
                path = t
            elif t.startswith("p"):
                prio = int(t[1:])
            elif t.startswith("r"):
                tprio = int(t[1:])
        return sched, float(tok[0]), prio, path, tprio

    # every knob the autotuner sets, as (choice key, tuning key)
    tuner_knobs = [("raster_threads", vuda.TUNE_RASTER_THREADS), ("rec_cap", vuda.TUNE_REC_CAP),
                   ("phys_persistent", vuda.TUNE_PHYS_PERSISTENT),
                   ("raster_persistent", vuda.TUNE_RASTER_PERSISTENT), ("phys_priority", vuda.TUNE_PHYS_PRIORITY),
                   ("broadphase", vuda.TUNE_BROADPHASE), ("presetup", vuda.TUNE_PRESETUP),
                   ("graphs", vuda.TUNE_GRAPHS), ("phys_envs_per_wave", vuda.TUNE_PHYS_ENVS_PER_WAVE),
                   ("tile_size", vuda.TUNE_TILE_SIZE), ("raster_fused", vuda.TUNE_RASTER_FUSED),
                   ("tile_waves", vuda.TUNE_TILE_WAVES), ("tile_priority", vuda.TUNE_TILE_PRIORITY)]
    base_knobs = {k: w.get_tuning(k) for _, k in tuner_knobs}

    def apply(split, prio, path, tprio=0):
        for k, v in base_knobs.items():
            w.set_tuning(k, v)
        w.cosched(split)
        w.set_tuning(vuda.TUNE_PHYS_PRIORITY, prio)
        w.set_tuning(vuda.TUNE_TILE_PRIORITY, tprio)
        set_path(path)

    for split, sched, prio, path, tprio in cands:
        apply(split, prio, path, tprio)
        dt = timed(torch, w, sched, n_envs, args.steps, args.warmup, st0)
        nm = name(sched, split, prio, path, tprio)
        sweep[nm] = n_envs * args.steps / dt
        log(f"  {nm:26s}: {n_envs * args.steps / dt:.0f} env-steps/s")
    # the library's autotuner on this workload (its own trials from the start
    # state); its choice joins the finalists
    choice, t_tune = None, None
    if not args.only and not args.no_autotune:
        w.load_state(st0)
        t0 = time.perf_counter()
        choice = w.autotune(steps=args.steps)  # trials as long as the headline's windows
        t_tune = time.perf_counter() - t0
        log(f"autotuner ({t_tune:.1f} s, {choice['trials']} trials): {choice}")

    def apply_choice():
        for key, k in tuner_knobs:
            w.set_tuning(k, int(choice[key]))
        w.cosched(float(choice["cu_split"]))

    # the three best sweep entries (one window each) and the autotuner's choice
    # are timed again as medians of windows; the best median is the headline
    finalists = [args.only] if args.only else sorted(sweep, key=sweep.get, reverse=True)[:3]
    if choice is not None:
        finalists.append(TUNED)
    medians = {}
    for nm in finalists:
        if nm == TUNED:
            apply_choice()
            medians[nm] = median_windows(vuda.SCHED_NAMES[int(choice["schedule"])])
        else:
            sched, split, prio, path, tprio = parse(nm)
            apply(split, prio, path, tprio)
            medians[nm] = median_windows(sched)
        log(f"  finalist {nm}: {n_envs * args.steps / medians[nm][0]:.0f} env-steps/s (median)")
    best = min(medians, key=lambda k: medians[k][0])
    if best == TUNED:
        apply_choice()
        sched = vuda.SCHED_NAMES[int(choice["schedule"])]
        split, prio, tprio = float(choice["cu_split"]), int(choice["phys_priority"]), int(choice["tile_priority"])
        path = "fused" if choice["raster_fused"] else "tuned"
        path_knobs["tuned"] = {vuda.TUNE_RASTER_FUSED: 0, vuda.TUNE_RASTER_THREADS: int(choice["raster_threads"]),
                               vuda.TUNE_TILE_WAVES: int(choice["tile_waves"])}
        if path == "fused":
            path_knobs["fused"] = {vuda.TUNE_RASTER_FUSED: 1, vuda.TUNE_RASTER_THREADS: int(choice["raster_threads"])}
    else:
        sched, split, prio, path, tprio = parse(best)
        apply(split, prio, path, tprio)
    dt, co_windows = medians[best]
    value = n_envs * args.steps / dt
    live = kernel_run(sched)
    log(f"co-scheduled ({best}): {value:.0f} env-steps/s (median of {len(co_windows)} windows), "
        f"{value / ser:.3f}x serialized")
    contacts = contact_stats(vuda, scene, st0)
    log(f"contacts at the start state: {contacts}")

    # roofline of the dominant kernel: algorithmic bytes per launch over its
    # average duration in the timed window
    px = int((scene.cam_w.astype("int64") * scene.cam_h).sum())
    body_cams = int(sum(scene.counts()[e] * (scene.cam_off[e + 1] - scene.cam_off[e]) for e in range(n_envs)))
    # algorithmic bytes: the raster setup reads 28 B of pose per body and
    # camera, the tile kernel writes 7 B per pixel
    step_bytes = {"physics": 120 * scene.n_bodies, "raster_setup": 28 * body_cams, "raster_tiles": 7 * px,
                  "raster_fused": 28 * body_cams + 7 * px}
    per_step = {k: live[k]["launches"] / args.steps for k in step_bytes}
    kinds = {}
    for kname in [k for k in step_bytes if per_step[k] > 0]:  # kernels the timed window launched
        lb = step_bytes[kname] / per_step[kname]  # launches split the env range evenly
        t = live[kname]["avg_s"]
        kinds[kname] = {"launch_us": round(t * 1e6, 2), "bytes_per_launch": int(lb),
                        "launches_per_step": per_step[kname], "GBs": round(lb / t / 1e9, 2) if t else None,
                        "alone_launch_us": round(alone[kname]["avg_s"] * 1e6, 2)}
    # the dominant kernel carries the most work per step: the largest launch
    # time alone (co-scheduled, a launch also stretches while it waits for
    # issue slots that other kernels hold)
    dom = max(kinds, key=lambda k: kinds[k]["alone_launch_us"] * per_step[k])
    ach = kinds[dom]["GBs"]
    # measured HBM bytes of a whole-workload launch, scaled to the share of
    # the workload one launch of the timed window covers
    tr_full = measured_traffic(dom, cfg)
    share = kinds[dom]["bytes_per_launch"] / step_bytes[dom]
    tr = int(tr_full * share) if tr_full is not None else None
    copy_gbs = copy_ceiling(torch)
    log(f"practical HBM ceiling (1 GiB device copy): {copy_gbs:.0f} GB/s")
    roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": tr,
            "traffic_note": (f"counters of a whole-workload launch from step {start} "
                             f"({tr_full} B), times the launch's share {share:g}") if tr_full else None,
            "bytes_per_launch": kinds[dom]["bytes_per_launch"], "launch_us": kinds[dom]["launch_us"],
            "practical_peak": round(copy_gbs, 1), "frac_of_practical": round(ach / copy_gbs, 5),
            **kinds}
    vi = measured_valu(dom, cfg)
    if vi is not None:
        vi *= kinds[dom]["bytes_per_launch"] / step_bytes[dom]  # the launch's share of the workload
        roof["valu"] = {"insts_per_launch": int(vi), "unit": "G wave-instructions/s",
                        "peak": round(VALU_PEAK_GINST, 1),
                        "achieved": round(vi / (kinds[dom]["launch_us"] * 1e-6) / 1e9, 1),
                        "frac": round(vi / (kinds[dom]["launch_us"] * 1e-6) / 1e9 / VALU_PEAK_GINST, 4),
                        "frac_alone": round(vi / (kinds[dom]["alone_launch_us"] * 1e-6) / 1e9 / VALU_PEAK_GINST, 4)
                        if kinds[dom]["alone_launch_us"] else None,
                        "note": "wave-VALU instructions per launch from the committed counters "
                                "(profiles/counters_c2.md), over the launch time of this run"}

    c3 = None
    if scene3 is not None:
        c3 = physics_leg(torch, vuda, scene3, sg.CONFIG_STEPS[3] // 2, 20, log)
        del scene3
    c4 = None
    if scene4 is not None:
        c4 = uneven_c4_leg(torch, vuda, scene4, sg.CONFIG_STEPS[4] // 2, 100, log)
        del scene4

    policy = None
    if hiddens and not args.only:
        if len(set(zip(scene.cam_w.tolist(), scene.cam_h.tolist()))) == 1:
            policy = [policy_bench(torch, vuda, sg, scene, w, st0, min(args.steps, 200), 10, h, log)
                      for h in hiddens]
        else:
            log("policy loop skipped: the policy reads one frame size, the cameras differ")

    features = None
    if not args.only:
        features = features_bench(torch, vuda, sg, scene, min(args.steps, 100), log)

    tuned = None
    if choice is not None:
        dt_t, t_windows = medians[TUNED]
        tuned = {"value": round(n_envs * args.steps / dt_t, 1),
                 "speedup_vs_serialized": round(dt_ser / dt_t, 4),
                 "windows_ms_per_step": [round(x / args.steps * 1e3, 4) for x in t_windows],
                 "choice": {k: (round(v, 1) if isinstance(v, float) else v) for k, v in choice.items()},
                 "seconds": round(t_tune, 2), "headline": best == TUNED}
        log(f"autotuned ({vuda.SCHED_NAMES[int(choice['schedule'])]}@{choice['cu_split']:g}): "
            f"{tuned['value']:.0f} env-steps/s, {tuned['speedup_vs_serialized']:.3f}x serialized")

    serving = None
    if args.serve_seconds > 0:
        from paper_2605_01352_amd import serving as srv
        log(f"serving: {args.serve_seconds:g} s of Poisson(50/s) requests ...")
        serving = srv.run(duration=args.serve_seconds, rate=50.0, log=log)
        log(f"serving: {serving}")
        rates = [float(x) for x in args.capacity_rates.split(",") if x.strip()]
        if rates:
            log("serving capacity: rising arrival rates ...")
            serving["capacity"] = srv.capacity(rates=rates, seconds=10.0, log=log)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        n_cpu = min(1024, n_envs)
        cpu_steps = {1: 50, 2: 100, 3: 5, 4: 30}.get(cfg, 20)
        st_cpu = {k: v[: int(scene.body_off[n_cpu])] for k, v in st0.items()}
        cpu = cpu_baseline(lambda n: scene if n == n_envs else scene.subset(range(n)), n_cpu, cpu_steps, st_cpu)
        cpu["per_core"] = round(cpu["value"] / cpu["cores"], 1)
        log(f"cpu baseline: {cpu['value']:.0f} env-steps/s on {cpu['cores']} threads")
        cpu["divergence"] = divergence_report(vuda, sg)
        log(f"divergence (GPU and oracle running free from the spawn): {cpu['divergence']}")
    w.close()

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "env-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded sphere/cube drops standing in for ManiSkill3 scenes)",
        "config": {"workload": CONFIG_NAMES.get(cfg, f"c{cfg}"), "envs": n_envs,
                   "bodies": int(scene.n_bodies), "cameras": int(scene.n_cams),
                   "schedule": sched, "cu_split": split, "step_priority": prio, "tile_priority": tprio,
                   "raster": {"path": "fused kernel" if path == "fused" else "setup + tile kernels",
                              "workgroup_threads": path_knobs[path][vuda.TUNE_RASTER_THREADS],
                              "tile_waves": path_knobs[path].get(vuda.TUNE_TILE_WAVES)},
                   "window": f"steps {start + args.warmup}..{start + args.warmup + args.steps} of the "
                             f"{horizon}-step horizon, median of {len(co_windows)} windows",
                   "chosen_by": "autotuner" if best == TUNED else "sweep",
                   "parallelism": "single GPU"},
        "windows_ms_per_step": {"co_scheduled": [round(x / args.steps * 1e3, 4) for x in co_windows],
                                "serialized": [round(x / args.steps * 1e3, 4) for x in ser_windows]},
        "serialized": {"value": round(ser, 1), "ms_per_step": round(dt_ser / args.steps * 1e3, 4),
                       "raster": ser_path,
                       "paths": {p: round(n_envs * args.steps / v[0], 1) for p, v in ser_paths.items()}},
        "speedup_vs_serialized": round(value / ser, 4),
        "overlap_bound": round((Ts + Tr) / max(Ts, Tr), 4),
        "phase_alone_us": {"step": round(Ts * 1e6, 2), "render": round(Tr * 1e6, 2), "presetup": presetup},
        "contacts": contacts,
        "sweep": {k: round(v, 1) for k, v in sweep.items()},
        "finalists": {k: round(n_envs * args.steps / v[0], 1) for k, v in medians.items()},
        "roofline": roof,
        "physics_c3": c3,
        "uneven_c4": c4,
        "autotuned": tuned,
        "device": device_info(torch),
        "cpu_baseline": cpu,
        "serving": serving,
        "policy": policy,
        "features": features,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
