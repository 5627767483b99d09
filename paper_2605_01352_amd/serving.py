"""Serving workload driver: Poisson arrivals of rollout requests into the
continuous-batching server (vuda_serve_*), reporting p50/p99 latency and the
env-steps/s served next to the offered load.

Requests follow the serving recipe of the synthetic workloads (env count
log-uniform in [16, 512], 8-64 bodies per env, horizon uniform in [50, 500],
square resolution from {64, 128, 256}, Poisson arrivals).  Building a scene
with rejection-sampled spawns costs up to seconds for the largest requests,
so a pool of the first `pool` request specs is generated once and request r
takes the content and shape of pool[r mod pool], at its own Poisson arrival
time.  The offered load is computed from the requests actually submitted.

Usage: python -m paper_2605_01352_amd.serving [--duration 120] [--rate 50]
"""
import argparse
import json
import sys
import time

import numpy as np

from . import scenegen as sg
from . import vuda


def run(duration: float = 120.0, rate: float = 50.0, pool: int = 24, budget_gb: float = 200.0,
        cu_split: float = 2.0, schedule: int = vuda.SCHED_INTERSTEP, seed: int = 1005,
        drain: bool = True, log=None, tune=None) -> dict:
    specs = sg.serving_requests(duration_s=duration, rate=rate, seed=seed)
    pool_specs = specs[:pool]
    t0 = time.perf_counter()
    scenes = [sg.request_scene(r, seed=seed) for r in pool_specs]
    gen_s = time.perf_counter() - t0
    if log:
        log(f"serving: {len(specs)} arrivals over {duration:.0f} s, pool of {len(scenes)} request "
            f"scenes built in {gen_s:.1f} s")
    # capacity: enough slots for the budget's worth of mean requests
    max_envs = max(r.n_envs for r in pool_specs)
    cap_envs = 64 * 1024
    cap_bodies = 64 * 1024 * 48
    cap_cams = cap_envs
    cap_pixels = 1 << 31
    budget = int(budget_gb * (1 << 30))
    srv = vuda.Server(cap_envs=cap_envs, cap_bodies=cap_bodies, cap_cams=cap_cams,
                      cap_pixels=cap_pixels, hbm_budget=budget, cu_split=cu_split,
                      schedule=schedule, keep_results=False)
    for k, v in (tune or {}).items():
        srv.set_tuning(k, v)
    offered_env_steps = 0
    nsub = 0
    lat = []
    t_start = time.perf_counter()
    last_log = t_start
    i = 0
    while True:
        now = time.perf_counter() - t_start
        while i < len(specs) and specs[i].arrival_s <= now:
            p = pool_specs[i % len(pool_specs)]
            srv.submit(specs[i].rid, scenes[i % len(scenes)], p.horizon)
            offered_env_steps += p.n_envs * p.horizon
            nsub += 1
            i += 1
        st = srv.stats()
        if st["active_requests"] or st["queued"]:
            srv.tick()
            lat += [x for _, x in srv.completed()]
        elif i < len(specs):
            time.sleep(max(0.0, min(0.01, specs[i].arrival_s - now)))
        else:
            break
        if now > duration and not drain:
            break
        if log and time.perf_counter() - last_log > 10.0:
            last_log = time.perf_counter()
            log(f"  t={now:6.1f} s submitted {nsub} completed {st['completed']} active "
                f"{st['active_requests']} ({st['active_envs']} envs) queued {st['queued']}")
    wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    return {
        "requests": nsub, "completed": st["completed"], "wall_s": round(wall, 2),
        "offered_env_steps_per_s": round(offered_env_steps / duration, 1),
        "served_env_steps_per_s": round(st["env_steps"] / wall, 1),
        "latency_p50_s": round(st["latency_p50_s"], 4), "latency_p99_s": round(st["latency_p99_s"], 4),
        "latency_max_s": round(st["latency_max_s"], 4), "queue_p50_s": round(st["queue_p50_s"], 4),
        "queue_p99_s": round(st["queue_p99_s"], 4), "ticks": st["ticks"],
        "peak_reserved_gb": round(st["peak_reserved_bytes"] / 2**30, 3),
        "duration_s": duration, "rate_per_s": rate, "pool": len(scenes),
        "cu_split": cu_split, "schedule": vuda.SCHED_NAMES[schedule],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--duration", type=float, default=120.0)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--pool", type=int, default=24)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--split", type=float, default=2.0)
    ap.add_argument("--schedule", default="interstep", choices=["serial", "interstep", "intertraj"])
    a = ap.parse_args()
    sched = {"serial": vuda.SCHED_SERIAL, "interstep": vuda.SCHED_INTERSTEP,
             "intertraj": vuda.SCHED_INTERTRAJ}[a.schedule]
    res = run(a.duration, a.rate, a.pool, a.budget_gb, a.split, sched,
              log=lambda *x: print(*x, file=sys.stderr, flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
