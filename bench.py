#!/usr/bin/env python3
"""Benchmark of the MPPI update on one MI355X.

Default workload: the single-instance configuration (K = 4096 rollouts, N = 100
steps of 10 ms, 20 spheres, straight-line reference at 12 m/s) run in closed loop:
every step is one full MPPI update (rollouts, weights, weighted update, apply and
shift) whose applied control the device writes into pinned host memory, one
noise-free plant step on the device queued behind it, and the host waiting (spinning
on an event) for the control before the next update ("plain": one solve per launch
sequence).  Inputs (references for every step, obstacles, warm start) are
resident on the device before the timed region starts.  The same line carries the
batched leg (256 uneven vehicles per graph replay) and a short served leg (Poisson
arrivals, each state estimate predicted over the running median latency).
--config c1 | c3 | paper selects another single-vehicle workload (paper: the paper's
own Table I/II setting, updates every 10 ms with the interpolated warm start), c4 the
batched and c5 the full 60 s served workload.

Prints ONE JSON line on stdout (everything else goes to stderr):
  value          rollout-steps/s = K * N * steps / wall time of the timed steps
  latency_ms     p50 / p99 / mean host-side latency per update (launch -> u_0 on host)
  roofline       the rollout kernel (dominant): algorithmic FP32 FLOP per launch over
                 its average duration, measured with HIP events on its stream
  reduction      weighted-sum kernel: algorithmic bytes over its duration (HBM)
  cpu_baseline   the FP64 oracle on the host cores, on a bounded sample
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout-steps/s + p50/p99 MPPI update latency, batched/served vs plain, 1 GPU"
PEAK_FP32_VECTOR = 157.3e12     # MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_UNPACKED = 78.6e12    # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz (no packed FP32)
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic work per unit (counted from the kernels' formulation; FMA = 2 FLOP,
# each transcendental (log2, sqrt, sin, cos, rsqrt) = 1 FLOP)
# ---------------------------------------------------------------------------

FLOP_STEP_BASE = {
    "noise": 22,          # 4 uniforms, 2 x (log, mul, sqrt), 4 x (trig, 2 mul)
    "perturb": 4,         # u = u_nom + du
    "input_cost": 28,     # u^T R u (12) and du^T R_d du (16)
    "controller": 40,     # Eqs. (8)-(12): rates, torques, Gamma^-1, clip
    "rk4": 425,           # stage wrenches 50, 4 x 51 body derivative, 130 stage combinations,
                          # 19 position (sum of stage accelerations), 12 renorm, 8 lag, 2
    "tracking": 44,       # Eq. (18) with Eq. (21)
    "obstacle_epilogue": 2,
    "accumulate": 5,      # Kahan add and the step sum
}
FLOP_PER_OBSTACLE_TEST = 11   # 2 sub, sub + mul (z mask), mul + 2 fma, 2 compares
FLOP_CULL_PER_STATE = 28       # wave x-range (2 x 6 DPP min/max), range bounds, bin lookups
FLOP_INITIAL_STATE = 44 + 2 + 5  # scoring of x_hat itself (tracking, obstacle epilogue, sum)


def flop_per_rollout_step() -> int:
    return sum(FLOP_STEP_BASE.values())


def rollout_flop_per_launch(K: int, N: int, M: int, obstacle_tests: float) -> float:
    """Algorithmic FP32 FLOP of one rollout launch: the per-step formulation count for
    K N sample-steps, the scoring of the initial state, the culling arithmetic when the
    obstacles are culled (16 <= M <= 512), and 11 FLOP per obstacle distance test
    actually performed (measured by the library's counter: obstacles outside a wave's
    reach are skipped and cost nothing)."""
    states = K * (N + 1)
    cull = states * FLOP_CULL_PER_STATE if 16 <= M <= 512 else 0
    return float(K) * N * flop_per_rollout_step() + K * FLOP_INITIAL_STATE + cull + \
        FLOP_PER_OBSTACLE_TEST * obstacle_tests


def reduction_bytes_per_launch(K: int, N: int) -> float:
    # delta_u [N][4][K] read once, costs [K] once, u_nom read and u_upd written
    return 4.0 * (4 * K * N + K + 8 * N)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("model.h", "stages.h", "kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2407_09812_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(K, N, M, launch):
    """HBM bytes per rollout launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source, this workload and this launch shape; else
    None."""
    path = os.path.join(ROOT, "profiles", "rollout_c2_pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("workload") != [K, N, M]
            or rec.get("launch") != launch):
        return None
    return rec.get("hbm_bytes_per_launch")


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host cores (bounded sample)
# ---------------------------------------------------------------------------

def cpu_baseline(sc, seconds: float):
    import numpy as np
    import oracle
    x = sc.x0.copy()
    u_nom = sc.u_nom0()
    n, t0 = 0, time.perf_counter()
    while True:
        r = oracle.update(sc.veh, sc.cost, sc.solve(n), x, u_nom, sc.x_ref(n), sc.obstacles)
        x = oracle.predict(sc.veh, sc.dt, sc.period, x, r["u_apply"][:4])
        u_nom = r["u_nom"]
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:        # the closed loop continues past the bench's update count
            break
    return {"value": sc.K * sc.N * n / el, "unit": "rollout-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} closed-loop FP64 updates of {sc.name} (K={sc.K}, N={sc.N}, M={sc.M}) "
                      f"in {el:.1f} s"}


# ---------------------------------------------------------------------------

def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def run(args):
    import numpy as np
    import torch

    import paper_2407_09812_amd as lib
    import workloads as W

    torch.cuda.set_device(0)
    sc = W.CONFIGS[args.config]()
    K, N, M = sc.K, sc.N, sc.M
    total = args.warmup + args.steps
    log(f"bench: {sc.name} K={K} N={N} M={M} warmup={args.warmup} steps={args.steps}")

    # device-resident inputs
    refs = torch.tensor(np.stack([sc.x_ref(t) for t in range(total)]), dtype=torch.float32,
                        device="cuda")
    obs = lib.obstacles_to_device(sc.obstacles)
    x_buf = [torch.tensor(sc.x0, dtype=torch.float32, device="cuda"),
             torch.empty(17, dtype=torch.float32, device="cuda")]
    u_nom = torch.tensor(sc.u_nom0(), dtype=torch.float32, device="cuda")
    u_apply = torch.empty(8, dtype=torch.float32, device="cuda")
    u_host = torch.empty(8, dtype=torch.float32, pin_memory=True)
    diag = lib.new_diag()
    ctx = lib.Context(0)
    lib.mppi_reserve(ctx, K, N, M)
    stream = torch.cuda.current_stream()
    solves = [sc.solve(t) for t in range(total)]
    if args.launch:
        lib.mppi_set_config(ctx, K, N, M, *(int(v) for v in args.launch.split(",")))
        launch = lib.mppi_get_config(ctx, K, N, M)
    elif args.autotune:
        launch = lib.mppi_autotune(ctx, sc.veh, sc.cost, solves[0], x_buf[0], refs[0], obs, M, u_nom,
                                   reps=8, stream=stream)
    else:
        launch = lib.mppi_get_config(ctx, K, N, M)
    if args.variant != "auto":                   # force one form of the update
        launch = dict(launch, fused=1 if args.variant in ("fused", "pipe-fused") else 0,
                      pipe=1 if args.variant in ("pipe", "pipe-fused") else 0)
        if launch["pipe"]:
            launch["block"] = 64
        lib.mppi_set_config(ctx, K, N, M, **launch)
    log(f"bench: rollout launch shape {launch}")

    lat = []
    # the per-step inputs in their C layout, built before the loop as a controller would,
    # and each step's update marshalled once (lib.prepare_update): the buffers are the
    # same device memory a C controller would pass by pointer
    veh_c, cost_c = lib.vehicle(sc.veh), lib.cost(sc.cost)
    solves_c = [lib.solve(s) for s in solves]
    updates = [lib.prepare_update(ctx, veh_c, cost_c, solves_c[t], x_buf[t % 2], refs[t], obs, M,
                                  u_nom, u_host, diag, stream=stream) for t in range(total)]
    # the command is written by the device straight into pinned host memory, and the
    # host spins on an event for it (no copy queued, no sleeping wait)
    done = torch.cuda.Event()

    def step(t, record):
        xi = x_buf[t % 2]
        t0 = time.perf_counter()
        updates[t]()
        done.record(stream)
        # the simulated plant (one control period with the command held) is queued
        # behind the update on the device; the controller waits for its command only
        lib.mppi_predict(ctx, veh_c, sc.dt, sc.period, xi, u_host, x_buf[(t + 1) % 2],
                         stream=stream)
        while not done.query():
            pass
        t1 = time.perf_counter()
        if record:
            lat.append((t1 - t0) * 1e3)

    for t in range(args.warmup):
        step(t, False)
    torch.cuda.synchronize()
    lib.mppi_profile_enable(ctx, True)
    lib.mppi_profile_read(ctx)                   # reset
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(args.warmup, total):
        step(t, True)
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof = lib.mppi_profile_read(ctx)
    lib.mppi_profile_enable(ctx, False)
    d = lib.diag_from_tensor(diag)
    final_x = x_buf[total % 2].cpu().numpy()
    log(f"bench: final diag {d}, final position {final_x[:3]}")
    if d["status"] != 0:
        raise RuntimeError(f"update failed on device: {d}")

    elapsed = t_end - t_start
    steps = args.steps
    value = K * N * steps / elapsed
    n_upd = max(1, prof["updates"])
    rollout_ms = prof["rollout_ms"] / n_upd
    sum_ms = prof["sum_ms"] / n_upd
    tests = prof["obstacle_tests"] / n_upd
    flop = rollout_flop_per_launch(K, N, M, tests)
    achieved = flop / (rollout_ms * 1e-3)
    rbytes = reduction_bytes_per_launch(K, N)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "rollout-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.name}: single vehicle, K={K}, N={N}, dt={sc.dt}, M={M}, "
                               f"lambda={sc.lam:g}, update period {sc.period} s, "
                               f"closed loop (plain: one solve per launch sequence)",
                   "K": K, "N": N, "M": M, "updates": steps, "rollout_launch": launch},
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "mean": sum(lat) / len(lat)},
        "device_ms_per_update": {"rollout": rollout_ms, "sum_and_apply": sum_ms},
        "roofline": {
            "kernel": ("rollout_pipe_kernel" if launch.get("pipe") else
                       "rollout_fused_kernel" if launch.get("fused") else "rollout_kernel"),
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "frac_of_unpacked_peak": achieved / PEAK_FP32_UNPACKED,
            "flop_per_launch": flop,
            "obstacle_tests_per_state": tests / (K * (N + 1)),
            "traffic": measured_traffic(K, N, M, launch),
        },
        "reduction": ({"kernel": "update_sum_kernel", "bound": "hbm",
                       "achieved": rbytes / (sum_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                       "unit": "GB/s", "frac": rbytes / (sum_ms * 1e-3) / PEAK_HBM,
                       "bytes_per_launch": rbytes}
                      if not launch.get("fused") else
                      {"kernel": "merge_sum_kernel", "bound": "latency",
                       "note": "single pass: delta_u is regenerated in the rollout launch, not "
                               "stored; this launch sums the per-wave partials"}),
    }
    ctx.close()
    if args.cpu_seconds > 0:
        log(f"bench: timing the FP64 oracle for about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_seconds)
    return out


def calibrate_copy(mib: int, reps: int):
    """A plain device-to-device copy of known size, run under the same HBM counters as
    the kernels so that FETCH_SIZE / WRITE_SIZE can be scaled to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    flush = torch.zeros(128 << 20, device="cuda")     # 512 MiB written after the source
    flush.add_(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    return {"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps,
            "GBps_read_plus_write": 8 * n / el / 1e9}


def summarize_rocpd(db_path: str, command: str) -> str:
    """Markdown table of per-kernel calls / total / average duration from a rocprofv3
    rocpd database (kernel trace)."""
    import sqlite3
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage "
                      "from top_kernels").fetchall()
    out = [f"Command:\n\n    {command}\n", "| kernel | calls | total (us) | average (us) | % |",
           "|---|---:|---:|---:|---:|"]
    for name, calls, total, avg, pct in rows:
        out.append(f"| `{name.split('(')[0]}` | {calls} | {total:.1f} | {avg:.3f} | {pct:.1f} |")
    return "\n".join(out) + "\n"


def run_batched(args, steps: int, warmup: int, plain_steps: int):
    """The batched configuration: 256 vehicles with uneven K, N and obstacle counts, one
    batched update (persistent kernel, HIP graph) per step, against the same updates
    issued as 256 sequential one-instance launch sequences."""
    import numpy as np
    import torch

    import paper_2407_09812_amd as lib
    import workloads as W

    fleet = W.c4_batch()
    total = warmup + steps
    ctx = lib.Context(0)
    lib.mppi_reserve(ctx, max(sc.K for sc in fleet), max(sc.N for sc in fleet),
                     max(sc.M for sc in fleet))
    dev = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    insts = []
    for sc in fleet:
        insts.append(dict(sc=sc, x_hat=dev(sc.x0), x_ref=dev(sc.x_ref(0)),
                          obs=lib.obstacles_to_device(sc.obstacles), u0=dev(sc.u_nom0()),
                          u_apply=torch.empty(8, device="cuda"),
                          diag=lib.new_diag()))
    for it in insts:
        it["u_nom"] = it["u0"].clone()

    def requests(t):
        return lib.make_requests([dict(veh=it["sc"].veh, cost=it["sc"].cost, solve=it["sc"].solve(t),
                                       x_hat=it["x_hat"], x_ref=it["x_ref"], obs=it["obs"],
                                       M=it["sc"].M, u_nom=it["u_nom"], u_apply=it["u_apply"],
                                       diag=it["diag"]) for it in insts])

    reqs = [requests(t) for t in range(total)]
    lib.mppi_batch_reserve(ctx, reqs[0])
    cfg = lib.mppi_batch_autotune(ctx, reqs[0], reps=1) if args.autotune else \
        lib.mppi_batch_get_config(ctx)
    log(f"bench: batched launch shape {cfg}")
    steps_per_batch = sum(sc.K * sc.N for sc in fleet)
    stream = torch.cuda.current_stream()

    for t in range(warmup):
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
    torch.cuda.synchronize()
    lat = []
    t_start = time.perf_counter()
    for t in range(warmup, total):
        t0 = time.perf_counter()
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    t_end = time.perf_counter()
    batched = steps_per_batch * steps / (t_end - t_start)

    # kernel time of the rollout stage: a profiled pass (events around the stage)
    lib.mppi_profile_enable(ctx, True)
    lib.mppi_profile_read(ctx)
    for t in range(min(steps, 5)):
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
    torch.cuda.synchronize()
    prof = lib.mppi_profile_read(ctx)
    lib.mppi_profile_enable(ctx, False)
    n_b = max(1, prof["batches"])
    rollout_ms = prof["batch_rollout_ms"] / n_b
    rest_ms = prof["batch_rest_ms"] / n_b
    tests = prof["obstacle_tests"] / n_b
    flop_per_batch = sum(rollout_flop_per_launch(sc.K, sc.N, sc.M, 0.0) for sc in fleet) + \
        FLOP_PER_OBSTACLE_TEST * tests
    dense_tests = sum(sc.K * (sc.N + 1) * sc.M for sc in fleet)
    du_bytes = sum(reduction_bytes_per_launch(sc.K, sc.N) for sc in fleet)

    # the same updates as sequential one-instance launch sequences
    for it in insts:
        it["u_nom"].copy_(it["u0"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(plain_steps):
        for it in insts:
            sc = it["sc"]
            lib.mppi_update(ctx, sc.veh, sc.cost, sc.solve(t), it["x_hat"], it["x_ref"], it["obs"],
                            sc.M, it["u_nom"], it["u_apply"], it["diag"], stream=stream)
        stream.synchronize()
    plain = steps_per_batch * plain_steps / (time.perf_counter() - t0)
    statuses = [lib.diag_from_tensor(it["diag"])["status"] for it in insts]
    ctx.close()
    if any(s != 0 for s in statuses):
        raise RuntimeError(f"batched updates failed on device: {statuses}")
    achieved = flop_per_batch / (rollout_ms * 1e-3)
    return {
        "workload": f"c4_batch: {len(fleet)} vehicles, K in {{1024..16384}}, N in [50, 200], "
                    f"0-200 spheres; one persistent hipGraph launch per batch",
        "rollout_steps_per_batch": steps_per_batch,
        "value": batched, "unit": "rollout-steps/s", "steps": steps,
        "ms_per_batch": (t_end - t_start) / steps * 1e3,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "plain_sequential": {"value": plain, "unit": "rollout-steps/s", "steps": plain_steps},
        "speedup_vs_plain": batched / plain,
        "launch": cfg,
        "device_ms_per_batch": {"rollout": rollout_ms, "weights_sum_apply": rest_ms},
        "roofline": {"kernel": "batch_rollout_kernel", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
                     "frac_of_unpacked_peak": achieved / PEAK_FP32_UNPACKED,
                     "flop_per_launch": flop_per_batch,
                     "obstacle_tests_per_batch": tests,
                     "obstacle_tests_fraction_of_dense": tests / max(1, dense_tests)},
        "reduction_stages": {"bytes_per_batch": du_bytes,
                             "achieved": du_bytes / (rest_ms * 1e-3) / 1e9, "unit": "GB/s",
                             "note": "weights + weighted sum + apply, bytes of the weighted sum"},
    }


def run_served(args, duration_s: float, rate_hz: float, batch_cfg=None):
    """The serving configuration: Poisson arrivals from 512 vehicles, each request with
    its own K and N, admitted by memory budget and batched continuously by the
    library's server; latency runs from submit to the result on the host."""
    import numpy as np

    import paper_2407_09812_amd as lib
    import workloads as W

    fleet, arrivals = W.c5_arrivals(rate_hz=rate_hz, duration_s=duration_s)
    dt = fleet[0].dt
    window = 200                                  # reference rows are reused cyclically
    rows = [sc.ref.rows(0.0, window + 200, dt).astype(np.float32) for sc in fleet]
    thrust = [np.float32(sc.ref.thrust(0.0, sc.veh["mass"]) / 4.0) for sc in fleet]
    obs = [lib.obstacles_host(sc.obstacles) for sc in fleet]
    veh, cost = fleet[0].veh, fleet[0].cost
    srv = lib.Server(veh, cost, W.hover_control(veh), n_vehicles=len(fleet), K_max=16384, N_max=200,
                     M_max=200, n_streams=args.serve_streams, max_batch=64,
                     budget_bytes=int(args.serve_budget_gib * (1 << 30)))
    if batch_cfg:
        srv.set_batch_config(batch_cfg["block"], batch_cfg["lanes"], batch_cfg["unroll"],
                             batch_cfg["blocks_per_cu"])
    count = [0] * len(fleet)
    rng = np.random.default_rng(5)

    def submit(vid, K, N):
        i = count[vid] % window
        count[vid] += 1
        x = np.empty(17, dtype=np.float32)
        x[:13] = rows[vid][i]
        x[13:] = thrust[vid]
        x[:3] += rng.normal(0.0, 0.05, 3).astype(np.float32)
        return srv.submit(vid, K, N, dt, 1.0, (1.0, 1.0, 1.0, 1.0), 5, x, rows[vid][i:i + N + 1],
                          obs[vid], delay=args.serve_delay)

    for vid in range(8):                          # warm-up: graph capture on every slot
        srv.wait(submit(vid, 1024, 50))
    srv.drain()
    tickets = []
    t_start = time.perf_counter()
    for (ta, vid, K, N) in arrivals:
        while True:
            lag = ta - (time.perf_counter() - t_start)
            if lag <= 0.0:
                break
            if lag > 0.002:
                time.sleep(lag - 0.001)
        tickets.append(submit(vid, K, N))
    late = (time.perf_counter() - t_start) - arrivals[-1][0]
    srv.drain()
    t_end = time.perf_counter()
    res = [srv.poll(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    lat = [1e3 * r["latency_s"] for r in res]
    delays = [1e3 * r["delay"] for r in res]
    bad = sum(1 for r in res if r["status"] != 0)
    steps = sum(r["K"] * r["N"] for r in res)
    return {
        "workload": f"c5_serve: Poisson {rate_hz:.0f} req/s from {len(fleet)} vehicles for "
                    f"{duration_s:.0f} s, K in {{1024..16384}}, N in [50, 200], 0-200 spheres",
        "requests": len(res), "failed": bad,
        "value": steps / (t_end - t_start), "unit": "rollout-steps/s",
        "offered_rollout_steps_per_s": steps / arrivals[-1][0],
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "mean": sum(lat) / len(lat), "max": max(lat)},
        "batches": stats["batches"], "mean_batch": stats["completed"] / max(1, stats["batches"]),
        "max_in_flight": stats["max_in_flight"], "device_busy_frac": stats["busy_s"] / (t_end - t_start),
        "streams": args.serve_streams, "budget_gib": args.serve_budget_gib,
        "submit_lag_s": late,
        "delay_compensation_ms": {"requested": args.serve_delay * 1e3 if args.serve_delay >= 0
                                  else "median served latency",
                                  "mean_used": sum(delays) / len(delays), "max_used": max(delays)},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "paper"])
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the served leg beside the plain line (0 skips it); "
                         "--config c5 runs the full 60 s")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--serve-delay", type=float, default=-1.0,
                    help="seconds each served state estimate is predicted forward before its "
                         "update; < 0: the server's running median latency (default)")
    ap.add_argument("--batched-steps", type=int, default=20,
                    help="batched updates of the 256-vehicle mix timed beside the plain line "
                         "(0 skips the batched leg)")
    ap.add_argument("--launch", default="", metavar="BLOCK,LANES,UNROLL,FUSED[,PIPE]",
                    help="fixed launch shape of the single-vehicle leg instead of autotuning "
                         "(profiling runs use it so that every pass runs the same kernels)")
    ap.add_argument("--variant", default="auto",
                    choices=["auto", "stored", "fused", "pipe", "pipe-fused"],
                    help="update variant of the single-vehicle leg: the autotuner's choice, "
                         "stored delta_u + weighted sum, the single pass, or the wave-specialised "
                         "rollouts with either")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="use the library's default rollout launch shape")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle CPU-baseline time budget (0 skips it)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit; "
                         "use a size well above the 256 MB MALL")
    ap.add_argument("--summarize-rocpd", nargs=2, metavar=("DB", "COMMAND"),
                    help="print a Markdown kernel summary of a rocprofv3 database and exit")
    args = ap.parse_args()
    if args.summarize_rocpd:
        sys.stdout.write(summarize_rocpd(*args.summarize_rocpd))
        return
    if args.calibrate_copy > 0:
        print(json.dumps(calibrate_copy(args.calibrate_copy, 5)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the MPPI update of one vehicle runs on one device; see the design notes "
              "on sharding vehicles or samples over several GPUs).", file=sys.stderr)
        sys.exit(2)
    if args.config == "c5":
        sv = run_served(args, 60.0, args.serve_rate)
        out = {"metric": METRIC, "value": sv["value"], "unit": "rollout-steps/s", "n_gpus": 1,
               "steps": sv["requests"], "warmup": 8, "ms_per_step": sv["latency_ms"]["mean"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic", "config": {"workload": sv["workload"]}, "served": sv}
        print(json.dumps(out), flush=True)
        return
    if args.config == "c4":
        b = run_batched(args, args.steps, args.warmup, plain_steps=2)
        out = {"metric": METRIC, "value": b["value"], "unit": "rollout-steps/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["ms_per_batch"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic", "config": {"workload": b["workload"]},
               "roofline": b["roofline"], "batched": b}
    else:
        out = run(args)
        if args.batched_steps > 0:
            out["batched"] = run_batched(args, args.batched_steps, 3, plain_steps=2)
        if args.serve_seconds > 0:
            out["served"] = run_served(args, args.serve_seconds, args.serve_rate,
                                       out.get("batched", {}).get("launch"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
