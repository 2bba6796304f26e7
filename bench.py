#!/usr/bin/env python3
"""Benchmark of the MPPI update on one MI355X.

Headline (the default run's top-level value): the batched configuration -- 256
vehicles with uneven K in {1024, ..., 16384}, N in [50, 200] and 0-200 spheres, one
batched update of all of them per step (persistent rollout kernel, HIP graph replay,
the library's default launch shapes, which its autotuners pick for these workloads;
--autotune runs them), the steps enqueued back to back (the host
plans the next batch while one runs), against the same 256 updates issued as
sequential one-instance launch sequences ("plain"); the latency percentiles come from a
second pass with one synchronisation per batch.  The driver's --steps / --warmup apply
to it.  Inputs are resident on the device before the timed region.

The same JSON line carries, each with its own roofline:
  plain.c2_line, plain.c3_agile  single-vehicle closed loops (K = 4096, N = 100,
                 20 spheres; K = 16384, N = 200, 200 cylinders): each step is one
                 full update whose command the device writes into pinned host memory,
                 one noise-free plant step queued behind it, and the host spinning on
                 an event for the command before the next update
  served         the served configuration: Poisson arrivals at 2000 requests/s from
                 512 vehicles for 60 s, admitted by memory budget and batched
                 continuously by the library's server, each state estimate predicted
                 over the running median latency
  serving_capacity  the same server at higher arrival rates, until it saturates
  cpu_baseline   the FP64 oracle on the host cores on a bounded sample of the batched
                 workload, single-threaded and on all cores, extrapolated

--config c1 | c2 | c3 | paper runs one single-vehicle closed loop, c4 only the batched
leg, c5 only the served leg; --launch / --batch-launch pin the launch shapes (profiling
runs use them, so that every dispatch of a kernel has one shape).

Work counts (rooflines): the FP32 operations per rollout are frozen from an
operation-counting run of the FP64 oracle (oracle/flop_count.cpp): 41 per rollout,
984 per rollout-step (9 of them transcendental) and, per state and obstacle, 11 for a
sphere and 9 for a vertical cylinder -- the method's dense work; the kernels skip the
obstacles culling proves out of reach, so they execute fewer.  The weighted sum
reads delta_u (16 K N bytes), the costs (4 K) and the warm start, writes the update.
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
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic work, frozen from the oracle's operation count (oracle/flop_count.py
# derives these from a counting run; a CPU test checks that they still agree)
# ---------------------------------------------------------------------------

FLOP_PER_ROLLOUT = 41            # the initial state's tracking cost and obstacle epilogue
FLOP_PER_STEP = 984              # noise, perturbation, controller, RK4, renormalisation,
                                 # input and input-change cost, tracking cost (9 transcendental)
FLOP_PER_TEST = {0: 11, 1: 9}    # per state and obstacle: sphere, vertical cylinder
DENSE_NOTE = ("algorithmic: the FP64 oracle's operation count (984 per rollout-step, 11 per "
              "sphere and 9 per cylinder test at every state), dense; the kernel skips the "
              "obstacle tests culling proves zero and computes the step in fewer operations, so "
              "it executes fewer (rocprofv3 FP32 lane-op counters in profiles/: 'executed'); "
              "a frac above 1 is the dense work the culling saves, not a rate the VALU ran at")


def rollout_flop(K: int, N: int, obstacle_types) -> float:
    """Algorithmic FP32 operations of K rollouts of N steps with the given obstacles
    (dense: every obstacle tested at every state)."""
    per_state = sum(FLOP_PER_TEST[int(t)] for t in obstacle_types)
    return float(K) * (FLOP_PER_ROLLOUT + FLOP_PER_STEP * N + (N + 1) * per_state)


def reduction_bytes(K: int, N: int) -> float:
    """The weighted sum's algorithmic HBM bytes: delta_u [N][4][K] and the costs read
    once, the warm start read and the update written."""
    return 4.0 * (4 * K * N + K + 8 * N)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("model.h", "stages.h", "kernels.hip", "kernels.h", "batch.hip", "batch.h"):
        with open(os.path.join(ROOT, "paper_2407_09812_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(kernel: str, workload: str) -> dict:
    """The committed rocprofv3 counter record of `kernel` on `workload`
    (profiles/hbm_traffic.json), if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh)
    for rec in recs.get("records", []):
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("kernel_source_hash") == kernel_source_hash()):
            return rec
    return None


def counter_fields(kernel: str, workload: str, duration_s: float) -> dict:
    """roofline fields from the committed counters: HBM traffic per launch (FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy) and the FP32 operations the kernel executed
    (SQ_INSTS_VALU_FLOPS_FP32), as a rate over the duration measured here; null when the
    kernel has changed since the counters were taken."""
    rec = profile_record(kernel, workload)
    if rec is None:
        return {"traffic": None, "executed": None}
    flop = rec["valu_flops_fp32_per_launch"]
    return {"traffic": rec["hbm_bytes_per_launch"],
            "executed": {"flop_per_launch": flop, "achieved": flop / duration_s / 1e12,
                         "unit": "TFLOP/s", "frac": flop / duration_s / PEAK_FP32_VECTOR,
                         "counters_launch": rec["launch"], "source": rec["summary"]}}


def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    i = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[i]


def parse_launch(text):
    return [int(v) for v in text.split(",")] if text else None


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle (as it stands) on the host cores, bounded samples
# ---------------------------------------------------------------------------

def _oracle_rate(instances, k_sample, seconds, threads):
    """Time the oracle's full update (rollouts, weights, update, apply) of the first
    k_sample samples of each instance, repeated until `seconds` have passed; returns
    (work units per second, rollout-steps per second, passes, elapsed)."""
    import oracle
    oracle.set_num_threads(threads)
    work = steps = 0.0
    passes, t0 = 0, time.perf_counter()
    while True:
        for sc in instances:
            s = dict(sc.solve(0), K=min(k_sample, sc.K))
            oracle.update(sc.veh, sc.cost, s, sc.x0, sc.u_nom0(), sc.x_ref(0), sc.obstacles)
            work += rollout_flop(s["K"], sc.N, sc.obstacles[:, 0])
            steps += s["K"] * sc.N
        passes += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            return work / el, steps / el, passes, el


def cpu_baseline_batch(fleet, seconds_single: float, seconds_all: float):
    """The batched workload on the oracle: 10 of its instances (every 25th vehicle),
    each with its first 256 samples, timed single-threaded and on all host cores, and
    extrapolated to the whole batch in the algorithmic work (rollouts are independent,
    so time grows with K N (984 + 11 M) as the work count does)."""
    import oracle
    all_threads = oracle.num_threads()
    sample = fleet[::25][:10]
    k_sample = 256
    full_work = sum(rollout_flop(sc.K, sc.N, sc.obstacles[:, 0]) for sc in fleet)
    full_steps = sum(sc.K * sc.N for sc in fleet)
    desc = (f"FP64 oracle updates of vehicles {[sc.vehicle_id for sc in sample]} of the batch "
            f"(N {[sc.N for sc in sample]}, M {[sc.M for sc in sample]}), the first {k_sample} "
            f"samples each; extrapolated to the 256-vehicle batch ({full_steps:.3g} rollout-steps, "
            f"{full_work:.3g} FLOP) in the algorithmic work")
    out = {}
    for name, threads, secs in (("single_thread", 1, seconds_single),
                                ("all_cores", all_threads, seconds_all)):
        w_rate, s_rate, passes, el = _oracle_rate(sample, k_sample, secs, threads)
        batch_s = full_work / w_rate
        out[name] = {"value": full_steps / batch_s, "unit": "rollout-steps/s", "cores": threads,
                     "extrapolated_s_per_batch": batch_s, "measured_s": el, "passes": passes,
                     "measured_rollout_steps_per_s": s_rate}
    oracle.set_num_threads(all_threads)
    return {"value": out["all_cores"]["value"], "unit": "rollout-steps/s",
            "cores": all_threads, "kind": "oracle", "extrapolated": True, "sample": desc,
            **out}


def cpu_baseline_plain(sc, seconds: float):
    """One single-vehicle workload's closed loop on the oracle, all host cores."""
    import oracle
    x, u_nom = sc.x0.copy(), sc.u_nom0()
    n, t0 = 0, time.perf_counter()
    while True:
        r = oracle.update(sc.veh, sc.cost, sc.solve(n), x, u_nom, sc.x_ref(n), sc.obstacles)
        x = oracle.predict(sc.veh, sc.dt, sc.period, x, r["u_apply"][:4])
        u_nom = r["u_nom"]
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": sc.K * sc.N * n / el, "unit": "rollout-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{n} closed-loop FP64 updates of {sc.name} (K={sc.K}, N={sc.N}, M={sc.M}) "
                      f"in {el:.1f} s"}


# ---------------------------------------------------------------------------
# Single-vehicle closed loop ("plain": one solve per launch sequence)
# ---------------------------------------------------------------------------

def run_plain(args, config: str, steps: int, warmup: int, launch_text: str = "",
              cpu_seconds: float = 0.0):
    import numpy as np
    import torch

    import paper_2407_09812_amd as lib
    import workloads as W

    torch.cuda.set_device(0)
    sc = W.CONFIGS[config]()
    K, N, M = sc.K, sc.N, sc.M
    total = warmup + steps
    log(f"bench: {sc.name} K={K} N={N} M={M} warmup={warmup} steps={steps}")
    refs = torch.tensor(np.stack([sc.x_ref(t) for t in range(total)]), dtype=torch.float32,
                        device="cuda")
    obs = lib.obstacles_to_device(sc.obstacles)
    x_buf = [torch.tensor(sc.x0, dtype=torch.float32, device="cuda"),
             torch.empty(17, dtype=torch.float32, device="cuda")]
    u_nom = torch.tensor(sc.u_nom0(), dtype=torch.float32, device="cuda")
    u_host = torch.empty(8, dtype=torch.float32, pin_memory=True)
    diag = lib.new_diag()
    ctx = lib.Context(0)
    lib.mppi_reserve(ctx, K, N, M)
    stream = torch.cuda.current_stream()
    solves = [sc.solve(t) for t in range(total)]
    fixed = parse_launch(launch_text)
    if fixed:
        lib.mppi_set_config(ctx, K, N, M, *fixed)
        launch = lib.mppi_get_config(ctx, K, N, M)
    elif args.autotune:
        launch = lib.mppi_autotune(ctx, sc.veh, sc.cost, solves[0], x_buf[0], refs[0], obs, M, u_nom,
                                   reps=8, stream=stream)
    else:
        launch = lib.mppi_get_config(ctx, K, N, M)
    log(f"bench: {sc.name} rollout launch shape {launch}")

    # per-step inputs in their C layout, built before the loop as a controller would,
    # and each step's update marshalled once (the pointers a C controller would pass)
    veh_c, cost_c = lib.vehicle(sc.veh), lib.cost(sc.cost)
    updates = [lib.prepare_update(ctx, veh_c, cost_c, lib.solve(solves[t]), x_buf[t % 2], refs[t],
                                  obs, M, u_nom, u_host, diag, stream=stream) for t in range(total)]
    done = torch.cuda.Event()
    lat = []

    def step(t, record):
        t0 = time.perf_counter()
        updates[t]()
        done.record(stream)
        # the plant (one control period with the command held) is queued behind the
        # update; the controller waits for its command only
        lib.mppi_predict(ctx, veh_c, sc.dt, sc.period, x_buf[t % 2], u_host, x_buf[(t + 1) % 2],
                         stream=stream)
        while not done.query():
            pass
        if record:
            lat.append((time.perf_counter() - t0) * 1e3)

    for t in range(warmup):
        step(t, False)
    torch.cuda.synchronize()
    lib.mppi_profile_enable(ctx, True)
    lib.mppi_profile_read(ctx)                   # reset
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for t in range(warmup, total):
        step(t, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = lib.mppi_profile_read(ctx)
    lib.mppi_profile_enable(ctx, False)
    d = lib.diag_from_tensor(diag)
    ctx.close()
    if d["status"] != 0:
        raise RuntimeError(f"update failed on device: {d}")

    n_upd = max(1, prof["updates"])
    rollout_ms = prof["rollout_ms"] / n_upd
    sum_ms = prof["sum_ms"] / n_upd
    tests = prof["obstacle_tests"] / n_upd
    flop = rollout_flop(K, N, sc.obstacles[:, 0])
    achieved = flop / (rollout_ms * 1e-3)
    rbytes = reduction_bytes(K, N)
    kernel = ("rollout_pipe_kernel" if launch.get("pipe") else
              "rollout_fused_kernel" if launch.get("fused") else "rollout_kernel")
    rec = {
        "workload": f"{sc.name}: single vehicle, K={K}, N={N}, dt={sc.dt}, M={M}, "
                    f"lambda={sc.lam:g}, update period {sc.period} s, closed loop "
                    f"(plain: one solve per launch sequence)",
        "value": K * N * steps / elapsed, "unit": "rollout-steps/s",
        "steps": steps, "warmup": warmup, "ms_per_step": elapsed / steps * 1e3,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "mean": sum(lat) / len(lat)},
        "launch": launch,
        "device_ms_per_update": {"rollout": rollout_ms, "sum_and_apply": sum_ms},
        "roofline": {
            "kernel": kernel, "bound": "alu", "achieved": achieved / 1e12,
            "peak": PEAK_FP32_VECTOR / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "flop_per_launch": flop,
            "flop_count": DENSE_NOTE,
            "obstacle_tests_per_state": tests / (K * (N + 1)),
            "obstacle_tests_fraction_of_dense": tests / max(1, K * (N + 1) * M),
            **counter_fields(kernel, sc.name, rollout_ms * 1e-3),
        },
        "reduction": ({"kernel": "update_sum_kernel", "bound": "hbm",
                       "achieved": rbytes / (sum_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                       "unit": "GB/s", "frac": rbytes / (sum_ms * 1e-3) / PEAK_HBM,
                       "bytes_per_launch": rbytes,
                       "note": "the sum launch's duration also holds the weight statistics "
                               "reduction and the apply and shift"}
                      if not launch.get("fused") else
                      {"kernel": "merge_sum_kernel", "bound": "latency",
                       "note": "single pass: delta_u is regenerated, not stored"}),
    }
    if cpu_seconds > 0:
        log(f"bench: timing the FP64 oracle on {sc.name} for about {cpu_seconds:.0f} s")
        rec["cpu_baseline"] = cpu_baseline_plain(sc, cpu_seconds)
    return rec


# ---------------------------------------------------------------------------
# Batched: 256 uneven vehicles per step
# ---------------------------------------------------------------------------

def run_batched(args, steps: int, warmup: int, plain_rounds: int):
    import numpy as np
    import torch

    import paper_2407_09812_amd as lib
    import workloads as W

    torch.cuda.set_device(0)
    fleet = W.c4_batch()
    total = warmup + steps
    ctx = lib.Context(0)
    lib.mppi_reserve(ctx, max(sc.K for sc in fleet), max(sc.N for sc in fleet),
                     max(sc.M for sc in fleet))
    dev = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device="cuda")
    insts = [dict(sc=sc, x_hat=dev(sc.x0), x_ref=dev(sc.x_ref(0)),
                  obs=lib.obstacles_to_device(sc.obstacles), u0=dev(sc.u_nom0()),
                  u_apply=torch.empty(8, device="cuda"), diag=lib.new_diag()) for sc in fleet]
    for it in insts:
        it["u_nom"] = it["u0"].clone()

    def requests(t):
        return lib.make_requests([dict(veh=it["sc"].veh, cost=it["sc"].cost, solve=it["sc"].solve(t),
                                       x_hat=it["x_hat"], x_ref=it["x_ref"], obs=it["obs"],
                                       M=it["sc"].M, u_nom=it["u_nom"], u_apply=it["u_apply"],
                                       diag=it["diag"]) for it in insts])

    reqs = [requests(t) for t in range(total)]
    lib.mppi_batch_reserve(ctx, reqs[0])
    stream = torch.cuda.current_stream()
    fixed = parse_launch(args.batch_launch)
    if fixed:
        lib.mppi_batch_set_config(ctx, *fixed)
        cfg = lib.mppi_batch_get_config(ctx)
    elif args.autotune:
        cfg = lib.mppi_batch_autotune(ctx, reqs[0], reps=1, stream=stream)
    else:
        cfg = lib.mppi_batch_get_config(ctx)
    log(f"bench: batched launch shape {cfg}")
    steps_per_batch = sum(sc.K * sc.N for sc in fleet)

    for t in range(warmup):
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
    torch.cuda.synchronize()
    # throughput: the batched updates enqueued back to back (the library plans batch
    # t + 1 on the host while batch t runs; each waits for the previous one's warm starts
    # on the stream), one synchronisation at the end
    t_start = time.perf_counter()
    for t in range(warmup, total):
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
    stream.synchronize()
    elapsed = time.perf_counter() - t_start
    batched = steps_per_batch * steps / elapsed
    # latency: the same batched updates one at a time, from the call to the results on
    # the device (synchronised)
    lat = []
    for t in range(warmup, total):
        t0 = time.perf_counter()
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)

    # the rollout kernel's duration: profiled batches (HIP events around the stage)
    lib.mppi_profile_enable(ctx, True)
    lib.mppi_profile_read(ctx)
    for t in range(min(steps, 10)):
        lib.mppi_batch_update(ctx, reqs[t], stream=stream)
    torch.cuda.synchronize()
    prof = lib.mppi_profile_read(ctx)
    lib.mppi_profile_enable(ctx, False)
    n_b = max(1, prof["batches"])
    rollout_ms = prof["batch_rollout_ms"] / n_b
    rest_ms = prof["batch_rest_ms"] / n_b
    tests = prof["obstacle_tests"] / n_b
    flop = sum(rollout_flop(sc.K, sc.N, sc.obstacles[:, 0]) for sc in fleet)
    dense_tests = sum(sc.K * (sc.N + 1) * sc.M for sc in fleet)
    rbytes = sum(reduction_bytes(sc.K, sc.N) for sc in fleet)

    # the same updates as sequential one-instance launch sequences (the library's
    # default single-instance shape), one host synchronisation per round of 256
    plain = plain_s = None
    if plain_rounds > 0:
        for it in insts:
            it["u_nom"].copy_(it["u0"])
        torch.cuda.synchronize()
        for it in insts:                               # warm-up round
            sc = it["sc"]
            lib.mppi_update(ctx, sc.veh, sc.cost, sc.solve(0), it["x_hat"], it["x_ref"], it["obs"],
                            sc.M, it["u_nom"], it["u_apply"], it["diag"], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(plain_rounds):
            for it in insts:
                sc = it["sc"]
                lib.mppi_update(ctx, sc.veh, sc.cost, sc.solve(t), it["x_hat"], it["x_ref"],
                                it["obs"], sc.M, it["u_nom"], it["u_apply"], it["diag"],
                                stream=stream)
            stream.synchronize()
        plain_s = (time.perf_counter() - t0) / plain_rounds
        plain = steps_per_batch / plain_s
    statuses = [lib.diag_from_tensor(it["diag"])["status"] for it in insts]
    ctx.close()
    if any(s != 0 for s in statuses):
        raise RuntimeError(f"batched updates failed on device: {statuses}")
    achieved = flop / (rollout_ms * 1e-3)
    workload = "c4_batch"
    return {
        "workload": f"{workload}: {len(fleet)} vehicles, K in {{1024..16384}}, N in [50, 200], "
                    f"0-200 spheres; one persistent hipGraph launch per batched update",
        "fleet": fleet,
        "rollout_steps_per_batch": steps_per_batch,
        "value": batched, "unit": "rollout-steps/s", "steps": steps, "warmup": warmup,
        "ms_per_batch": elapsed / steps * 1e3,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "mean": sum(lat) / len(lat)},
        "plain_sequential": {"value": plain, "unit": "rollout-steps/s", "rounds": plain_rounds,
                             "ms_per_round": plain_s * 1e3 if plain_s else None,
                             "note": "the same 256 updates as one-instance launch sequences "
                                     "(mppi_update, default shape), one host wait per round"},
        "speedup_vs_plain": batched / plain if plain else None,
        "launch": cfg,
        "device_ms_per_batch": {"rollout": rollout_ms, "stats_sum_apply": rest_ms},
        "roofline": {"kernel": "batch_rollout_kernel", "bound": "alu",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32_VECTOR / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR,
                     "flop_per_launch": flop, "flop_count": DENSE_NOTE,
                     "obstacle_tests_fraction_of_dense": tests / max(1, dense_tests),
                     **counter_fields("batch_rollout_kernel", workload, rollout_ms * 1e-3)},
        "reduction": {"kernels": "batch_stats_kernel + batch_wsum_kernel + batch_apply_kernel",
                      "bound": "hbm", "bytes_per_launch": rbytes,
                      "achieved": rbytes / (rest_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                      "unit": "GB/s", "frac": rbytes / (rest_ms * 1e-3) / PEAK_HBM},
    }


# ---------------------------------------------------------------------------
# Served: Poisson arrivals, continuous batching
# ---------------------------------------------------------------------------

def run_served(args, duration_s: float, rate_hz: float, batch_cfg=None, n_streams=None):
    """Poisson arrivals from 512 vehicles, each request with its own K and N, admitted by
    memory budget and batched continuously by the library's server; latency runs from
    submit to the result on the host."""
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
    streams = args.serve_streams if n_streams is None else n_streams
    srv = lib.Server(veh, cost, W.hover_control(veh), n_vehicles=len(fleet), K_max=16384, N_max=200,
                     M_max=200, n_streams=streams, max_batch=args.serve_max_batch,
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
    base = srv.stats()
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
    batches = stats["batches"] - base["batches"]
    return {
        "workload": f"c5_serve: Poisson {rate_hz:.0f} req/s from {len(fleet)} vehicles for "
                    f"{duration_s:.0f} s, K in {{1024..16384}}, N in [50, 200], 0-200 spheres",
        "rate_hz": rate_hz, "requests": len(res), "failed": bad,
        "value": steps / (t_end - t_start), "unit": "rollout-steps/s",
        "offered_rollout_steps_per_s": steps / arrivals[-1][0],
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                       "mean": sum(lat) / len(lat), "max": max(lat)},
        "batches": batches, "mean_batch": len(res) / max(1, batches),
        "lone_requests": sum(1 for r in res if r["pipe"]),
        "max_in_flight": stats["max_in_flight"],
        "device_busy_frac": (stats["busy_s"] - base["busy_s"]) / (t_end - t_start),
        "streams": streams, "budget_gib": args.serve_budget_gib,
        "footprint_bytes": {
            "budget": int(args.serve_budget_gib * (1 << 30)),
            "lone_request_reserve": streams * 16 * 200 * 16384,
            "note": "the budget bounds the batched requests' scratch (delta_u) per slot share; "
                    "each slot also reserves delta_u for one K_max x N_max request run alone "
                    "(16 K_max N_max bytes), beyond the budget"},
        "submit_lag_s": late,
        "delay_compensation_ms": {"requested": args.serve_delay * 1e3 if args.serve_delay >= 0
                                  else "median served latency",
                                  "mean_used": sum(delays) / len(delays), "max_used": max(delays)},
    }


def run_capacity(args, batch_cfg):
    """The server under rising arrival rates: served throughput, batch size, latency and
    device busy fraction at each, until the device is busy nearly all the time."""
    out = []
    for rate in [float(r) for r in args.capacity_rates.split(",") if r]:
        rec = run_served(args, args.capacity_seconds, rate, batch_cfg)
        rec.pop("workload")
        log(f"bench: served at {rate:.0f} req/s: {rec['value']:.3g} rollout-steps/s, mean batch "
            f"{rec['mean_batch']:.2f}, busy {rec['device_busy_frac']:.2f}, "
            f"p50 {rec['latency_ms']['p50']:.2f} ms p99 {rec['latency_ms']['p99']:.2f} ms")
        out.append(rec)
        if rec["value"] < 0.8 * rec["offered_rollout_steps_per_s"]:
            break                                  # saturated: the queue grows without bound
    return out


# ---------------------------------------------------------------------------
# Counter calibration and rocprofv3 summaries
# ---------------------------------------------------------------------------

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


# ---------------------------------------------------------------------------

def headline(value, steps, warmup, ms_per_step, workload, extra):
    out = {"metric": METRIC, "value": value, "unit": "rollout-steps/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": workload}}
    out.update(extra)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed batched updates (headline)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="all",
                    choices=["all", "c1", "c2", "c3", "paper", "c4", "c5", "capacity"])
    ap.add_argument("--plain-steps", type=int, default=200,
                    help="closed-loop updates of each single-vehicle leg")
    ap.add_argument("--plain-warmup", type=int, default=20)
    ap.add_argument("--plain-rounds", type=int, default=10,
                    help="rounds of 256 sequential one-instance updates timed against the batch")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served leg (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-max-batch", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=float, default=2.0)
    ap.add_argument("--serve-delay", type=float, default=-1.0,
                    help="seconds each served state estimate is predicted forward before its "
                         "update; < 0: the server's running median latency (default)")
    ap.add_argument("--capacity-rates", default="12000,24000,48000,72000,96000",
                    help="arrival rates (req/s) of the serving-capacity leg ('' skips it)")
    ap.add_argument("--capacity-seconds", type=float, default=4.0)
    ap.add_argument("--launch", default="", metavar="BLOCK,LANES,UNROLL,FUSED,PIPE",
                    help="fixed launch shape of a single-vehicle --config")
    ap.add_argument("--batch-launch", default="", metavar="BLOCK,LANES,UNROLL,BLOCKS_PER_CU",
                    help="fixed batched launch shape")
    ap.add_argument("--autotune", action="store_true",
                    help="time the launch shapes first (mppi_autotune, mppi_batch_autotune) "
                         "instead of the library's defaults; the committed profiles are taken "
                         "at the default shapes")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="oracle CPU-baseline budget per timed mode (0 skips it)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB (counter calibration) and exit")
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
              "(an MPPI update of one vehicle runs on one device; the design notes describe "
              "sharding vehicles or samples over several GPUs).", file=sys.stderr)
        sys.exit(2)

    if args.config in ("c1", "c2", "c3", "paper"):
        p = run_plain(args, args.config, args.steps, args.warmup, args.launch, args.cpu_seconds)
        out = headline(p.pop("value"), args.steps, args.warmup, p["ms_per_step"], p["workload"],
                       {"roofline": p.pop("roofline"), "plain": p})
        if "cpu_baseline" in p:
            out["cpu_baseline"] = p.pop("cpu_baseline")
        print(json.dumps(out), flush=True)
        return
    if args.config == "capacity":
        fixed = parse_launch(args.batch_launch)
        cfg = dict(zip(("block", "lanes", "unroll", "blocks_per_cu"), fixed)) if fixed else None
        caps = run_capacity(args, cfg)
        best = max(caps, key=lambda r: r["value"])
        out = headline(best["value"], best["requests"], 8, best["latency_ms"]["mean"],
                       f"c5_serve capacity sweep: Poisson arrivals at {args.capacity_rates} req/s, "
                       f"{args.capacity_seconds:.0f} s each", {"serving_capacity": caps})
        print(json.dumps(out), flush=True)
        return
    if args.config == "c5":
        sv = run_served(args, args.serve_seconds, args.serve_rate)
        out = headline(sv["value"], sv["requests"], 8, sv["latency_ms"]["mean"], sv["workload"],
                       {"served": sv})
        print(json.dumps(out), flush=True)
        return

    b = run_batched(args, args.steps, args.warmup, args.plain_rounds)
    fleet = b.pop("fleet")
    out = headline(b["value"], args.steps, args.warmup, b["ms_per_batch"], b["workload"],
                   {"roofline": b["roofline"], "latency_ms": b["latency_ms"], "batched": b})
    if args.config == "all":
        out["plain"] = {}
        for name in ("c2", "c3"):
            rec = run_plain(args, name, args.plain_steps, args.plain_warmup, "",
                            args.cpu_seconds / 2 if args.cpu_seconds > 0 else 0.0)
            out["plain"][rec["workload"].split(":")[0]] = rec
        if args.serve_seconds > 0:
            out["served"] = run_served(args, args.serve_seconds, args.serve_rate, b["launch"])
        if args.capacity_rates:
            out["serving_capacity"] = run_capacity(args, b["launch"])
    if args.cpu_seconds > 0:
        log(f"bench: timing the FP64 oracle on the batched workload (single thread, all cores)")
        out["cpu_baseline"] = cpu_baseline_batch(fleet, args.cpu_seconds, args.cpu_seconds / 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
