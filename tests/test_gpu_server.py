"""Serving: continuous batching of MPPI updates for many vehicles.

Bars: every served result (applied control, diagnostics, final warm starts) is bit-
identical to the same vehicle's updates run alone, in order, with mppi_update in the
shape the server used (a lone request: the default, wave-specialised; in a batch: the
one-wave kernel with the reported lanes) --
also with the warm start advanced by interpolation (Sec. IV-B) and the state
estimate predicted over a delay with the vehicle's last served command (Sec. IV-E),
run alone as mppi_predict then mppi_update; requests are coalesced into batches and
two slots run at once; a snapshot restores the exact continuation; budget and
argument errors are reported.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import dev

pytestmark = pytest.mark.gpu

K_CHOICES = (64, 200, 1024, 2048)


@pytest.fixture(scope="module")
def lib():
    import paper_2407_09812_amd as lib
    return lib


def make_requests(n_req, n_veh, seed, N_max=64, M_max=40, dt_ctrl_frac=0.0, delay=0.0):
    rng = np.random.default_rng(seed)
    fleet = [W.random_vehicle(rng, v, seed, K=64, N=N_max, M=int(rng.integers(0, M_max + 1)))
             for v in range(n_veh)]
    reqs, count = [], [0] * n_veh
    for _ in range(n_req):
        v = int(rng.integers(0, n_veh))
        sc = fleet[v]
        K, N = int(rng.choice(K_CHOICES)), int(rng.integers(5, N_max + 1))
        t = count[v]
        count[v] += 1
        x_hat = W.state_on_reference(sc.ref, t * sc.dt, sc.veh)
        x_hat[:3] += rng.normal(0, 0.05, 3)
        reqs.append(dict(vid=v, K=K, N=N, dt=sc.dt, lam=sc.lam, sigma=sc.sigma, seed=seed,
                         x_hat=x_hat.astype(np.float32),
                         x_ref=sc.ref.rows(t * sc.dt, N, sc.dt).astype(np.float32),
                         obs=sc.obstacles, dt_ctrl=dt_ctrl_frac * sc.dt, delay=delay))
    return fleet, reqs


def new_server(lib, n_veh, n_streams=2, max_batch=4, budget=64 << 20, N_max=64, cost=None):
    veh, cost = W.vehicle_benchmark(), (W.cost_benchmark() if cost is None else cost)
    srv = lib.Server(veh, cost, W.hover_control(veh), n_vehicles=n_veh, K_max=2048, N_max=N_max,
                     M_max=40, n_streams=n_streams, max_batch=max_batch, budget_bytes=budget)
    srv.set_batch_config(256, 0, 4, 4)           # lanes chosen per instance
    return srv


def submit_all(lib, srv, reqs):
    return [srv.submit(r["vid"], r["K"], r["N"], r["dt"], r["lam"], r["sigma"], r["seed"],
                       r["x_hat"], r["x_ref"], lib.obstacles_host(r["obs"]),
                       dt_ctrl=r.get("dt_ctrl", 0.0), delay=r.get("delay", 0.0)) for r in reqs]


def replay_alone(lib, reqs, results, n_veh, N_max=64, warm=None, t0=None):
    """Each vehicle's requests in order through mppi_predict (over the delay the
    server reports, with the vehicle's previous command) and mppi_update from its own
    warm start."""
    veh, cost = W.vehicle_benchmark(), W.cost_benchmark()
    u_init = W.hover_control(veh)
    ctx = lib.Context(0)
    lib.mppi_reserve(ctx, 2048, N_max, 40)
    u_full = [dev(np.tile(u_init, (N_max, 1))) if warm is None else dev(warm[v]) for v in range(n_veh)]
    hold = [dev(u_init) for _ in range(n_veh)]
    outs = []
    for r, res in zip(reqs, results):
        v, K, N = r["vid"], r["K"], r["N"]
        M = r["obs"].shape[0]
        if res["pipe"]:                                   # a lone request: the default shape
            lib.mppi_set_config(ctx, K, N, M, 64, res["lanes"], 1, 0, 1)
        else:                                             # batched: the one-wave kernel
            lib.mppi_set_config(ctx, K, N, M, 64, res["lanes"], 1)
        solve = dict(K=K, N=N, dt=r["dt"], lam=r["lam"], sigma=r["sigma"], u_init=u_init,
                     seed=r["seed"], vehicle_id=v, t=res["t"], dt_ctrl=r.get("dt_ctrl", 0.0))
        u_apply = torch.empty(8, device="cuda")
        diag = lib.new_diag()
        x_hat = dev(r["x_hat"])
        if res["delay"] > 0:
            lib.mppi_predict(ctx, veh, r["dt"], res["delay"], x_hat, hold[v], x_hat)
        lib.mppi_update(ctx, veh, cost, solve, x_hat, dev(r["x_ref"]),
                        lib.obstacles_to_device(r["obs"]), M, u_full[v][:N], u_apply, diag)
        hold[v] = u_apply[:4].clone()
        torch.cuda.synchronize()
        outs.append((u_apply.cpu().numpy(), lib.diag_from_tensor(diag)))
    warm_out = np.stack([u.cpu().numpy() for u in u_full])
    ctx.close()
    return outs, warm_out


@pytest.mark.parametrize("dt_ctrl_frac,delay", [(0.0, 0.0), (0.25, 0.004)])
def test_served_equals_alone_bitwise(lib, dt_ctrl_frac, delay):
    n_veh = 6
    fleet, reqs = make_requests(40, n_veh, seed=61, dt_ctrl_frac=dt_ctrl_frac, delay=delay)
    srv = new_server(lib, n_veh)
    try:
        tickets = submit_all(lib, srv, reqs)
        results = [srv.wait(t) for t in tickets]
        stats = srv.stats()
        snap = np.frombuffer(srv.snapshot(), dtype=np.uint8)
    finally:
        srv.close()
    print("server stats", stats, "lone requests run by the pipe:", sum(r["pipe"] for r in results))
    assert stats["completed"] == 40 and stats["batches"] < 40          # coalesced
    assert all(r["status"] == 0 for r in results)
    per_vehicle_t = {}
    for r, res in zip(reqs, results):                                    # per-vehicle order
        assert res["t"] == per_vehicle_t.get(r["vid"], 0)
        per_vehicle_t[r["vid"]] = res["t"] + 1
    alone, warm = replay_alone(lib, reqs, results, n_veh)
    for res, (ua, dg) in zip(results, alone):
        assert res["delay"] == np.float32(delay)
        assert np.array_equal(res["u_apply"].astype(np.float32), ua)
        assert res["rho"] == dg["rho"] and res["argmin"] == dg["argmin"] and res["ess"] == dg["ess"]
    warm_srv = snap[: warm.nbytes].view(np.float32).reshape(warm.shape)
    assert np.array_equal(warm_srv, warm)


def test_two_slots_overlap_and_batches_coalesce(lib):
    n_veh = 16
    _, reqs = make_requests(64, n_veh, seed=62)
    srv = new_server(lib, n_veh, n_streams=2, max_batch=4)
    try:
        tickets = submit_all(lib, srv, reqs)
        srv.drain()
        stats = srv.stats()
        lat = [srv.poll(t)["latency_s"] for t in tickets]
    finally:
        srv.close()
    print("stats", stats, "p50 latency ms", 1e3 * np.median(lat))
    assert stats["completed"] == 64 and stats["batches"] <= 64
    assert stats["max_in_flight"] > 4          # more than one slot's batch in flight at once
    assert all(np.isfinite(lat)) and min(lat) > 0


def test_snapshot_restore_continues_exactly(lib):
    """Warm starts, last served commands (used by the delay prediction) and update
    counters come back exactly: the restored server continues bit for bit while a
    vehicle's requests ran in the same shape on both servers (their slots and batch
    sizes differ, so a request may run alone on one and batched on the other; from
    then on the two agree to rounding)."""
    n_veh = 4
    _, reqs = make_requests(24, n_veh, seed=63, dt_ctrl_frac=0.5, delay=0.012)
    first, second = reqs[:12], reqs[12:]
    a = new_server(lib, n_veh)
    try:
        [a.wait(t) for t in submit_all(lib, a, first)]
        snap = a.snapshot()
        res_a = [a.wait(t) for t in submit_all(lib, a, second)]
    finally:
        a.close()
    b = new_server(lib, n_veh, n_streams=1, max_batch=3)
    try:
        b.restore(snap)
        res_b = [b.wait(t) for t in submit_all(lib, b, second)]
    finally:
        b.close()
    same = {}
    for x, y in zip(res_a, res_b):
        v = x["vehicle_id"]
        same[v] = same.get(v, True) and (x["pipe"], x["lanes"]) == (y["pipe"], y["lanes"])
        assert x["t"] == y["t"] and x["status"] == 0 and y["status"] == 0
        if same[v]:
            assert np.array_equal(x["u_apply"], y["u_apply"])
        else:
            e = np.abs(x["u_apply"] - y["u_apply"]) / np.maximum(np.abs(y["u_apply"]), 1.0)
            assert e.max() <= 1e-4


def test_delay_from_the_served_latency(lib):
    """delay < 0: each request is predicted over the running median of the served
    submit-to-result latency -- 0 before any request has finished, then positive and
    of the order of the measured latencies."""
    n_veh = 8
    _, reqs = make_requests(48, n_veh, seed=65, delay=-1.0)
    srv = new_server(lib, n_veh)
    try:
        results = []
        for i in range(0, 48, 8):                        # in waves, so that latencies exist
            results += [srv.wait(t) for t in submit_all(lib, srv, reqs[i:i + 8])]
    finally:
        srv.close()
    delays = np.array([r["delay"] for r in results])
    lat = np.array([r["latency_s"] for r in results])
    print("delays used (ms)", np.round(1e3 * delays, 3), "median latency (ms)", 1e3 * np.median(lat))
    assert all(r["status"] == 0 and np.all(np.isfinite(r["u_apply"])) for r in results)
    assert delays[0] == 0.0 and np.all(delays >= 0) and np.all(delays[8:] > 0)
    assert delays.max() <= lat.max() * 1.0001


def test_budget_and_argument_errors(lib):
    srv = new_server(lib, 3, n_streams=1, budget=1 << 20)        # 1 MiB of delta_u per slot
    try:
        _, reqs = make_requests(1, 3, seed=64)
        r = dict(reqs[0], K=2048, N=64, x_ref=np.zeros((65, 13), np.float32))
        with pytest.raises(lib.MPPIError) as e:                  # 2048 x 64 x 16 B > 1 MiB
            submit_all(lib, srv, [r])
        assert e.value.status == -4
        with pytest.raises(lib.MPPIError) as e:
            submit_all(lib, srv, [dict(reqs[0], vid=7)])
        assert e.value.status == -1
        with pytest.raises(ValueError):
            submit_all(lib, srv, [dict(reqs[0], x_ref=np.zeros((3, 13), np.float32))])
        with pytest.raises(lib.MPPIError) as e:                  # never issued
            srv.poll(12345)
        assert e.value.status == -1
        for bad in (dict(dt_ctrl=-0.001), dict(dt_ctrl=1.0), dict(delay=float("nan")),
                    dict(delay=1e3)):
            with pytest.raises(lib.MPPIError) as e:
                submit_all(lib, srv, [dict(reqs[0], **bad)])
            assert e.value.status == -1
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()


def test_served_results_match_oracle(lib, orc):
    """Served updates against the FP64 oracle, teacher-forced per wave: before each
    wave the server's snapshot gives every vehicle's warm start and last served
    command; the oracle then predicts each request's state estimate over the delay the
    server reports with that command held (Sec. IV-E), runs the update (Algorithm 1)
    with the interpolating advance (Sec. IV-B), and the served applied control and the
    advanced warm start must agree at 1e-4.  The temperature is raised so that the
    softmin's amplification of binary32 cost rounding (kappa) stays below 1e-5, checked
    through the minimum cost the server reports.  Waves mix requests that run alone
    (wave-specialised rollouts) and in batches (one-wave kernel).  The obstacles keep
    their quadratic margin term but no collision constant: a state within binary32
    reach of a surface would flip that constant and move a cost by far more than the
    softmin tolerates at any useful temperature (the rollout tests cover the flips)."""
    from gpu_support import f32, f32_params, rel_err
    n_veh, N_max, lam = 8, 64, 3e5
    fleet, reqs = make_requests(40, n_veh, seed=66, dt_ctrl_frac=0.5, delay=0.006)
    by_vehicle = {}
    for r in reqs:
        by_vehicle.setdefault(r["vid"], []).append(dict(r, lam=lam))
    waves = [[q.pop(0) for q in by_vehicle.values() if q] for _ in range(3)]
    waves = [waves[0], waves[1][:1], waves[2]]       # all at once, one alone, all at once
    veh, cost = W.vehicle_benchmark(), dict(W.cost_benchmark(), obs_collision=0.0)
    o_veh, o_cost = f32_params(veh), f32_params(cost)
    u_init = W.hover_control(veh)
    srv = new_server(lib, n_veh, max_batch=4, cost=cost)
    worst = dict(u_apply=0.0, u_nom=0.0, kappa=0.0)
    shapes = set()
    t_of = [0] * n_veh
    try:
        for wave in waves:
            snap = np.frombuffer(srv.snapshot(), dtype=np.uint8)
            nw = n_veh * N_max * 4
            warm = snap[: 4 * nw].view(np.float32).reshape(n_veh, N_max, 4).astype(np.float64)
            hold = snap[4 * nw: 4 * (nw + 4 * n_veh)].view(np.float32).reshape(n_veh, 4)
            results = [srv.wait(t) for t in submit_all(lib, srv, wave)]
            after = np.frombuffer(srv.snapshot(), dtype=np.uint8)
            warm_after = after[: 4 * nw].view(np.float32).reshape(n_veh, N_max, 4)
            for r, res in zip(wave, results):
                v, K, N = r["vid"], r["K"], r["N"]
                assert res["status"] == 0 and res["t"] == t_of[v]
                t_of[v] += 1
                shapes.add(res["pipe"])
                solve = f32_params(dict(K=K, N=N, dt=r["dt"], lam=lam, sigma=r["sigma"],
                                        u_init=u_init, seed=r["seed"], vehicle_id=v, t=res["t"],
                                        dt_ctrl=r["dt_ctrl"]))
                x_hat = orc.predict(o_veh, solve["dt"], float(res["delay"]), f32(r["x_hat"]),
                                    hold[v].astype(np.float64))
                o = orc.update(o_veh, o_cost, solve, x_hat, warm[v, :N], f32(r["x_ref"]),
                               np.column_stack([r["obs"][:, :1], f32(r["obs"][:, 1:])]))
                sigma = np.asarray(r["sigma"], float)
                floors = np.concatenate([sigma, np.ones(4)])
                worst["u_apply"] = max(worst["u_apply"],
                                       rel_err(res["u_apply"], o["u_apply"], floors).max())
                worst["u_nom"] = max(worst["u_nom"],
                                     rel_err(warm_after[v, :N], o["u_nom"], sigma).max())
                # the cost error at the minimum over lambda, and eta's relative error,
                # which is the weighted mean of (dS_k - dS_rho) / lambda: both bound kappa
                # from below where it matters
                worst["kappa"] = max(worst["kappa"], abs(res["rho"] - o["diag"][0]) / lam,
                                     rel_err(res["eta"], o["diag"][1], 1.0))
                assert rel_err(res["ess"], o["diag"][2], 1.0) <= 1e-4
    finally:
        srv.close()
    print(f"served vs oracle over {sum(len(w) for w in waves)} requests, shapes {shapes}: {worst}")
    assert shapes == {0, 1}                           # both lone and batched requests
    assert worst["kappa"] <= 1e-5
    assert worst["u_apply"] <= 1e-4 and worst["u_nom"] <= 1e-4
