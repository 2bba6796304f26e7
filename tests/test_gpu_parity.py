"""GPU parity: the HIP path, called through the C ABI, against the FP64 oracle on the
same seeded inputs.

Bars (relative error as defined in gpu_support, binary32 device arithmetic):
  - Philox words: bit-exact.   - diag rho / argmin from the same costs: exact.
  - noise, states, costs, weights (floor 1/K), update, applied input: <= 1e-4.
  - Samples with a state on an obstacle surface closer than the binary32 and
    binary64 trajectories differ may see the collision indicator flip; their costs
    must then differ by a whole multiple of the collision constant (both are
    correct), and they are counted.
  - End-to-end updates (oracle's own costs) are compared at 1e-4 when the measured
    kappa = max_k |(dS_k - dS_rho)| / lambda <= 1e-5, since the softmin amplifies
    cost differences by 1/lambda.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import TOL, DeviceProblem, check_costs, dev, f32, f32_params, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2407_09812_amd as lib
    return lib


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    lib.mppi_reserve(c, 16384, 200, 256)
    yield c
    c.close()


def run_rollout(lib, ctx, P, dump=True, ld=None):
    K, N = P.K, P.N
    ld = K if ld is None else ld
    du = torch.full((N * 4 * ld,), float("nan"), device="cuda")
    S = torch.empty(K, device="cuda")
    states = torch.empty((N + 1) * 17 * ld, device="cuda") if dump else None
    lib.mppi_rollout(ctx, P.sc.veh, P.sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom,
                     du, ld, S, states)
    torch.cuda.synchronize()
    du = du.view(N, 4, ld)[:, :, :K]
    st = states.view(N + 1, 17, ld)[:, :, :K] if dump else None
    return du, S, st


def check_rollouts(orc, P, du_g, S_g, st_g, ks, n_exact=None):
    """Compare sampled rollouts ks (GPU tensors [N,4,K], [K], [N+1,17,K]).  States
    are held to TOL over the first n_exact steps (all by default); beyond that,
    binary32 drift over long horizons is bounded separately by the caller."""
    st_o, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                          P.o_x_ref, P.o_obs)
    kt = torch.as_tensor(ks, device="cuda", dtype=torch.long)
    du_gk = du_g[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
    st_gk = st_g[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
    S_gk = S_g[kt].double().cpu().numpy()
    sigma = np.maximum(np.asarray(P.solve["sigma"], float), 1e-30)
    n = st_o.shape[1] if n_exact is None else n_exact + 1
    e_du = rel_err(du_gk, du_o, sigma).max()
    e_st = rel_err(st_gk[:, :n], st_o[:, :n], 1.0).max()
    e_S, flips = check_costs(S_gk, S_o, st_gk, st_o, P.o_obs, P.o_cost["obs_collision"], TOL)
    print(f"K={P.K} N={P.N} M={P.M} sampled={len(ks)} max rel err: du {e_du:.2e} "
          f"states {e_st:.2e} S {e_S:.2e} collision-boundary samples {flips}")
    assert e_du <= TOL and e_st <= TOL
    if n_exact is None:
        assert e_S <= TOL
    assert flips <= max(2, 0.05 * len(ks))
    return st_gk, st_o, S_gk, S_o


# ---------------------------------------------------------------------------
# noise
# ---------------------------------------------------------------------------

def test_philox_bitwise_1e6(lib, ctx, orc):
    rng = np.random.default_rng(11)
    n = 1 << 20
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[: n // 2, 0] = np.arange(n // 2) % 16384            # (k, j) like counters
    ctr[: n // 2, 1] = np.arange(n // 2) // 16384
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    lib.mppi_philox(ctx, dev(ctr.view(np.int32), torch.int32), dev(key.view(np.int32), torch.int32),
                    out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, orc.philox_many(ctr, key))


def test_noise_matches_oracle(lib, ctx, orc):
    K, N = 4096, 100
    slv = dict(K=K, N=N, dt=0.01, lam=1.0, sigma=(1.0, 0.5, 2.0, 0.25), u_init=(9.81, 0, 0, 0),
               seed=(3 << 32) | 77, vehicle_id=7, t=13)
    ld = K + 64
    du = torch.empty(N * 4 * ld, device="cuda")
    lib.mppi_noise(ctx, slv, du, ld)
    torch.cuda.synchronize()
    g = du.view(N, 4, ld)[:, :, :K].permute(2, 0, 1).double().cpu().numpy()
    o = orc.noise(K, N, f32(slv["sigma"]), slv["seed"], 7, 13)
    err = rel_err(g, o, f32(slv["sigma"])).max()
    print(f"noise max rel err {err:.2e}")
    assert err <= TOL


# ---------------------------------------------------------------------------
# rollouts and costs
# ---------------------------------------------------------------------------

def test_rollout_parity_c1_full(lib, ctx, orc):
    P = DeviceProblem(lib, W.c1_plain())
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(P.K))


def test_rollout_parity_c2_ragged(lib, ctx, orc):
    """K = 1000 is not a multiple of the 64-lane workgroup: the tail is partial."""
    P = DeviceProblem(lib, W.c2_line(K=1000, N=100))
    du, S, st = run_rollout(lib, ctx, P, ld=1024)
    check_rollouts(orc, P, du, S, st, np.arange(P.K))


def test_rollout_parity_c2_full_size(lib, ctx, orc):
    P = DeviceProblem(lib, W.c2_line())
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(P.K))


def test_rollout_parity_c3_full_size_sampled(lib, ctx, orc):
    """K = 16384, N = 200, 200 cylinders: the oracle recomputes 160 sampled rollouts."""
    P = DeviceProblem(lib, W.c3_agile())
    du, S, st = run_rollout(lib, ctx, P)
    rng = np.random.default_rng(3)
    ks = np.unique(np.concatenate([[0, 63, 64, P.K - 1], rng.integers(0, P.K, 156)]))
    check_rollouts(orc, P, du, S, st, ks)
    assert torch.isfinite(S).all()


def test_rollout_parity_paper_model(lib, ctx, orc):
    """The paper's algebraic rotor model (no lag), Table I vehicle, Table II weights and
    the indicator-only obstacle cost, with a pillar on the path."""
    sc = W.c2_line(K=512, N=60)
    sc.veh, sc.cost = W.vehicle_paper(), W.cost_paper()
    sc.obstacles = np.array([[W.VCYL, 4.0, 0.2, 0.0, 0.5], [W.SPHERE, 2.0, -0.5, 2.5, 0.4]])
    sc.x0 = W.state_on_reference(sc.ref, 0.0, sc.veh)
    sc.u_init = W.hover_control(sc.veh)
    sol = sc.solve(5)
    sol["sigma"] = np.sqrt([0.60, 0.15, 0.15, 0.05])
    sol["lam"] = 1e-4
    P = DeviceProblem(lib, sc, t=5, solve=sol)
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(P.K))


@pytest.mark.parametrize("lanes,block,unroll", [(1, 64, 1), (2, 128, 4), (4, 64, 4), (8, 256, 1),
                                                (8, 64, 4)])
def test_rollout_parity_every_launch_shape(lib, ctx, orc, lanes, block, unroll):
    """Each shape (lanes per sample dividing the obstacle tests, workgroup size,
    unroll) computes the same rollouts; K = 700 leaves a partial last workgroup."""
    P = DeviceProblem(lib, W.c2_line(K=700, N=60))
    lib.mppi_set_config(ctx, P.K, P.N, P.M, block, lanes, unroll)
    assert lib.mppi_get_config(ctx, P.K, P.N, P.M) == dict(block=block, lanes=lanes, unroll=unroll,
                                                            fused=0, pipe=0)
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(P.K))
    P3 = DeviceProblem(lib, W.c3_agile(K=2000, N=120))
    lib.mppi_set_config(ctx, P3.K, P3.N, P3.M, block, lanes, unroll)
    du, S, st = run_rollout(lib, ctx, P3)
    check_rollouts(orc, P3, du, S, st, np.arange(0, P3.K, 13))


def test_autotune_picks_a_valid_shape(lib, ctx, orc):
    P = DeviceProblem(lib, W.c3_agile(K=4096, N=50))
    best = lib.mppi_autotune(ctx, P.sc.veh, P.sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M,
                             P.u_nom, reps=2)
    print("autotuned", best)
    assert best["lanes"] in (1, 2, 4, 8) and best["block"] in (64, 128, 256)
    assert lib.mppi_get_config(ctx, P.K, P.N, P.M) == best
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(0, P.K, 41))


def test_rollout_edge_shapes(lib, ctx, orc):
    """K = 1, K = 65 (one lane in the last workgroup), N = 1, M = 0."""
    for K, N in ((1, 30), (65, 1), (130, 7)):
        P = DeviceProblem(lib, W.c2_line(K=K, N=N))
        du, S, st = run_rollout(lib, ctx, P)
        check_rollouts(orc, P, du, S, st, np.arange(K))


@pytest.mark.parametrize("N", [5, 6, 7])
def test_rollout_chunked_culling_mixed_obstacles(lib, ctx, orc, N):
    """The one-wave rollouts take the obstacle terms four steps at a time by the box of
    those steps' positions: horizons that end inside a chunk, for every lane count, in a
    scene of cylinders and spheres on the reference path (centred above it, so that
    their z terms decide), against the oracle."""
    sc = W.c3_agile(K=256, N=N)
    obs = sc.obstacles.copy()
    rows = sc.ref.rows(0, sc.N, sc.dt)
    idx = np.random.default_rng(8).choice(len(obs), 30, replace=False)
    at = np.linspace(1, sc.N, 30).astype(int)
    obs[idx, 0] = 0.0
    obs[idx, 1:3] = rows[at, 0:2]
    obs[idx, 4] = 0.4
    obs[idx, 3] = rows[at, 2] + 0.7 * obs[idx, 4]
    sc.obstacles = obs
    P = DeviceProblem(lib, sc)
    for lanes in (1, 2, 4, 8):
        lib.mppi_set_config(ctx, P.K, P.N, P.M, 64, lanes, 1)
        du, S, st = run_rollout(lib, ctx, P)
        check_rollouts(orc, P, du, S, st, np.arange(P.K))


def test_rollout_longest_horizon(lib, ctx, orc):
    """N = 4096 (41 s of flight): states match at 1e-4 over the first 200 steps (the
    longest configured horizon); over the whole horizon binary32 drift stays below
    1e-2, quaternions stay unit and costs finite."""
    P = DeviceProblem(lib, W.c1_plain(K=64, N=4096))
    du, S, st = run_rollout(lib, ctx, P)
    st_g, st_o, S_g, S_o = check_rollouts(orc, P, du, S, st, np.array([0, 31, 63]), n_exact=200)
    drift = rel_err(st_g, st_o, 1.0).max()
    qn = np.linalg.norm(st[:, 3:7, :].double().cpu().numpy(), axis=1)
    print(f"N=4096 drift {drift:.2e}, |q| - 1 max {np.abs(qn - 1).max():.1e}")
    assert drift < 1e-2 and np.abs(qn - 1).max() < 1e-5
    assert torch.isfinite(S).all() and rel_err(S_g, S_o, 1.0).max() < 1e-2


def test_rollout_max_obstacles(lib, ctx, orc):
    rng = np.random.default_rng(9)
    sc = W.c2_line(K=128, N=20)
    sc.obstacles = W.spheres_in_box(rng, 2048, (-2, -3, 0), (8, 3, 5), 0.05, 0.2)
    lib.mppi_reserve(ctx, 128, 20, 2048)
    P = DeviceProblem(lib, sc)
    du, S, st = run_rollout(lib, ctx, P)
    check_rollouts(orc, P, du, S, st, np.arange(0, 128, 5))


# ---------------------------------------------------------------------------
# weights, weighted sum, apply/shift (stage-isolated: the oracle is given the
# GPU's own costs and perturbations)
# ---------------------------------------------------------------------------

def stage_check(lib, ctx, orc, P, lam):
    K, N = P.K, P.N
    du, S, _ = run_rollout(lib, ctx, P, dump=False)
    w = torch.empty(K, device="cuda")
    diag = lib.new_diag()
    lib.mppi_weights(ctx, K, S, lam, w, diag)
    u_upd = torch.empty(N * 4, device="cuda")
    du_c = du.contiguous()
    lib.mppi_weighted_sum(ctx, K, N, w, du_c, K, P.u_nom, u_upd, diag)
    u_nom2 = torch.empty(N * 4, device="cuda")
    u_apply = torch.empty(8, device="cuda")
    lib.mppi_apply_shift(ctx, P.sc.veh, P.solve, P.x_hat, u_upd, u_nom2, u_apply)
    torch.cuda.synchronize()
    dg = lib.diag_from_tensor(diag)

    S64 = S.double().cpu().numpy()
    w_o, d_o = orc.weights(S64, float(np.float32(lam)))
    assert dg["status"] == 0 and dg["n_finite"] == K and dg["lanes"] == 0   # stage call
    assert dg["rho"] == S64.min() and dg["argmin"] == int(d_o[3])          # same binary32 costs
    assert rel_err(dg["eta"], d_o[1], 1.0) <= TOL and rel_err(dg["ess"], d_o[2], 1.0) <= TOL
    e_w = rel_err(w.double().cpu().numpy(), w_o, 1.0 / K).max()

    du64 = du.permute(2, 0, 1).double().cpu().numpy()
    w64 = w.double().cpu().numpy()
    u_o = orc.weighted_update(w64, du64, P.o_u_nom)
    sigma = np.maximum(np.asarray(P.solve["sigma"], float), 1e-30)
    e_u = rel_err(u_upd.view(N, 4).double().cpu().numpy(), u_o, sigma).max()

    ua_o, un_o = orc.apply_shift(P.o_veh, P.o_solve["dt"], P.o_x_hat, u_upd.view(N, 4).double().cpu().numpy(),
                                 P.o_solve["u_init"])
    ua = u_apply.double().cpu().numpy()
    assert np.array_equal(ua[:4], u_upd[:4].double().cpu().numpy())
    e_a = rel_err(ua[4:], ua_o[4:], 1.0).max()
    assert np.array_equal(u_nom2.view(N, 4).double().cpu().numpy(), f32(un_o))
    print(f"stage K={K} N={N} lam={lam}: w {e_w:.2e} update {e_u:.2e} applied {e_a:.2e} "
          f"ess {dg['ess']:.3g}")
    assert e_w <= TOL and e_u <= TOL and e_a <= TOL
    return S, du, w, u_upd, u_apply, u_nom2, diag


@pytest.mark.parametrize("lam", [1.0, 300.0, 1e6])
def test_update_stages_c2(lib, ctx, orc, lam):
    P = DeviceProblem(lib, W.c2_line())
    stage_check(lib, ctx, orc, P, lam)


def test_update_stages_c1_ragged(lib, ctx, orc):
    P = DeviceProblem(lib, W.c1_plain(K=250, N=20))
    stage_check(lib, ctx, orc, P, 50.0)


@pytest.mark.parametrize("lam", [1.0, 300.0])
def test_full_update_equals_stages_and_is_deterministic(lib, ctx, orc, lam):
    """The full update (two launches: rollouts with the weight statistics, then the
    weighted sum with apply and advance) agrees with the stage entry points, and
    repeats bit for bit."""
    sc = W.c2_line()
    sol = dict(sc.solve(3), lam=lam)
    P = DeviceProblem(lib, sc, t=3, solve=sol)
    _, _, _, u_upd, u_apply_s, u_nom_s, diag_s = stage_check(lib, ctx, orc, P, lam)
    outs = []
    for _ in range(2):
        u_nom = P.u_nom.clone()
        u_apply = torch.empty(8, device="cuda")
        diag = lib.new_diag()
        lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, u_nom, u_apply,
                        diag)
        torch.cuda.synchronize()
        outs.append((u_nom.cpu(), u_apply.cpu(), diag.cpu()))
    assert all(torch.equal(a, b) for a, b in zip(outs[0], outs[1]))
    d_s = lib.diag_from_tensor(diag_s)
    sigma = np.asarray(sc.sigma)
    u_nom, u_apply, diag = outs[0]
    e_n = rel_err(u_nom.view(-1, 4).double().numpy(), u_nom_s.view(-1, 4).double().cpu().numpy(),
                  sigma).max()
    e_a = rel_err(u_apply.double().numpy(), u_apply_s.double().cpu().numpy(), 1.0).max()
    d = lib.diag_from_tensor(diag)
    print(f"full vs stages lam={lam}: u_nom {e_n:.2e} u_apply {e_a:.2e} eta {d['eta']} vs {d_s['eta']}")
    assert e_n <= TOL and e_a <= TOL
    assert d["lanes"] == lib.mppi_get_config(ctx, P.K, P.N, P.M)["lanes"]
    for k in ("rho", "argmin", "n_finite", "status"):
        assert d[k] == d_s[k]
    assert rel_err(d["eta"], d_s["eta"], 1.0) <= TOL and rel_err(d["ess"], d_s["ess"], 1.0) <= TOL


def test_weight_statistics_do_not_depend_on_workgroup_size(lib):
    """K = 40000 with eight lanes per sample gives 5000 wave records (more than one
    batch per lane of each part): the reduced statistics are bit for bit the same when
    one, four or twelve waves reduce them (one-wave kernel with 64- and 256-thread
    workgroups, the pipe), and agree with the stage weights at the tolerance."""
    sc = W.c2_line(K=40000, N=10)
    P = DeviceProblem(lib, sc)
    ctx = lib.Context(0)                     # its own capacity: the shared context stays small
    lib.mppi_reserve(ctx, P.K, P.N, P.M)
    diags = []
    for shape in ((64, 8, 1, 0, 0), (256, 8, 1, 0, 0), (64, 8, 1, 0, 1)):
        lib.mppi_set_config(ctx, P.K, P.N, P.M, *shape)
        u_nom = P.u_nom.clone()
        u_apply = torch.empty(8, device="cuda")
        diag = lib.new_diag()
        lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, u_nom, u_apply,
                        diag)
        torch.cuda.synchronize()
        diags.append(lib.diag_from_tensor(diag))
    for d in diags[1:]:
        for k in ("rho", "argmin", "n_finite", "status", "eta", "ess", "lanes"):
            assert d[k] == diags[0][k], (k, d[k], diags[0][k])
    du, S, _ = run_rollout(lib, ctx, P, dump=False)
    w = torch.empty(P.K, device="cuda")
    ds = lib.new_diag()
    lib.mppi_weights(ctx, P.K, S, P.solve["lam"], w, ds)
    torch.cuda.synchronize()
    d_s = lib.diag_from_tensor(ds)
    assert diags[0]["rho"] == d_s["rho"] and diags[0]["argmin"] == d_s["argmin"]
    assert rel_err(diags[0]["eta"], d_s["eta"], 1.0) <= TOL
    assert rel_err(diags[0]["ess"], d_s["ess"], 1.0) <= TOL


def test_prepared_update_equals_update(lib, ctx):
    """lib.prepare_update marshals the arguments once; calling it twice gives what two
    mppi_update calls on the same buffers give, bit for bit, and it reads the buffers'
    current contents at each call."""
    sc = W.c2_line(K=512, N=30)
    P = DeviceProblem(lib, sc)
    outs = []
    for prepared in (False, True):
        u_nom, u_apply, diag = P.u_nom.clone(), torch.empty(8, device="cuda"), lib.new_diag()
        x_hat = P.x_hat.clone()
        call = (lib.prepare_update(ctx, sc.veh, sc.cost, P.solve, x_hat, P.x_ref, P.obs, P.M,
                                   u_nom, u_apply, diag) if prepared else
                (lambda: lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, x_hat, P.x_ref, P.obs, P.M,
                                         u_nom, u_apply, diag)))
        call()
        x_hat[0] += 0.5                          # the second call sees the new state
        call()
        torch.cuda.synchronize()
        outs.append((u_nom.cpu(), u_apply.cpu(), diag.cpu()))
    assert all(torch.equal(a, b) for a, b in zip(outs[0], outs[1]))
    bad = dict(P.solve, lam=-1.0)
    with pytest.raises(lib.MPPIError):
        lib.prepare_update(ctx, sc.veh, sc.cost, bad, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom,
                           torch.empty(8, device="cuda"))()


def test_update_writes_pinned_host_output(lib, ctx):
    """u_apply in pinned host memory (through mppi_device_address): the command lands
    on the host without a copy, bit for bit the device-memory result, over consecutive
    updates of a closed loop (warm start carried in u_nom)."""
    sc = W.c2_line(K=1024, N=40)
    P = DeviceProblem(lib, sc, t=1)
    un_d, un_h = P.u_nom.clone(), P.u_nom.clone()
    ua_d = torch.empty(8, device="cuda")
    ua_h = torch.full((8,), float("nan"), pin_memory=True)
    for t in range(3):
        sol = sc.solve(1 + t)
        lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, un_d, ua_d)
        lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, un_h, ua_h)
        torch.cuda.synchronize()
        assert torch.equal(ua_h, ua_d.cpu()) and torch.equal(un_h, un_d)
    assert lib.device_address(ua_h) == lib.device_address(ua_h)       # cached
    with pytest.raises(lib.MPPIError):                                 # pageable memory
        lib.device_address(torch.zeros(8))


def test_end_to_end_update_when_kappa_small(lib, ctx, orc):
    """Oracle's own costs: with lambda large enough that kappa <= 1e-5 the whole
    update must match at 1e-4."""
    sc = W.c1_plain()
    sol = sc.solve(0)
    sol["lam"] = 1e5
    P = DeviceProblem(lib, sc, solve=sol)
    u_nom = P.u_nom.clone()
    u_apply = torch.empty(8, device="cuda")
    diag = lib.new_diag()
    lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, u_nom, u_apply, diag)
    du, S, _ = run_rollout(lib, ctx, P, dump=False)
    torch.cuda.synchronize()
    r = orc.update(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref, P.o_obs)
    dS = S.double().cpu().numpy() - r["S"]
    kappa = np.max(np.abs(dS - dS[int(r["diag"][3])])) / sol["lam"]
    e_a = rel_err(u_apply.double().cpu().numpy(), r["u_apply"], 1.0).max()
    e_n = rel_err(u_nom.view(-1, 4).double().cpu().numpy(), r["u_nom"], 1.0).max()
    print(f"kappa {kappa:.2e} u_apply {e_a:.2e} u_nom {e_n:.2e}")
    assert kappa <= 1e-5
    assert e_a <= TOL and e_n <= TOL


def test_obstacle_test_counter(lib, ctx):
    """With profiling on, the library counts the obstacle distance tests it performs:
    every (sample, state, obstacle) without culling (M < 16), and no more than that
    -- here far fewer, but some -- when the culling by the wave's box of positions is
    on (spheres scattered over the path's first metres, some within reach)."""
    rng = np.random.default_rng(12)
    for M, dense_only in ((10, True), (200, False)):
        sc = W.c2_line(K=1000, N=40)
        sc.obstacles = W.spheres_in_box(rng, M, (-1.0, -4.0, 0.5), (9.0, 4.0, 4.5), 0.2, 0.6)
        P = DeviceProblem(lib, sc)
        lib.mppi_reserve(ctx, P.K, P.N, M)
        lib.mppi_profile_enable(ctx, True)
        lib.mppi_profile_read(ctx)
        u_nom, u_apply = P.u_nom.clone(), torch.empty(8, device="cuda")
        lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, M, u_nom, u_apply)
        prof = lib.mppi_profile_read(ctx)
        lib.mppi_profile_enable(ctx, False)
        dense = P.K * (P.N + 1) * M
        print(f"M={M}: {prof['obstacle_tests']} tests of {dense} dense")
        if dense_only:
            assert prof["obstacle_tests"] == dense
        else:
            assert 0 < prof["obstacle_tests"] < 0.5 * dense


def test_single_sample_update_is_brute_force(lib, ctx, orc):
    sc = W.c1_plain(K=1, N=12)
    P = DeviceProblem(lib, sc)
    _, du, w, u_upd, _, _, _ = stage_check(lib, ctx, orc, P, 1.0)
    assert w.item() == 1.0
    assert torch.equal(u_upd.view(12, 4), P.u_nom + du[:, :, 0])


def test_zero_noise_update_keeps_nominal(lib, ctx, orc):
    sc = W.c2_line(K=300, N=40)
    sol = sc.solve(0)
    sol["sigma"] = (0.0, 0.0, 0.0, 0.0)
    P = DeviceProblem(lib, sc, solve=sol)
    S, du, w, u_upd, _, _, _ = stage_check(lib, ctx, orc, P, 1.0)
    assert torch.all(du == 0) and torch.all(S == S[0])
    assert torch.all(w == w[0]) and abs(w[0].item() * 300 - 1.0) < 1e-6
    assert torch.equal(u_upd, P.u_nom.view(-1))


def test_all_nonfinite_costs_leave_warm_start(lib, ctx):
    sc = W.c2_line(K=256, N=20)
    x = sc.x0.copy()
    x[7] = np.nan
    P = DeviceProblem(lib, sc, x_hat=x)
    u_nom = P.u_nom.clone() + 0.25
    before = u_nom.clone()
    u_apply = torch.empty(8, device="cuda")
    diag = lib.new_diag()
    lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, u_nom, u_apply, diag)
    torch.cuda.synchronize()
    d = lib.diag_from_tensor(diag)
    assert d["status"] == -3                               # MPPI_E_ALL_NONFINITE
    assert d["n_finite"] == 0
    assert torch.equal(u_nom, before)
    assert torch.equal(u_apply[:4], before[0])


def test_capacity_and_argument_errors(lib, ctx):
    sc = W.c2_line(K=20000, N=20)
    P = DeviceProblem(lib, W.c2_line(K=64, N=20))
    u_apply = torch.empty(8, device="cuda")
    with pytest.raises(lib.MPPIError) as e:
        lib.mppi_update(ctx, sc.veh, sc.cost, sc.solve(0), P.x_hat, P.x_ref, P.obs, P.M,
                        P.u_nom, u_apply)
    assert e.value.status == -8
    bad = dict(P.solve, lam=-1.0)
    with pytest.raises(lib.MPPIError) as e:
        lib.mppi_update(ctx, sc.veh, sc.cost, bad, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom, u_apply)
    assert e.value.status == -1


# ---------------------------------------------------------------------------
# closed loop
# ---------------------------------------------------------------------------

def test_plant_step_parity(lib, ctx, orc):
    sc = W.c3_agile(K=64, N=10)
    rng = np.random.default_rng(4)
    for _ in range(20):
        x = sc.x0.copy()
        x[7:13] += rng.normal(0, 1, 6)
        u = np.array([rng.uniform(5, 30), *rng.normal(0, 2, 3)])
        xo = torch.empty(17, device="cuda")
        lib.mppi_plant_step(ctx, sc.veh, sc.dt, dev(x), dev(u), xo)
        torch.cuda.synchronize()
        ref = orc.model_step(f32_params(sc.veh), f32(x), f32(u), float(np.float32(sc.dt)))
        assert rel_err(xo.double().cpu().numpy(), ref, 1.0).max() <= TOL


def test_closed_loop_c1_teacher_forced(lib, ctx, orc):
    """50 closed-loop updates of the plain configuration; each update starts from the
    GPU's own (x_hat, u_nom) and is checked stage by stage against the oracle."""
    sc = W.c1_plain()
    x = sc.x0.copy()
    u_nom = sc.u_nom0()
    worst = dict(S=0.0, upd=0.0, plant=0.0)
    for t in range(sc.updates):
        P = DeviceProblem(lib, sc, t=t, x_hat=x, u_nom=u_nom)
        du, S, _ = run_rollout(lib, ctx, P, dump=False)
        _, _, S_o = orc.rollouts(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref)
        worst["S"] = max(worst["S"], rel_err(S.double().cpu().numpy(), S_o, 1.0).max())
        un = P.u_nom.clone()
        ua = torch.empty(8, device="cuda")
        lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un, ua)
        w_o, _ = orc.weights(S.double().cpu().numpy(), 1.0)
        upd_o = orc.weighted_update(w_o, du.permute(2, 0, 1).double().cpu().numpy(), P.o_u_nom)
        worst["upd"] = max(worst["upd"], rel_err(ua[:4].double().cpu().numpy(), upd_o[0], 1.0).max())
        xo = torch.empty(17, device="cuda")
        lib.mppi_plant_step(ctx, sc.veh, sc.dt, P.x_hat, ua, xo)
        torch.cuda.synchronize()
        ref = orc.model_step(P.o_veh, P.o_x_hat, f32(ua[:4].cpu().numpy()), P.o_solve["dt"])
        worst["plant"] = max(worst["plant"], rel_err(xo.double().cpu().numpy(), ref, 1.0).max())
        x, u_nom = xo.double().cpu().numpy(), un.view(-1, 4).double().cpu().numpy()
    print("closed loop worst rel err", worst, "final position", x[:3])
    assert max(worst.values()) <= TOL
    assert np.all(np.isfinite(x)) and abs(np.linalg.norm(x[3:7]) - 1.0) < 1e-5
