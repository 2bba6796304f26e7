"""Wave-specialised rollouts (launch shape pipe = 1): noise, body rates, attitude,
translation with the tracking cost, and obstacle costs on different waves of a
workgroup, handing chunks of steps over through LDS.  The dynamics and cost are the
one-wave kernel's operation for operation; the obstacles each tests differ (the pipe's
obstacle waves test the x-sorted window of their samples' x-range with one or two
lanes, the obstacles near the box of a chunk's positions with four or eight; the
one-wave kernel those near the box of four steps' positions), all exact: the skipped
obstacles add zero, but the L lanes of a sample divide the tests differently, so
penalty sums may round differently, and the compiler's fusion of multiplies into adds
differs at a few places, so costs agree to the last unit or two of binary32.  Bars,
for every lane count and unroll, ragged K and N not a multiple of the chunk: the
perturbations bit for bit; the costs within 1e-5 relative (a state on an obstacle
surface may flip the collision indicator: then a whole multiple of the collision
constant); the whole update within 1e-4 (sigma floors); neither kernel tests more than
all the obstacles at every state; and the oracle at 1e-4.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import (TOL, DeviceProblem, check_cost_flips, check_costs, rel_err,
                         surface_gap)

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


def rollout(lib, ctx, P, lanes, unroll, pipe):
    lib.mppi_set_config(ctx, P.K, P.N, P.M, 64, lanes, unroll, 0, pipe)
    du = torch.full((P.N * 4 * P.K,), float("nan"), device="cuda")
    S = torch.full((P.K,), float("nan"), device="cuda")
    lib.mppi_rollout(ctx, P.sc.veh, P.sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom, du,
                     P.K, S)
    torch.cuda.synchronize()
    return du, S


def update(lib, ctx, P, lanes, unroll, pipe, fused=0):
    lib.mppi_set_config(ctx, P.K, P.N, P.M, 64, lanes, unroll, fused, pipe)
    un, ua, dg = P.u_nom.clone(), torch.empty(8, device="cuda"), lib.new_diag()
    lib.mppi_profile_enable(ctx, True)
    lib.mppi_profile_read(ctx)
    lib.mppi_update(ctx, P.sc.veh, P.sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un, ua, dg)
    prof = lib.mppi_profile_read(ctx)
    lib.mppi_profile_enable(ctx, False)
    torch.cuda.synchronize()
    return un, ua, dg, prof["obstacle_tests"]


SCENES = [("c2", lambda: W.c2_line(K=700, N=61)), ("c3", lambda: W.c3_agile(K=2000, N=122)),
          ("c1", lambda: W.c1_plain(K=130, N=7)), ("paper", W.paper_preset)]


@pytest.mark.parametrize("scene", [s[0] for s in SCENES])
def test_pipe_matches_one_wave_kernel(lib, ctx, scene):
    sc = dict(SCENES)[scene]()
    P = DeviceProblem(lib, sc, t=2)
    for lanes in (1, 2, 4, 8):
        if lanes > 1 and P.M < 2 * lanes:
            continue
        for unroll in (1, 4):
            du0, S0 = rollout(lib, ctx, P, lanes, unroll, 0)
            du1, S1 = rollout(lib, ctx, P, lanes, unroll, 1)
            assert torch.equal(du0, du1), (scene, lanes, unroll)
            s0, s1 = S0.double().cpu().numpy(), S1.double().cpu().numpy()
            r = (s1 - s0) / sc.cost["obs_collision"]
            flip = np.abs(r) >= 0.5
            assert np.abs(r[flip] - np.round(r[flip])).max(initial=0.0) * sc.cost["obs_collision"] \
                <= 1e-5 * np.abs(s0[flip]).max(initial=1.0)
            e_S = (np.abs(s1 - s0) / np.maximum(np.abs(s0), 1.0))[~flip].max()
            n_diff = int((s1 != s0).sum())
            a = update(lib, ctx, P, lanes, unroll, 0)
            b = update(lib, ctx, P, lanes, unroll, 1)
            sigma = np.asarray(sc.sigma)
            e_u = rel_err(b[0].view(-1, 4).double().cpu().numpy(), a[0].view(-1, 4).double().cpu().numpy(),
                          sigma).max()
            e_a = rel_err(b[1].double().cpu().numpy(), a[1].double().cpu().numpy(), 1.0).max()
            print(f"{scene} lanes={lanes} unroll={unroll}: costs differing {n_diff}/{P.K} (max rel "
                  f"{e_S:.1e}, flips {int(flip.sum())}), update {e_u:.1e}, applied {e_a:.1e}, "
                  f"obstacle tests {a[3]} / {b[3]}")
            assert e_S <= 1e-5 and flip.sum() <= 2 and e_u <= TOL and e_a <= TOL
            dense = P.K * (P.N + 1) * P.M
            assert a[3] <= dense and b[3] <= dense
            # single pass, both kernels
            f0 = update(lib, ctx, P, lanes, unroll, 0, 1)
            f1 = update(lib, ctx, P, lanes, unroll, 1, 1)
            e_f = rel_err(f1[0].view(-1, 4).double().cpu().numpy(),
                          f0[0].view(-1, 4).double().cpu().numpy(), sigma).max()
            e_s = rel_err(f1[0].view(-1, 4).double().cpu().numpy(),
                          a[0].view(-1, 4).double().cpu().numpy(), sigma).max()
            print(f"   single pass: pipe vs one-wave {e_f:.1e}, vs stored {e_s:.1e}")
            assert e_f <= TOL and e_s <= TOL and f0[3] == a[3] and f1[3] == b[3]


@pytest.mark.parametrize("spheres", [0, 1, 100])
def test_pipe_obstacle_types_match_oracle(lib, ctx, orc, spheres):
    """The obstacle waves skip the z terms when a block holds vertical cylinders only:
    the c3 scene with none, one and half of its cylinders turned into spheres, against
    the oracle, for one and eight obstacle lanes."""
    sc = W.c3_agile(K=512, N=41)
    obs = sc.obstacles.copy()
    # spheres of radius 0.4 on the reference path, centred 0.28 above it: every
    # sample's cost depends on their z terms (the oracle's costs change everywhere when
    # they are taken for cylinders)
    idx = np.random.default_rng(7).choice(len(obs), spheres, replace=False)
    rows = sc.ref.rows(0, sc.N, sc.dt)
    at = np.linspace(5, sc.N, spheres).astype(int)
    obs[idx, 0] = 0.0
    obs[idx, 1:3] = rows[at, 0:2]
    obs[idx, 4] = 0.4
    obs[idx, 3] = rows[at, 2] + 0.7 * obs[idx, 4]
    sc.obstacles = obs
    P = DeviceProblem(lib, sc)
    ks = np.arange(0, P.K, 5)
    _, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                       P.o_x_ref, P.o_obs, want_states=False)
    kt = torch.as_tensor(ks, device="cuda")
    for lanes in (1, 8):
        du, S = rollout(lib, ctx, P, lanes, 1, 1)
        du_g = du.view(P.N, 4, P.K)[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
        e_du = rel_err(du_g, du_o, np.asarray(sc.sigma)).max()
        e_S, flips = check_cost_flips(S[kt].double().cpu().numpy(), S_o, sc.cost["obs_collision"], TOL)
        print(f"spheres {spheres} lanes {lanes}: du {e_du:.2e} S {e_S:.2e} flips {flips}")
        assert e_du <= TOL and e_S <= TOL and flips <= 2


def test_pipe_rollouts_match_oracle(lib, ctx, orc):
    sc = W.c3_agile(K=512, N=41)
    P = DeviceProblem(lib, sc)
    du, S = rollout(lib, ctx, P, 4, 4, 1)
    ks = np.arange(0, P.K, 7)
    _, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                       P.o_x_ref, P.o_obs, want_states=False)
    kt = torch.as_tensor(ks, device="cuda")
    du_g = du.view(P.N, 4, P.K)[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
    S_g = S[kt].double().cpu().numpy()
    e_du = rel_err(du_g, du_o, np.asarray(sc.sigma)).max()
    e_S, flips = check_cost_flips(S_g, S_o, sc.cost["obs_collision"], TOL)
    print(f"pipe vs oracle: du {e_du:.2e} S {e_S:.2e} collision-boundary {flips}")
    assert e_du <= TOL and e_S <= TOL and flips <= 2


def pipe_vs_oracle(lib, ctx, orc, sc, lanes, unroll, ks, n_exact=None):
    lib.mppi_reserve(ctx, sc.K, sc.N, max(sc.M, 1))
    P = DeviceProblem(lib, sc)
    du, S = rollout(lib, ctx, P, lanes, unroll, 1)
    _, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                       P.o_x_ref, P.o_obs, want_states=False)
    kt = torch.as_tensor(ks, device="cuda")
    du_g = du.view(P.N, 4, P.K)[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
    S_g = S[kt].double().cpu().numpy()
    e_du = rel_err(du_g, du_o, np.asarray(sc.sigma)).max()
    e_S, flips = check_cost_flips(S_g, S_o, sc.cost["obs_collision"], TOL)
    return e_du, e_S, flips, S, rel_err(S_g, S_o, 1.0)


@pytest.mark.parametrize("K,N,M,lanes", [(1, 30, 20, 2), (65, 1, 20, 4), (130, 7, 0, 1),
                                         (200, 23, 384, 8), (64, 9, 384, 1), (70, 6, 1536, 8)])
def test_pipe_edge_shapes_match_oracle(lib, ctx, orc, K, N, M, lanes):
    """One sample; one lane in the last workgroup (K = 65); a single step; no
    obstacles; culled lists (M = 384) and the largest list the pipe takes (M = 1536,
    uncut, 150 KB of LDS): the perturbations and costs match the oracle at 1e-4."""
    rng = np.random.default_rng(K + N + M)
    sc = W.c2_line(K=K, N=N)
    sc.obstacles = (W.spheres_in_box(rng, M, (-2, -3, 0), (8, 3, 5), 0.05, 0.3) if M
                    else np.zeros((0, 5)))
    assert sc.M == M
    ks = np.arange(K) if K <= 130 else np.arange(0, K, 3)
    for unroll in (1, 4):
        e_du, e_S, flips, _, _ = pipe_vs_oracle(lib, ctx, orc, sc, lanes, unroll, ks)
        print(f"K={K} N={N} M={M} lanes={lanes} unroll={unroll}: du {e_du:.1e} "
              f"S {e_S:.1e} collision-boundary {flips}")
        assert e_du <= TOL and e_S <= TOL and flips <= 2


@pytest.mark.parametrize("M", [40, 160])
def test_obstacles_with_equal_x_match_oracle(lib, ctx, orc, M):
    """Obstacle centres on a 0.5 m grid in x, so many share their sort key: the rank
    sort breaks ties by index (M = 40: one wave's lane-held keys; M = 160: keys in LDS),
    every obstacle lands in its own slot and culling stays exact -- costs match the
    oracle, which tests every obstacle, through the pipe and the one-wave kernel."""
    rng = np.random.default_rng(M)
    sc = W.c2_line(K=192, N=12)
    obs = W.spheres_in_box(rng, M, (-1, -3, 0), (7, 3, 5), 0.1, 0.4)
    obs[:, 1] = np.round(obs[:, 1] * 2.0) / 2.0
    assert len(np.unique(obs[:, 1])) < M // 2
    sc.obstacles = obs
    ks = np.arange(0, sc.K, 2)
    lib.mppi_reserve(ctx, sc.K, sc.N, sc.M)
    P = DeviceProblem(lib, sc)
    _, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                       P.o_x_ref, P.o_obs, want_states=False)
    kt = torch.as_tensor(ks, device="cuda")
    for pipe, lanes in ((1, 2), (1, 8), (0, 1), (0, 4)):
        du, S = rollout(lib, ctx, P, lanes, 1, pipe)
        S_g = S[kt].double().cpu().numpy()
        e_S, flips = check_cost_flips(S_g, S_o, sc.cost["obs_collision"], TOL)
        print(f"M={M} pipe={pipe} lanes={lanes}: S {e_S:.1e} collision-boundary {flips}")
        assert e_S <= TOL and flips <= 2


def test_pipe_longest_horizon(lib, ctx, orc):
    """N = 4096 through the pipe: costs match the oracle within binary32 drift over
    41 s of flight (1e-2, as for the one-wave kernel's states) and stay finite."""
    sc = W.c1_plain(K=64, N=4096)
    e_du, _, _, S, e_all = pipe_vs_oracle(lib, ctx, orc, sc, 1, 1, np.array([0, 31, 63]))
    print(f"N=4096 pipe: du {e_du:.1e} S {e_all.max():.1e}")
    assert e_du <= TOL and e_all.max() < 1e-2 and torch.isfinite(S).all()


def test_pipe_rejects_too_many_obstacles(lib, ctx):
    with pytest.raises(lib.MPPIError) as e:
        lib.mppi_set_config(ctx, 1024, 50, 1537, 64, 4, 1, 0, 1)
    assert e.value.status == -1


# ---------------------------------------------------------------------------
# The wave-specialised rollouts at the benchmarked sizes and launch shapes, against
# the oracle directly (not through the one-wave kernel)
# ---------------------------------------------------------------------------

C2_SHAPE = (64, 2, 1, 0, 1)          # block, lanes, unroll, fused, pipe


def test_pipe_c2_bench_shape_every_sample(lib, ctx, orc):
    """c2 at full size (K = 4096, N = 100, 20 spheres) in the benchmark's launch shape:
    every sample's perturbations and cost against the oracle at 1e-4; a cost that
    differs by a whole multiple of the collision constant must belong to a sample
    whose binary64 trajectory passes within binary32 reach of an obstacle surface."""
    sc = W.c2_line()
    P = DeviceProblem(lib, sc, t=4)
    lib.mppi_set_config(ctx, P.K, P.N, P.M, *C2_SHAPE)
    du, S = rollout(lib, ctx, P, C2_SHAPE[1], C2_SHAPE[2], 1)
    st_o, du_o, S_o = orc.rollouts(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref,
                                   P.o_obs, want_states=True)
    du_g = du.view(P.N, 4, P.K).permute(2, 0, 1).double().cpu().numpy()
    e_du = rel_err(du_g, du_o, np.asarray(sc.sigma)).max()
    gap, reach = surface_gap(st_o, P.o_obs)
    e_S, flips = check_cost_flips(S.double().cpu().numpy(), S_o, sc.cost["obs_collision"], TOL,
                                  gap, reach)
    print(f"c2 pipe {C2_SHAPE}: du {e_du:.2e} S {e_S:.2e} over {P.K} samples, flips {flips}")
    assert e_du <= TOL and e_S <= TOL and flips <= max(2, P.K // 200)


@pytest.mark.parametrize("unroll", [1, 4])
def test_pipe_c3_bench_shape_sampled(lib, ctx, orc, unroll):
    """c3 at full size (K = 16384, N = 200, 200 cylinders) with eight obstacle lanes:
    160 sampled rollouts including the first and last sample of a workgroup and of the
    launch, against the oracle at 1e-4 under the same flip rule."""
    sc = W.c3_agile()
    P = DeviceProblem(lib, sc, t=7)
    du, S = rollout(lib, ctx, P, 8, unroll, 1)
    rng = np.random.default_rng(33)
    ks = np.unique(np.concatenate([[0, 63, 64, 127, 8191, P.K - 64, P.K - 1],
                                   rng.integers(0, P.K, 160)]))
    st_o, du_o, S_o = orc.rollouts_subset(P.o_veh, P.o_cost, P.o_solve, ks, P.o_x_hat, P.o_u_nom,
                                          P.o_x_ref, P.o_obs, want_states=True)
    kt = torch.as_tensor(ks, device="cuda")
    du_g = du.view(P.N, 4, P.K)[:, :, kt].permute(2, 0, 1).double().cpu().numpy()
    e_du = rel_err(du_g, du_o, np.asarray(sc.sigma)).max()
    gap, reach = surface_gap(st_o, P.o_obs)
    e_S, flips = check_cost_flips(S[kt].double().cpu().numpy(), S_o, sc.cost["obs_collision"], TOL,
                                  gap, reach)
    print(f"c3 pipe lanes=8 unroll={unroll}: du {e_du:.2e} S {e_S:.2e} over {ks.size} samples, "
          f"flips {flips}")
    assert e_du <= TOL and e_S <= TOL and flips <= 2
    assert torch.isfinite(S).all()


@pytest.mark.parametrize("lam", [1.0, 300.0])
def test_pipe_c2_full_update_stage_isolated(lib, ctx, orc, lam):
    """The whole update as the benchmark runs it (c2, pipe shape, stored form: the
    rollout launch with the weight statistics, then the sum launch that applies and
    shifts) against the oracle's weights, weighted update, feasible input and shift
    computed from the device's own costs and perturbations (the same launch shape's
    rollouts, which are deterministic)."""
    sc = W.c2_line()
    sol = dict(sc.solve(2), lam=lam)
    P = DeviceProblem(lib, sc, t=2, solve=sol)
    lib.mppi_set_config(ctx, P.K, P.N, P.M, *C2_SHAPE)
    un, ua, dg = P.u_nom.clone(), torch.empty(8, device="cuda"), lib.new_diag()
    lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, un, ua, dg)
    du, S = rollout(lib, ctx, P, C2_SHAPE[1], C2_SHAPE[2], 1)
    S64 = S.double().cpu().numpy()
    w_o, d_o = orc.weights(S64, float(np.float32(lam)))
    u_o = orc.weighted_update(w_o, du.view(P.N, 4, P.K).permute(2, 0, 1).double().cpu().numpy(),
                              P.o_u_nom)
    ua_o, un_o = orc.apply_shift(P.o_veh, P.o_solve["dt"], P.o_x_hat, u_o, P.o_solve["u_init"])
    d = lib.diag_from_tensor(dg)
    sigma = np.asarray(sc.sigma)
    e_a = rel_err(ua.double().cpu().numpy(), ua_o, np.concatenate([sigma, np.ones(4)])).max()
    e_n = rel_err(un.view(-1, 4).double().cpu().numpy(), un_o, sigma).max()
    print(f"c2 pipe update lam={lam}: u_apply {e_a:.2e} u_nom {e_n:.2e} ess {d['ess']:.4g} "
          f"vs {d_o[2]:.4g}")
    assert d["status"] == 0 and d["lanes"] == C2_SHAPE[1]
    assert d["rho"] == S64.min() and d["argmin"] == int(d_o[3])
    assert rel_err(d["eta"], d_o[1], 1.0) <= TOL and rel_err(d["ess"], d_o[2], 1.0) <= TOL
    assert e_a <= TOL and e_n <= TOL


def test_pipe_c2_end_to_end_when_kappa_small(lib, ctx, orc):
    """c2 through the pipe against the oracle's own update (its own costs): with the
    temperature raised until kappa <= 1e-5 the applied control and the shifted warm
    start agree at 1e-4."""
    sc = W.c2_line()
    sol = dict(sc.solve(1), lam=3e5)
    P = DeviceProblem(lib, sc, t=1, solve=sol)
    lib.mppi_set_config(ctx, P.K, P.N, P.M, *C2_SHAPE)
    un, ua = P.u_nom.clone(), torch.empty(8, device="cuda")
    lib.mppi_update(ctx, sc.veh, sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, un, ua)
    _, S = rollout(lib, ctx, P, C2_SHAPE[1], C2_SHAPE[2], 1)
    r = orc.update(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref, P.o_obs)
    dS = S.double().cpu().numpy() - r["S"]
    kappa = np.max(np.abs(dS - dS[int(r["diag"][3])])) / P.o_solve["lam"]
    sigma = np.asarray(sc.sigma)
    e_a = rel_err(ua.double().cpu().numpy(), r["u_apply"], np.concatenate([sigma, np.ones(4)])).max()
    e_n = rel_err(un.view(-1, 4).double().cpu().numpy(), r["u_nom"], sigma).max()
    print(f"c2 pipe end to end: kappa {kappa:.2e} u_apply {e_a:.2e} u_nom {e_n:.2e}")
    assert kappa <= 1e-5 and e_a <= TOL and e_n <= TOL


def test_stored_pipe_shape_past_its_obstacle_limit(lib, ctx, orc):
    """A pipe shape stored for the size class of M = 1536 also covers M = 2000 (same
    power-of-two class), past the pipe's limit: the update then runs the one-wave
    kernel with the stored lanes and unroll; its rollouts match the oracle, and the
    update matches the oracle's weights and update from the device's own costs."""
    rng = np.random.default_rng(2000)
    sc = W.c2_line(K=256, N=20)
    sc.obstacles = W.spheres_in_box(rng, 2000, (-2, -3, 0), (8, 3, 5), 0.05, 0.2)
    lib.mppi_reserve(ctx, sc.K, sc.N, 2048)
    lib.mppi_set_config(ctx, sc.K, sc.N, 1536, 64, 4, 4, 0, 1)
    cfg = lib.mppi_get_config(ctx, sc.K, sc.N, 2000)
    assert cfg["pipe"] == 0 and cfg["lanes"] == 4 and cfg["unroll"] == 4
    P = DeviceProblem(lib, sc)
    un, ua, dg = P.u_nom.clone(), torch.empty(8, device="cuda"), lib.new_diag()
    lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un, ua, dg)
    du = torch.empty(P.N * 4 * P.K, device="cuda")
    S = torch.empty(P.K, device="cuda")
    lib.mppi_rollout(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom, du,
                     P.K, S)
    torch.cuda.synchronize()
    d = lib.diag_from_tensor(dg)
    assert d["status"] == 0 and d["lanes"] == 4
    _, du_o, S_o = orc.rollouts(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref,
                                P.o_obs)
    du_g = du.view(P.N, 4, P.K).permute(2, 0, 1).double().cpu().numpy()
    S_g = S.double().cpu().numpy()
    sigma = np.asarray(sc.sigma)
    e_du = rel_err(du_g, du_o, sigma).max()
    e_S, flips = check_cost_flips(S_g, S_o, sc.cost["obs_collision"], TOL)
    w_o, _ = orc.weights(S_g, P.o_solve["lam"])
    u_o = orc.weighted_update(w_o, du_g, P.o_u_nom)
    e_a = rel_err(ua[:4].double().cpu().numpy(), u_o[0], sigma).max()
    e_n = rel_err(un.view(-1, 4).double().cpu().numpy(), np.vstack([u_o[1:], P.o_solve["u_init"]]),
                  sigma).max()
    print(f"M=2000 under a stored pipe shape: du {e_du:.2e} S {e_S:.2e} flips {flips} "
          f"u_apply {e_a:.2e} u_nom {e_n:.2e}")
    assert e_du <= TOL and e_S <= TOL and flips <= 2
    assert e_a <= TOL and e_n <= TOL
