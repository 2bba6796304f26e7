"""The single-pass update (launch shape fused = 1): per-wave minima, weights and
partial weighted sums at the end of the rollout launch, perturbations regenerated
from the counter-based noise instead of stored, then one merge launch (Eqs. (4),
(5)).

Bars (relative error <= 1e-4, floors as in the other parity tests): the oracle's
weights and weighted update computed from the GPU's own costs and perturbations
(stage-isolated, any lambda); the whole update against the oracle's own when
kappa <= 1e-5; diagnostics; the all-non-finite case; determinism; every lane count,
ragged K and N not a multiple of the four-step chunk.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import TOL, DeviceProblem, f32, rel_err

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


def fused_update(lib, ctx, P, lanes, block=64, unroll=1, fused=1, solve=None):
    """Full update with the given shape; returns (u_upd [N,4] reconstructed from the
    applied control and the shifted warm start, u_apply, diag).  The warm start is
    shifted by a whole step here (dt_ctrl = 0) so that u_upd can be read back."""
    sol = dict(P.solve if solve is None else solve, dt_ctrl=0.0)
    lib.mppi_set_config(ctx, P.K, P.N, P.M, block, lanes, unroll, fused)
    un, ua, dg = P.u_nom.clone(), torch.empty(8, device="cuda"), lib.new_diag()
    lib.mppi_update(ctx, P.sc.veh, P.sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, un, ua, dg)
    torch.cuda.synchronize()
    un = un.view(P.N, 4).double().cpu().numpy()
    upd = np.vstack([ua[:4].double().cpu().numpy()[None], un[:-1]])
    return upd, ua, lib.diag_from_tensor(dg)


def stored_rollout(lib, ctx, P, lanes, block=64, unroll=1, solve=None):
    sol = P.solve if solve is None else solve
    lib.mppi_set_config(ctx, P.K, P.N, P.M, block, lanes, unroll, 0)
    du = torch.empty(P.N * 4 * P.K, device="cuda")
    S = torch.empty(P.K, device="cuda")
    lib.mppi_rollout(ctx, P.sc.veh, P.sc.cost, sol, P.x_hat, P.x_ref, P.obs, P.M, P.u_nom, du, P.K, S)
    torch.cuda.synchronize()
    return (du.view(P.N, 4, P.K).permute(2, 0, 1).double().cpu().numpy(),
            S.double().cpu().numpy())


def stage_check(lib, ctx, orc, P, lanes, lam, block=64, unroll=1):
    sol = dict(P.solve, lam=lam)
    du, S = stored_rollout(lib, ctx, P, lanes, block, unroll, sol)
    upd, _, dg = fused_update(lib, ctx, P, lanes, block, unroll, 1, sol)
    w_o, d_o = orc.weights(S, float(np.float32(lam)))
    upd_o = orc.weighted_update(w_o, du, P.o_u_nom)
    sigma = np.maximum(np.asarray(P.solve["sigma"], float), 1e-30)
    e_u = rel_err(upd, upd_o, sigma).max()
    e_eta = rel_err(dg["eta"], d_o[1], 1.0)
    e_ess = rel_err(dg["ess"], d_o[2], 1.0)
    print(f"fused K={P.K} N={P.N} M={P.M} lanes={lanes} block={block} lam={lam:g}: update {e_u:.2e} "
          f"eta {e_eta:.2e} ess {e_ess:.2e} ({dg['ess']:.4g})")
    assert dg["status"] == 0 and dg["n_finite"] == P.K and dg["lanes"] == lanes
    assert dg["argmin"] == int(d_o[3]) and dg["rho"] == S.min()
    assert e_u <= TOL and e_eta <= TOL and e_ess <= TOL
    return upd, dg


@pytest.mark.parametrize("lanes,block,unroll", [(1, 64, 1), (2, 128, 4), (4, 64, 4), (8, 256, 1),
                                                (4, 256, 4)])
def test_fused_stage_parity_every_shape(lib, ctx, orc, lanes, block, unroll):
    """K = 700 (partial last wave and workgroup), N = 61 (not a multiple of 4)."""
    P = DeviceProblem(lib, W.c2_line(K=700, N=61))
    stage_check(lib, ctx, orc, P, lanes, 1.0, block, unroll)
    P3 = DeviceProblem(lib, W.c3_agile(K=2000, N=122))
    stage_check(lib, ctx, orc, P3, lanes, 1.0, block, unroll)


@pytest.mark.parametrize("lam", [1e-4, 1.0, 300.0, 1e6])
def test_fused_stage_parity_temperatures(lib, ctx, orc, lam):
    P = DeviceProblem(lib, W.c2_line())
    stage_check(lib, ctx, orc, P, 4, lam)


def test_fused_edge_shapes(lib, ctx, orc):
    """K = 1, 65, 130 and N = 1, 3, 7; no obstacles (c1) and the paper preset."""
    for K, N in ((1, 30), (65, 1), (130, 7), (257, 3)):
        stage_check(lib, ctx, orc, DeviceProblem(lib, W.c1_plain(K=K, N=N)), 1, 1.0)
    stage_check(lib, ctx, orc, DeviceProblem(lib, W.paper_preset()), 4, 1e-4)


def test_fused_full_size_c3(lib, ctx, orc):
    """K = 16384, N = 200, 200 cylinders: 1024 partial sums of 800 values merged."""
    P = DeviceProblem(lib, W.c3_agile())
    stage_check(lib, ctx, orc, P, 4, 1.0, 256, 4)


def test_fused_end_to_end_when_kappa_small(lib, ctx, orc):
    sc = W.c1_plain()
    P = DeviceProblem(lib, sc, solve=dict(sc.solve(0), lam=1e5))
    upd, ua, dg = fused_update(lib, ctx, P, 1)
    r = orc.update(P.o_veh, P.o_cost, P.o_solve, P.o_x_hat, P.o_u_nom, P.o_x_ref, P.o_obs)
    _, S = stored_rollout(lib, ctx, P, 1)
    dS = S - r["S"]
    kappa = np.max(np.abs(dS - dS[int(r["diag"][3])])) / 1e5
    e_a = rel_err(ua.double().cpu().numpy(), r["u_apply"], 1.0).max()
    print(f"fused end to end: kappa {kappa:.2e} u_apply {e_a:.2e}")
    assert kappa <= 1e-5 and e_a <= TOL


def test_fused_deterministic_and_close_to_stored(lib, ctx):
    P = DeviceProblem(lib, W.c3_agile(K=3000, N=80))
    a = fused_update(lib, ctx, P, 4, 256, 4)
    b = fused_update(lib, ctx, P, 4, 256, 4)
    assert np.array_equal(a[0], b[0]) and a[2] == b[2]
    s = fused_update(lib, ctx, P, 4, 256, 4, fused=0)
    sigma = np.asarray(P.solve["sigma"], float)
    assert rel_err(a[0], s[0], sigma).max() <= TOL
    assert a[2]["argmin"] == s[2]["argmin"] and a[2]["rho"] == s[2]["rho"]


def test_fused_all_nonfinite_costs_leave_warm_start(lib, ctx):
    sc = W.c2_line(K=256, N=20)
    x = sc.x0.copy()
    x[7] = np.nan
    P = DeviceProblem(lib, sc, x_hat=x)
    lib.mppi_set_config(ctx, P.K, P.N, P.M, 64, 2, 1, 1)
    u_nom = P.u_nom.clone() + 0.25
    before = u_nom.clone()
    ua, dg = torch.empty(8, device="cuda"), lib.new_diag()
    lib.mppi_update(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, u_nom, ua, dg)
    torch.cuda.synchronize()
    d = lib.diag_from_tensor(dg)
    assert d["status"] == -3 and d["n_finite"] == 0
    assert torch.equal(u_nom, before) and torch.equal(ua[:4], before[0])
