"""Batched execution of uneven MPPI instances (persistent kernel, HIP graph, autotuner).

Bars: an instance's results (shifted warm start, applied control, diagnostics) are
bit-identical alone (mppi_update) and inside a batch when both use the same lanes per
sample; graph replays equal eager launches bit for bit; a poisoned instance leaves the
others untouched; a batch member with kappa <= 1e-5 matches the FP64 oracle at 1e-4.
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import TOL, dev, f32, f32_params, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [  # (K, N, M) -- uneven, with partial tiles, tiny and large instances
    (1, 7, 0), (65, 1, 3), (700, 50, 40), (1024, 133, 200), (3000, 90, 12), (4096, 200, 0),
    (513, 64, 77), (2048, 120, 150), (130, 33, 5), (16384, 50, 20),
]


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


def make_fleet(seed=44, shapes=SHAPES, paper_model_every=4):
    rng = np.random.default_rng(seed)
    fleet = []
    for i, (K, N, M) in enumerate(shapes):
        sc = W.random_vehicle(rng, i, seed, K=K, N=N, M=M)
        if paper_model_every and i % paper_model_every == 3:      # algebraic rotor model
            sc.veh = W.vehicle_paper()
            sc.x0 = W.state_on_reference(sc.ref, 0.0, sc.veh)
            sc.u_init = W.hover_control(sc.veh)
        if i % 3 == 1:                     # warm start advanced by interpolation (Sec. IV-B)
            sc.dt_ctrl = sc.dt / 4
        fleet.append(sc)
    return fleet


class Inst:
    """Device inputs of one instance and a fresh copy of its warm start."""

    def __init__(self, lib, sc, t=0, solve=None, x_hat=None):
        self.sc = sc
        self.solve = dict(sc.solve(t) if solve is None else solve)
        self.x_hat = dev(sc.x0 if x_hat is None else x_hat)
        self.x_ref = dev(sc.x_ref(t))
        self.obs = lib.obstacles_to_device(sc.obstacles)
        self.u0 = dev(sc.u_nom0() + 0.01 * np.arange(sc.N)[:, None])
        self.reset()

    def reset(self):
        self.u_nom = self.u0.clone()
        self.u_apply = torch.full((8,), float("nan"), device="cuda")
        self.diag = torch.zeros(32, dtype=torch.uint8, device="cuda")

    def item(self):
        return dict(veh=self.sc.veh, cost=self.sc.cost, solve=self.solve, x_hat=self.x_hat,
                    x_ref=self.x_ref, obs=self.obs, M=self.sc.M, u_nom=self.u_nom,
                    u_apply=self.u_apply, diag=self.diag)

    def alone(self, lib, ctx):
        lib.mppi_update(ctx, self.sc.veh, self.sc.cost, self.solve, self.x_hat, self.x_ref,
                        self.obs, self.sc.M, self.u_nom, self.u_apply, self.diag)

    def outputs(self):
        return self.u_nom.clone(), self.u_apply.clone(), self.diag.clone()


def set_lanes(lib, ctx, insts, lanes, block=256, bpc=4, use_graph=True):
    lib.mppi_batch_set_config(ctx, block, lanes, 4, bpc, use_graph)
    if lanes > 0:
        for it in insts:
            lib.mppi_set_config(ctx, it.sc.K, it.sc.N, it.sc.M, 64, lanes, 1)


def run_batch(lib, ctx, insts):
    for it in insts:
        it.reset()
    reqs = lib.make_requests([it.item() for it in insts])
    lib.mppi_batch_reserve(ctx, reqs)
    lib.mppi_batch_update(ctx, reqs)
    torch.cuda.synchronize()
    return [it.outputs() for it in insts]


def run_alone(lib, ctx, insts, lanes_from=None):
    """Each instance alone; with lanes_from (batched outputs), at the lanes per sample
    each instance reported in the batch."""
    out = []
    for i, it in enumerate(insts):
        if lanes_from is not None:
            lanes = lib.diag_from_tensor(lanes_from[i][2])["lanes"]
            lib.mppi_set_config(ctx, it.sc.K, it.sc.N, it.sc.M, 64, lanes, 1)
        it.reset()
        it.alone(lib, ctx)
        torch.cuda.synchronize()
        out.append(it.outputs())
    return out


def assert_same(a, b):
    for (un1, ua1, d1), (un2, ua2, d2) in zip(a, b):
        assert torch.equal(un1, un2) and torch.equal(ua1, ua2) and torch.equal(d1, d2)


@pytest.mark.parametrize("lanes", [1, 2, 0])
def test_batch_equals_alone_bitwise(lib, ctx, lanes):
    """Fixed lanes per sample, and lanes = 0 (chosen per instance from the batch's
    occupancy): each instance equals its solo update at the lanes it reports."""
    insts = [Inst(lib, sc, t=3) for sc in make_fleet()]
    set_lanes(lib, ctx, insts, lanes)
    batched = run_batch(lib, ctx, insts)
    alone = run_alone(lib, ctx, insts, lanes_from=batched)
    assert_same(batched, alone)
    for it, (un, ua, d) in zip(insts, batched):
        dg = lib.diag_from_tensor(d)
        assert dg["status"] == 0 and torch.isfinite(ua).all()
        assert dg["lanes"] == lanes if lanes else dg["lanes"] in (1, 2, 4, 8)
    if lanes == 0:   # a small mix: instances with many obstacles get more than one lane
        assert max(lib.diag_from_tensor(d)["lanes"] for _, _, d in batched) > 1


def test_auto_lanes_fall_to_one_when_the_batch_fills_the_chip(lib, ctx):
    fleet = make_fleet(seed=51, shapes=[(16384, 20, 200)] * 6, paper_model_every=0)
    insts = [Inst(lib, sc) for sc in fleet]
    set_lanes(lib, ctx, insts, 0)
    batched = run_batch(lib, ctx, insts)
    assert all(lib.diag_from_tensor(d)["lanes"] == 1 for _, _, d in batched)


def test_graph_replays_equal_eager_launches(lib, ctx):
    insts = [Inst(lib, sc, t=1) for sc in make_fleet(seed=45)]
    set_lanes(lib, ctx, insts, 1, use_graph=False)
    eager = run_batch(lib, ctx, insts)
    set_lanes(lib, ctx, insts, 1, use_graph=True)
    for rep in range(4):
        scratch = torch.randn(1 << 20, device="cuda").cumsum(0)     # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(scratch).all()
        assert_same(run_batch(lib, ctx, insts), eager)


def test_batches_of_changing_composition_reuse_the_graph(lib, ctx):
    """One captured graph serves batches of different sizes and mixes."""
    fleet = make_fleet(seed=46)
    set_lanes(lib, ctx, [Inst(lib, sc) for sc in fleet], 1, use_graph=True)
    for subset in (fleet[:3], fleet[2:9], fleet[::2], fleet):
        insts = [Inst(lib, sc, t=2) for sc in subset]
        assert_same(run_batch(lib, ctx, insts), run_alone(lib, ctx, insts))


def test_poisoned_instance_leaves_the_others_untouched(lib, ctx):
    fleet = make_fleet(seed=47)
    insts = [Inst(lib, sc, t=0) for sc in fleet]
    x = fleet[4].x0.copy()
    x[8] = np.inf
    insts[4] = Inst(lib, fleet[4], t=0, x_hat=x)
    set_lanes(lib, ctx, insts, 1)
    batched = run_batch(lib, ctx, insts)
    alone = run_alone(lib, ctx, insts)
    assert_same(batched, alone)
    d = lib.diag_from_tensor(batched[4][2])
    assert d["status"] == -3 and d["n_finite"] == 0
    assert torch.equal(batched[4][0], insts[4].u0)                   # warm start kept
    for i, (un, ua, dg) in enumerate(batched):
        if i != 4:
            assert lib.diag_from_tensor(dg)["status"] == 0


def test_batch_member_matches_oracle_end_to_end(lib, ctx, orc):
    fleet = make_fleet(seed=48, shapes=[(256, 30, 10), (300, 25, 0), (128, 40, 30)])
    assert fleet[1].dt_ctrl > 0
    insts = []
    for sc in fleet:
        sol = sc.solve(0)
        sol["lam"] = 1e6                         # kappa <= 1e-5: end-to-end comparable
        insts.append(Inst(lib, sc, solve=sol))
    set_lanes(lib, ctx, insts, 1)
    batched = run_batch(lib, ctx, insts)
    for it, (un, ua, _) in zip(insts, batched):
        sc = it.sc
        r = orc.update(f32_params(sc.veh), f32_params(sc.cost), f32_params(it.solve), f32(sc.x0),
                       f32(it.u0.cpu().numpy()), f32(sc.x_ref(0)), sc.obstacles)
        e = rel_err(ua.double().cpu().numpy(), r["u_apply"], 1.0).max()
        e2 = rel_err(un.view(-1, 4).double().cpu().numpy(), r["u_nom"], 1.0).max()
        print(f"batch member K={sc.K} N={sc.N} M={sc.M}: u_apply {e:.2e} u_nom {e2:.2e}")
        assert e <= TOL and e2 <= TOL


def test_batch_capacity_error(lib):
    c = lib.Context(0)
    try:
        small = [Inst(lib, sc) for sc in make_fleet(seed=49, shapes=[(64, 10, 0), (64, 10, 0)])]
        lib.mppi_batch_reserve(c, lib.make_requests([it.item() for it in small]))
        big = [Inst(lib, sc) for sc in make_fleet(seed=49, shapes=[(64, 10, 0)] * 3)]
        with pytest.raises(lib.MPPIError) as e:
            lib.mppi_batch_update(c, lib.make_requests([it.item() for it in big]))
        assert e.value.status == -8
    finally:
        c.close()


def test_batch_autotune(lib, ctx):
    insts = [Inst(lib, sc, t=5) for sc in make_fleet(seed=50)]
    reqs = lib.make_requests([it.item() for it in insts])
    lib.mppi_batch_reserve(ctx, reqs)
    best = lib.mppi_batch_autotune(ctx, reqs, reps=1)
    print("batch autotune", best)
    assert best["lanes"] in (1, 2, 4) and best["block"] in (64, 128, 256)
    assert lib.mppi_batch_get_config(ctx) == best
    batched = run_batch(lib, ctx, insts)
    assert_same(batched, run_alone(lib, ctx, insts, lanes_from=batched))


def test_default_batch_shape(lib):
    """A fresh context's batch shape is the one its header documents."""
    ctx = lib.Context(0)
    assert lib.mppi_batch_get_config(ctx) == dict(block=256, lanes=0, unroll=1, blocks_per_cu=8,
                                                  use_graph=1)
