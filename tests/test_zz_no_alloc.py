"""The update that allocates nothing (mppi_update_static): its scratch is carved out
of the library's static device array, whose device address mppi_create takes.  Bars:
the applied control, the advanced warm start and the diagnostics equal mppi_update's in
the same launch shape bit for bit, on consecutive calls whose second is smaller than the
first (the array keeps the last call's contents), in the wave-specialised and the
one-wave shape, with and without a caller diag; a stored single-pass shape runs as the
stored form; an update larger than the array is rejected before any launch; and, for
the callers under graph capture it is for, the update recorded once into a HIP graph
and replayed three times (eager device work and synchronisations between the replays)
equals the same three updates issued eagerly, bit for bit, at every replay."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_support import DeviceProblem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2407_09812_amd as lib
    return lib


def run(lib, ctx, P, entry, shape, with_diag=True):
    lib.mppi_set_config(ctx, P.K, P.N, P.M, *shape)
    un, ua = P.u_nom.clone(), torch.full((8,), float("nan"), device="cuda")
    dg = lib.new_diag() if with_diag else None
    entry(ctx, P.sc.veh, P.sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un, ua, dg)
    torch.cuda.synchronize()
    return un.cpu(), ua.cpu(), (dg.cpu() if with_diag else None)


CASES = [  # scenario, update index, launch shape (block, lanes, unroll, fused, pipe)
    (lambda: W.c2_line(), 3, (64, 2, 1, 0, 1)),
    (lambda: W.c2_line(K=700, N=37), 4, (64, 2, 1, 0, 1)),
    (lambda: W.c3_agile(K=2000, N=50), 1, (256, 4, 4, 0, 0)),
    (lambda: W.c1_plain(K=130, N=9), 2, (64, 1, 1, 0, 1)),
]


def test_static_update_equals_update():
    import paper_2407_09812_amd as lib
    ctx = lib.Context(0)
    try:
        lib.mppi_reserve(ctx, 4096, 100, 200)         # for mppi_update only
        for make, t, shape in CASES:                  # sizes shrink from the first call on
            sc = make()
            P = DeviceProblem(lib, sc, t=t)
            want = run(lib, ctx, P, lib.mppi_update, shape)
            got = run(lib, ctx, P, lib.mppi_update_static, shape)
            print(f"{sc.name} K={P.K} N={P.N} M={P.M} shape {shape}: u_apply {got[1][:4].numpy()}")
            for a, b in zip(want, got):
                assert torch.equal(a, b)
            d = lib.diag_from_tensor(got[2])
            assert d["status"] == 0 and d["lanes"] == shape[1]
            # no caller diag: the array's own record is used
            nodiag = run(lib, ctx, P, lib.mppi_update_static, shape, with_diag=False)
            assert torch.equal(nodiag[0], want[0]) and torch.equal(nodiag[1], want[1])
    finally:
        ctx.close()


def test_static_update_runs_the_stored_form():
    import paper_2407_09812_amd as lib
    ctx = lib.Context(0)
    try:
        sc = W.c2_line(K=1024, N=40)
        lib.mppi_reserve(ctx, sc.K, sc.N, sc.M)
        P = DeviceProblem(lib, sc, t=1)
        want = run(lib, ctx, P, lib.mppi_update, (64, 2, 1, 0, 1))
        got = run(lib, ctx, P, lib.mppi_update_static, (64, 2, 1, 1, 1))   # stored as fused
        for a, b in zip(want, got):
            assert torch.equal(a, b)
    finally:
        ctx.close()


def test_static_update_rejects_what_does_not_fit():
    import paper_2407_09812_amd as lib
    ctx = lib.Context(0)
    try:
        sc = W.c3_agile()                              # 16 K N = 52 MB of delta_u
        P = DeviceProblem(lib, sc)
        with pytest.raises(lib.MPPIError) as e:
            lib.mppi_update_static(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M,
                                   P.u_nom.clone(), torch.empty(8, device="cuda"))
        assert e.value.status == -8
        assert "static array" in str(e.value)
    finally:
        ctx.close()


@pytest.mark.parametrize("shape", [(64, 2, 1, 0, 1), (256, 4, 1, 0, 0)])
def test_static_update_replays_in_a_graph(shape):
    import paper_2407_09812_amd as lib
    ctx = lib.Context(0)
    try:
        sc = W.c2_line(K=1024, N=40)
        P = DeviceProblem(lib, sc, t=1)
        lib.mppi_set_config(ctx, P.K, P.N, P.M, *shape)
        want = []
        un, ua, dg = P.u_nom.clone(), torch.full((8,), float("nan"), device="cuda"), lib.new_diag()
        for _ in range(3):
            lib.mppi_update_static(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un,
                                   ua, dg)
            torch.cuda.synchronize()
            want.append((un.clone(), ua.clone(), dg.clone()))

        un, ua, dg = P.u_nom.clone(), torch.full((8,), float("nan"), device="cuda"), lib.new_diag()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):                      # recorded, not run
            lib.mppi_update_static(ctx, sc.veh, sc.cost, P.solve, P.x_hat, P.x_ref, P.obs, P.M, un,
                                   ua, dg)
        torch.cuda.synchronize()
        assert torch.equal(un, P.u_nom)                # capture ran nothing
        for r in range(3):
            g.replay()
            torch.cuda.synchronize()
            junk = torch.randn(4096, device="cuda").cumsum(0)   # eager work between replays
            torch.cuda.synchronize()
            del junk
            assert torch.equal(un, want[r][0]), r
            assert torch.equal(ua, want[r][1]), r
            assert torch.equal(dg, want[r][2]), r
        del g
    finally:
        ctx.close()
