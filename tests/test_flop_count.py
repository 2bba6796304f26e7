"""The work counts the benchmark's rooflines use are the FP64 oracle's own operation
counts (oracle/flop_count.cpp: the oracle compiled with a counting scalar type), with
the vehicle-constant allocation work it redoes at each step taken out."""
import shutil

import pytest

import bench


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_bench_work_counts_are_the_oracles():
    from oracle import flop_count
    c = flop_count.derive()
    assert bench.FLOP_PER_ROLLOUT == c["per_rollout"]
    assert bench.FLOP_PER_STEP == c["per_step"]
    assert bench.FLOP_PER_TEST == {0: c["per_test_sphere"], 1: c["per_test_cylinder"]}
    # Gamma^-1 by elimination plus Gamma in four derivative evaluations per step
    assert c["vehicle_constants_per_step"] > 200


def test_rollout_flop_formula():
    assert bench.rollout_flop(1, 1, []) == bench.FLOP_PER_ROLLOUT + bench.FLOP_PER_STEP
    assert bench.rollout_flop(2, 3, [0, 1, 1]) == 2 * (bench.FLOP_PER_ROLLOUT + 3 * bench.FLOP_PER_STEP
                                                       + 4 * (bench.FLOP_PER_TEST[0]
                                                              + 2 * bench.FLOP_PER_TEST[1]))
