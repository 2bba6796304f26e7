"""Frozen work counts of one rollout, from an operation-counting run of the FP64 oracle
(TEST INFRASTRUCTURE, like the oracle itself).

``flop_count.cpp`` compiles ``mppi_oracle.c`` once more with its scalar type replaced by a
counting double and tallies the operations ``orc_rollout_one`` executes for N = 1..3 steps
and M = 0..2 spheres or vertical cylinders.  The counts are exactly linear:

    rollout(N, M) = per_rollout + per_step_raw * N + per_test[type] * (N + 1) * M

where per_step_raw still holds work that depends on the vehicle alone and that the oracle
redoes at every step: Gamma^-1 by elimination in the controller (Eqs. (10)-(11)) and Gamma
in each of the four derivative evaluations (Eq. (13)).  Subtracting it gives the
algorithmic count per rollout-step.  add, sub, mul, div count 1; sqrt, log, sin, cos are
listed apart and count 1 each in the FLOP totals; comparisons, negation and fabs count 0.
The obstacles sit far from the path (no margin penalty), the common case.
"""
import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "flop_count.cpp")
TRANS = ("sqrt", "log", "exp", "sin", "cos")


def run_counter() -> dict:
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "flop_count")
        subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-o", exe, SRC, "-lm"],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True,
                             env=dict(os.environ, OMP_NUM_THREADS="1")).stdout
    return json.loads(out)


def total(c: dict) -> int:
    """FLOP with each transcendental counted once."""
    return c["flop"] + sum(c[t] for t in TRANS)


def derive(raw: dict = None) -> dict:
    raw = run_counter() if raw is None else raw
    r = {k: total(v) for k, v in raw.items()}
    tr = {k: sum(v[t] for t in TRANS) for k, v in raw.items()}
    step_raw = r["rollout_sph_N2_M0"] - r["rollout_sph_N1_M0"]
    per_rollout = r["rollout_sph_N1_M0"] - step_raw
    for typ in ("sph", "cyl"):                   # the linear form holds at every point
        per_test = (r[f"rollout_{typ}_N1_M1"] - r[f"rollout_{typ}_N1_M0"]) / 2
        for N in (1, 2, 3):
            for M in (0, 1, 2):
                want = per_rollout + step_raw * N + per_test * (N + 1) * M
                assert r[f"rollout_{typ}_N{N}_M{M}"] == want, (typ, N, M)
    constants = total(raw["allocation_inverse"]) + 4 * total(raw["allocation"])
    return {
        "per_step": step_raw - constants,
        "per_step_transcendental": tr["rollout_sph_N2_M0"] - tr["rollout_sph_N1_M0"],
        "per_rollout": per_rollout,
        "per_test_sphere": (r["rollout_sph_N1_M1"] - r["rollout_sph_N1_M0"]) // 2,
        "per_test_cylinder": (r["rollout_cyl_N1_M1"] - r["rollout_cyl_N1_M0"]) // 2,
        "vehicle_constants_per_step": constants,
        "noise_per_step": total(raw["noise"]),
    }


if __name__ == "__main__":
    print(json.dumps(derive(), indent=1))
