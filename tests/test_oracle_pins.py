"""Pins for the FP64 oracle: each test checks it against something other than itself
(published values, closed forms, library routines, invariants the paper states), so
that a dropped term, a flipped sign, a wrong index or a transposed operand fails.

Citations are to arXiv 2407.09812 (sections, equations, algorithm, tables).
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def hover_state(veh, p=(0.0, 0.0, 0.0)):
    return np.concatenate([p, [1.0, 0, 0, 0], np.zeros(6), np.full(4, veh["mass"] * veh["g"] / 4)])


def quat_axis_angle(axis, ang):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * axis])


def qmul(a, b):  # Hamilton product, written out independently for test expectations
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


# ---------------------------------------------------------------------------
# P1: Philox4x32-10 and the Gaussian draws (Sec. III-A: delta_u ~ N(0, Sigma))
# ---------------------------------------------------------------------------

def test_philox_known_answers(orc):
    """Random123's published known-answer vectors (Salmon et al., SC'11)."""
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]
        n += 1
    assert n == 3


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host(orc, tmp_path):
    """rocRAND's Philox4x32-10 engine (host build) agrees bit for bit on random
    counters and keys, including counters with large high words."""
    exe = tmp_path / "rr"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), os.path.join(HERE, "rocrand_philox_ref.cpp")],
                   check=True, capture_output=True)
    rng = np.random.default_rng(1234)
    rows = rng.integers(0, 2 ** 32, size=(4000, 6), dtype=np.uint64)
    rows[:1000, 0:2] = rng.integers(0, 300, size=(1000, 2))   # small counters like (k, j)
    text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    got = [list(map(int, l.split())) for l in out.strip().split("\n")]
    assert len(got) == len(rows)
    for r, g in zip(rows, got):
        assert orc.philox4x32_10([int(x) for x in r[:4]], [int(x) for x in r[4:]]) == g


def test_uniform_is_exact_and_open(orc):
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for w in (1, 511, 512, 0x80000000, 0x12345678):
        u = orc.uniform(w)
        assert np.float32(u) == u                     # exactly representable in binary32
        assert u == ((w >> 9) * 2 + 1) * 2.0 ** -24


def test_gaussian_statistics(orc):
    """Mean, standard deviation, independence and a KS test over 1e6 draws with
    per-dimension sigma (Box-Muller from two uniforms)."""
    from scipy import stats
    sigma = np.array([1.0, 0.5, 2.0, 0.25])
    du = orc.noise(250000, 1, sigma, seed=7, vehicle_id=3, t=11).reshape(-1, 4)
    z = du / sigma
    assert np.all(np.abs(z.mean(axis=0)) < 5.0 / math.sqrt(z.shape[0]))
    assert np.all(np.abs(z.std(axis=0) - 1.0) < 5e-3)
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(4))) < 6e-3
    for d in range(4):
        assert stats.kstest(z[:, d], "norm").pvalue > 1e-4


def test_noise_counter_layout(orc):
    """Sample k, step j, update t, vehicle and seed address disjoint counters: the
    draw for (k, j) is the same whatever K and N are requested."""
    a = orc.noise(8, 5, [1, 1, 1, 1], seed=(5 << 32) | 9, vehicle_id=2, t=4)
    b = orc.noise(3, 2, [1, 1, 1, 1], seed=(5 << 32) | 9, vehicle_id=2, t=4)
    assert np.array_equal(a[:3, :2], b)
    for other in (dict(seed=9, vehicle_id=2, t=4), dict(seed=(5 << 32) | 9, vehicle_id=3, t=4),
                  dict(seed=(5 << 32) | 9, vehicle_id=2, t=5)):
        c = orc.noise(3, 2, [1, 1, 1, 1], **other)
        assert not np.any(c == b)


# ---------------------------------------------------------------------------
# P2: allocation matrix Gamma (Eqs. (10)-(11))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("veh", [W.vehicle_benchmark(), W.vehicle_paper()])
def test_allocation_matrix(orc, veh):
    G = orc.allocation(veh)
    Gi = orc.allocation_inverse(veh)
    l, c = veh["arm_l"], veh["c_tf"]
    np.testing.assert_allclose(G @ G.T, np.diag([4, 2 * l * l, 2 * l * l, 4 * c * c]), atol=1e-15)
    np.testing.assert_allclose(Gi, np.linalg.inv(G), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(Gi @ G, np.eye(4), atol=1e-13)
    # hover allocation: each rotor carries a quarter of the weight
    mg = veh["mass"] * veh["g"]
    np.testing.assert_allclose(Gi @ np.array([mg, 0, 0, 0]), np.full(4, mg / 4), rtol=1e-15)


def printed_allocation(l, c):
    """Eq. (11) typed in as printed: rows [1 1 1 1], (l/sqrt2)[-1 1 1 -1],
    (l/sqrt2)[-1 1 -1 1], c_tf[-1 -1 1 1]."""
    s = l / math.sqrt(2.0)
    return np.array([[1.0, 1.0, 1.0, 1.0],
                     [-s, s, s, -s],
                     [-s, s, -s, s],
                     [-c, -c, c, c]])


@pytest.mark.parametrize("l,c", [(0.15, 0.012), (0.23, 0.05)])
def test_allocation_is_the_printed_matrix(orc, l, c):
    """Eq. (11) element by element: a row sign flipped or two rotors swapped keeps
    the rows orthogonal (so the checks above pass) but fails here."""
    veh = W.vehicle_benchmark()
    veh.update(arm_l=l, c_tf=c)
    np.testing.assert_allclose(orc.allocation(veh), printed_allocation(l, c), rtol=0, atol=1e-15)


@pytest.mark.parametrize("axis,up", [(1, (1, 2)), (2, (1, 3)), (3, (2, 3))])
def test_saturated_rotor_pattern(orc, axis, up):
    """A large positive rate demand about one body axis from hover saturates the
    rotors whose Eq. (11) coefficient in that torque row is positive at T_max and
    the others at T_min (roll: rotors 2, 3; pitch: 2, 4; yaw: 3, 4, zero-based
    indices in `up`).  The expectation is read off the printed matrix by hand, not
    computed by the oracle."""
    veh = W.vehicle_benchmark()
    x = hover_state(veh)
    u = np.array([veh["mass"] * veh["g"], 0.0, 0.0, 0.0])
    u[axis] = 400.0                                   # rad/s: far beyond what 8 N rotors give
    T = orc.controller(veh, x, u, 0.01)
    want = np.full(4, veh["T_min"])
    want[list(up)] = veh["T_max"]
    np.testing.assert_array_equal(T, want)
    # and the same demand negated swaps the two pairs
    u[axis] = -400.0
    T = orc.controller(veh, x, u, 0.01)
    want = np.full(4, veh["T_max"])
    want[list(up)] = veh["T_min"]
    np.testing.assert_array_equal(T, want)


def test_saturated_controller_from_printed_matrix(orc):
    """Eq. (12) with partial saturation at a spinning, tilted state: the command is
    clip(Gamma^-1 [F; J wdot_d + w x J w]) with Gamma the printed matrix of Eq. (11)
    (numpy's solve of that matrix; the gyroscopic term written out), and the
    feasible input of Eqs. (13)-(15) is recomposed from it through the same printed
    matrix."""
    veh = W.vehicle_benchmark()
    veh.update(J=(0.012, 0.015, 0.021))
    G = printed_allocation(veh["arm_l"], veh["c_tf"])
    Jx, Jy, Jz = veh["J"]
    dt = 0.01
    rng = np.random.default_rng(11)
    n_partial = 0
    for _ in range(200):
        x = hover_state(veh)
        x[3:7] = quat_axis_angle(rng.normal(size=3), rng.uniform(0, 1))
        wx, wy, wz = rng.normal(0, 2, 3)
        x[10:13] = [wx, wy, wz]
        u = np.concatenate([[rng.uniform(2, 30)], rng.normal(0, 2, 3)])
        gyro = np.array([(Jz - Jy) * wy * wz, (Jx - Jz) * wz * wx, (Jy - Jx) * wx * wy])
        tau_d = np.array([Jx, Jy, Jz]) * (u[1:] - x[10:13]) / dt + gyro
        T_d = np.linalg.solve(G, np.concatenate([[u[0]], tau_d]))
        want = np.clip(T_d, veh["T_min"], veh["T_max"])
        T = orc.controller(veh, x, u, dt)
        np.testing.assert_allclose(T, want, rtol=1e-12, atol=1e-12)
        n_clip = int(np.sum((T_d < veh["T_min"]) | (T_d > veh["T_max"])))
        n_partial += 0 < n_clip < 4
        wrench = G @ want
        w_clip = x[10:13] + (wrench[1:] - gyro) / np.array([Jx, Jy, Jz]) * dt
        np.testing.assert_allclose(orc.applied_input(veh, x, u, dt),
                                   np.concatenate([[wrench[0]], w_clip]), rtol=1e-11, atol=1e-11)
    assert n_partial >= 10                            # saturation of some rotors, not all


# ---------------------------------------------------------------------------
# Controller, clipping and the feasible input (Eqs. (8)-(15))
# ---------------------------------------------------------------------------

def test_controller_unsaturated_reproduces_wrench(orc):
    """omega = 0: tau_d = J omega_d / dt; the rotor split re-composes [F; tau_d]."""
    veh = W.vehicle_benchmark()
    veh.update(T_min=-1e9, T_max=1e9)
    x = hover_state(veh)
    u = np.array([9.0, 0.3, -0.2, 0.1])
    dt = 0.01
    T = orc.controller(veh, x, u, dt)
    J = np.array(veh["J"])
    np.testing.assert_allclose(orc.allocation(veh) @ T, np.concatenate([[9.0], J * u[1:] / dt]),
                               rtol=1e-13, atol=1e-12)


def test_controller_gyroscopic_term(orc):
    """omega = (a, b, 0) with Jx != Jy: omega x J omega = (0, 0, a b (Jy - Jx))."""
    veh = W.vehicle_benchmark()
    veh.update(J=(0.01, 0.03, 0.02), T_min=-1e9, T_max=1e9, k_rate=50.0)
    a, b = 0.7, -1.3
    x = hover_state(veh)
    x[10:13] = [a, b, 0.0]
    u = np.array([8.0, a, b, 0.0])                  # omega_d = omega -> no rate demand
    T = orc.controller(veh, x, u, 0.01)
    wrench = orc.allocation(veh) @ T
    np.testing.assert_allclose(wrench, [8.0, 0.0, 0.0, a * b * (0.03 - 0.01)], atol=1e-12)


def test_controller_clips_to_rotor_limits(orc):
    """Eq. (12): the command is the element-wise clip of Gamma^-1 [F; tau_d]."""
    veh = W.vehicle_benchmark()
    x = hover_state(veh)
    dt = 0.01
    rng = np.random.default_rng(0)
    J = np.array(veh["J"])
    for _ in range(50):
        u = np.concatenate([[rng.uniform(0, 40)], rng.normal(0, 3, 3)])
        T = orc.controller(veh, x, u, dt)
        want = np.clip(np.linalg.solve(orc.allocation(veh), np.concatenate([[u[0]], J * u[1:] / dt])),
                       veh["T_min"], veh["T_max"])
        np.testing.assert_allclose(T, want, rtol=1e-12, atol=1e-12)


def test_feasible_input_unsaturated_is_deadbeat(orc):
    """Eqs. (14)-(15): without saturation omega_clip = omega_d and F_clip = F_t."""
    veh = W.vehicle_benchmark()
    veh.update(T_min=-1e9, T_max=1e9)
    x = hover_state(veh)
    x[10:13] = [0.2, -0.1, 0.3]
    u = np.array([10.0, 0.5, 0.4, -0.2])
    out = orc.applied_input(veh, x, u, 0.01)
    np.testing.assert_allclose(out, u, rtol=1e-12, atol=1e-12)


def test_feasible_input_saturated(orc):
    """Saturated: F_clip is the sum of the clipped thrusts and the rate limits
    clamp only the body rates sent out."""
    veh = W.vehicle_benchmark()
    veh.update(w_xy_max=0.5, w_z_max=0.1)
    x = hover_state(veh)
    u = np.array([40.0, 30.0, -30.0, 5.0])
    T = orc.controller(veh, x, u, 0.01)
    out = orc.applied_input(veh, x, u, 0.01)
    assert out[0] == pytest.approx(T.sum(), rel=1e-14)
    assert abs(out[1]) <= 0.5 and abs(out[2]) <= 0.5 and abs(out[3]) <= 0.1


# ---------------------------------------------------------------------------
# P3-P8, P13: dynamics and integration (Eq. (6), Eq. (2))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("tau_m", [0.0, 0.03])
def test_hover_is_an_equilibrium(orc, tau_m):
    veh = W.vehicle_benchmark()
    veh["tau_m"] = tau_m
    x = hover_state(veh, p=(1.0, -2.0, 3.0))
    u = W.hover_control(veh)
    x0 = x.copy()
    for _ in range(200):
        x = orc.model_step(veh, x, u, 0.01)
    np.testing.assert_allclose(x, x0, atol=1e-12)


def test_free_fall(orc):
    """Zero thrust: p(t) = p0 + v0 t - g t^2 / 2 e_z, exact for RK4."""
    veh = W.vehicle_benchmark()
    x = hover_state(veh)
    x[7:10] = [1.0, -2.0, 0.5]
    x[13:17] = 0.0
    dt, n = 0.01, 50
    for _ in range(n):
        x = orc.rk4_step(veh, x, np.zeros(4), dt)
    t = n * dt
    np.testing.assert_allclose(x[0:3], np.array([1.0, -2.0, 0.5]) * t + [0, 0, -0.5 * 9.81 * t * t],
                               atol=1e-12)
    np.testing.assert_allclose(x[7:10], [1.0, -2.0, 0.5 - 9.81 * t], atol=1e-12)


def test_tilted_thrust_direction(orc):
    """Roll by phi about body x tilts the thrust towards -y (R(q) body to world):
    a = (0, -F sin(phi) / m, F cos(phi) / m - g), constant over the step."""
    veh = W.vehicle_benchmark()
    veh["tau_m"] = 0.0
    phi, F = 0.3, 12.0
    x = hover_state(veh)
    x[3:7] = quat_axis_angle([1, 0, 0], phi)
    dt = 0.02
    x1 = orc.rk4_step(veh, x, np.full(4, F / 4), dt)
    a = np.array([0.0, -F * math.sin(phi), F * math.cos(phi)]) / veh["mass"] - [0, 0, 9.81]
    np.testing.assert_allclose(x1[7:10], a * dt, atol=1e-13)
    np.testing.assert_allclose(x1[0:3], 0.5 * a * dt * dt, atol=1e-13)
    # yaw does not change where the thrust points; pitch theta tilts it to +x
    x[3:7] = qmul(quat_axis_angle([0, 0, 1], 0.7), quat_axis_angle([0, 1, 0], phi))
    x1 = orc.rk4_step(veh, x, np.full(4, F / 4), dt)
    zb = F / veh["mass"] * np.array([math.cos(0.7) * math.sin(phi), math.sin(0.7) * math.sin(phi),
                                     math.cos(phi)])
    np.testing.assert_allclose(x1[7:10], (zb - [0, 0, 9.81]) * dt, atol=1e-13)


def test_torque_free_spin_about_body_axes(orc):
    """omega on a principal axis stays constant and q(t) = q0 (x) exp(omega t / 2)
    (body-frame rates, Hamilton product q (x) [0, omega]).  Error per step is
    O((Omega dt)^5)."""
    veh = W.vehicle_benchmark()
    veh["tau_m"] = 0.0
    dt, n, Om = 0.01, 100, 2.0
    T = np.full(4, 2.5)                               # equal thrusts: zero torque
    q0 = quat_axis_angle([0, 0, 1], math.pi / 2)
    for axis in ([0, 0, 1], [1, 0, 0]):
        x = hover_state(veh)
        x[3:7] = q0
        x[10:13] = Om * np.array(axis, float)
        for _ in range(n):
            x = orc.rk4_step(veh, x, T, dt)
        want = qmul(q0, quat_axis_angle(axis, Om * n * dt))
        np.testing.assert_allclose(x[3:7], want, atol=1e-9)
        np.testing.assert_allclose(x[10:13], Om * np.array(axis, float), atol=1e-14)


def test_torque_free_rigid_body_invariants(orc):
    """Asymmetric body, no torque: world-frame angular momentum R(q) J omega and the
    kinetic energy omega^T J omega / 2 are conserved (Euler's equations, Eq. (6))."""
    from scipy.spatial.transform import Rotation
    veh = W.vehicle_benchmark()
    veh.update(J=(0.01, 0.02, 0.03), tau_m=0.0)
    J = np.array(veh["J"])
    x = hover_state(veh)
    x[10:13] = [3.0, 0.5, -1.0]
    x[3:7] = quat_axis_angle([1, 2, 3], 0.4)

    def invariants(x):
        q = x[3:7]
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        return Rm @ (J * x[10:13]), 0.5 * np.dot(x[10:13], J * x[10:13])

    L0, E0 = invariants(x)
    for _ in range(500):
        x = orc.rk4_step(veh, x, np.full(4, 2.0), 0.002)
    L1, E1 = invariants(x)
    np.testing.assert_allclose(L1, L0, rtol=1e-8, atol=1e-10)
    assert E1 == pytest.approx(E0, rel=1e-8)


def test_rotor_lag_exact_rk4_factor(orc):
    """T' = (T_cmd - T)/tau: RK4 gives T1 = T_cmd + R(-dt/tau)(T0 - T_cmd) with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 (configs' 30 ms lag, held command)."""
    veh = W.vehicle_benchmark()
    x = hover_state(veh)
    x[13:17] = [1.0, 2.0, 3.0, 4.0]
    T_cmd = np.array([4.0, 0.5, 7.0, 3.0])
    z = -0.01 / 0.03
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    assert R == pytest.approx(0.7165638, abs=1e-7)
    x1 = orc.rk4_step(veh, x, T_cmd, 0.01)
    np.testing.assert_allclose(x1[13:17], T_cmd + R * (x[13:17] - T_cmd), rtol=1e-14)


def test_rate_controller_deadbeat_paper_model(orc):
    """Paper model (no lag), unsaturated, rates about z with Jx = Jy: one step of the
    P law omega_dot_d = (omega_d - omega)/dt lands exactly on omega_d."""
    veh = W.vehicle_paper()
    veh.update(T_min=-1e9, T_max=1e9)
    x = hover_state(veh)
    x[10:13] = [0.0, 0.0, 0.3]
    u = np.array([veh["mass"] * 9.81, 0.0, 0.0, -0.8])
    x1 = orc.model_step(veh, x, u, 0.01)
    np.testing.assert_allclose(x1[10:13], [0.0, 0.0, -0.8], atol=1e-12)


def test_quaternion_norm_preserved(orc):
    veh = W.vehicle_benchmark()
    rng = np.random.default_rng(3)
    x = hover_state(veh)
    for _ in range(300):
        u = np.concatenate([[rng.uniform(5, 15)], rng.normal(0, 2, 3)])
        x = orc.model_step(veh, x, u, 0.01)
        assert abs(np.linalg.norm(x[3:7]) - 1.0) < 1e-14


def test_rk4_is_fourth_order(orc):
    """Against a tight adaptive reference solution (scipy DOP853) of the same
    vector field, halving dt cuts the one-step error by about 2^5."""
    from scipy.integrate import solve_ivp
    veh = W.vehicle_benchmark()
    veh["J"] = (0.01, 0.015, 0.02)
    x0 = hover_state(veh)
    x0[3:7] = quat_axis_angle([1, 1, 0], 0.5)
    x0[7:13] = [1.0, -0.5, 0.2, 2.0, -1.0, 3.0]
    x0[13:17] = [1.0, 3.0, 2.0, 4.0]
    T_cmd = np.array([3.0, 1.0, 4.0, 2.0])

    def f(_t, y):
        return orc.dynamics(veh, y, T_cmd)

    errs = []
    for dt in (0.04, 0.02, 0.01):
        ref = solve_ivp(f, (0, dt), x0, method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
        ref[3:7] /= np.linalg.norm(ref[3:7])
        errs.append(np.max(np.abs(orc.rk4_step(veh, x0, T_cmd, dt) - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 20 < r1 < 45 and 20 < r2 < 45, errs


# ---------------------------------------------------------------------------
# P9, P14: cost terms (Eqs. (16)-(22))
# ---------------------------------------------------------------------------

def test_quaternion_distance(orc):
    """d(q, q) = d(q, -q) = 0 and d = 1 - <q1, q2>^2 = sin^2(theta/2), theta being
    the relative rotation angle (Eqs. (19)-(21))."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(5)
    for _ in range(100):
        r1, r2 = Rotation.random(random_state=rng), Rotation.random(random_state=rng)
        q1 = np.roll(r1.as_quat(), 1)
        q2 = np.roll(r2.as_quat(), 1)
        theta = (r1.inv() * r2).magnitude()
        assert orc.quat_distance(q1, q2) == pytest.approx(math.sin(theta / 2) ** 2, abs=1e-12)
        assert orc.quat_distance(q1, q1) == pytest.approx(0.0, abs=1e-15)
        assert orc.quat_distance(q1, -q1) == pytest.approx(0.0, abs=1e-15)


def test_tracking_cost_closed_forms(orc):
    cost = W.cost_benchmark()
    xr = np.concatenate([[1.0, 2.0, 3.0], [1.0, 0, 0, 0], [4.0, 5.0, 6.0], [0.1, 0.2, 0.3]])
    x = np.concatenate([xr, np.zeros(4)])
    assert orc.tracking_cost(cost, x, xr) == 0.0
    x2 = x.copy(); x2[0:3] += [0.3, -0.4, 1.2]
    assert orc.tracking_cost(cost, x2, xr) == pytest.approx(400.0 * 1.69, rel=1e-14)
    x2 = x.copy(); x2[7:10] += [1.0, 2.0, 2.0]
    assert orc.tracking_cost(cost, x2, xr) == pytest.approx(40.0 * 9.0, rel=1e-14)
    x2 = x.copy(); x2[10:13] -= [0.0, 3.0, 4.0]
    assert orc.tracking_cost(cost, x2, xr) == pytest.approx(20.0 * 25.0, rel=1e-14)
    theta = 0.8
    x2 = x.copy(); x2[3:7] = quat_axis_angle([0, 1, 1], theta)
    # attitude term is c_q d_q^2 with d_q = sin^2(theta/2)   (Eq. (18) with Eq. (21))
    assert orc.tracking_cost(cost, x2, xr) == pytest.approx(20.0 * math.sin(theta / 2) ** 4, rel=1e-12)


def test_obstacle_cost_closed_forms(orc):
    cost = W.cost_benchmark()
    r, m, w, col = 0.5, cost["obs_margin"], cost["obs_w"], cost["obs_collision"]
    sph = np.array([[W.SPHERE, 1.0, 2.0, 3.0, r]])
    c = np.array([1.0, 2.0, 3.0])
    u = np.array([2.0, -1.0, 2.0]) / 3.0
    assert orc.obstacle_cost(cost, c + (r + m) * u, sph) == pytest.approx(0.0, abs=1e-20)
    assert orc.obstacle_cost(cost, c + (r + m + 1.0) * u, sph) == 0.0
    eps = 0.01
    assert orc.obstacle_cost(cost, c + (r - eps) * u, sph) == pytest.approx(col + w * (m + eps) ** 2, rel=1e-12)
    assert orc.obstacle_cost(cost, c + (r + 0.1) * u, sph) == pytest.approx(w * (m - 0.1) ** 2, rel=1e-12)
    # vertical cylinder: height does not matter
    cyl = np.array([[W.VCYL, 1.0, 2.0, -50.0, r]])
    p = np.array([1.0 + 0.36, 2.0 + 0.48, 100.0])    # horizontal distance 0.6: inside the margin
    assert orc.obstacle_cost(cost, p, cyl) == pytest.approx(w * (r + m - 0.6) ** 2, rel=1e-12)
    p = np.array([1.0 + 0.3, 2.0 + 0.3, 100.0])
    d = math.hypot(0.3, 0.3)
    assert orc.obstacle_cost(cost, p, cyl) == pytest.approx(col + w * (r + m - d) ** 2, rel=1e-12)
    # inside two obstacles: the collision constant counts once (union), margins add
    both = np.vstack([sph, np.array([[W.SPHERE, 1.0, 2.0, 3.2, r]])])
    val = orc.obstacle_cost(cost, c, both)
    assert val == pytest.approx(col + w * ((r + m) ** 2 + (r + m - 0.2) ** 2), rel=1e-12)
    # paper form (Eq. (22)): indicator only
    paper = W.cost_paper()
    assert orc.obstacle_cost(paper, c, sph) == 1.0e6
    assert orc.obstacle_cost(paper, c + 0.6 * u, sph) == 0.0


def test_trajectory_cost_control_terms(orc):
    """Eq. (16): constant input costs N u^T R u; a ramp u_j = u0 + j a adds
    (N-1) a^T R_d a for the changes."""
    cost = W.cost_benchmark()
    N = 7
    xr = np.tile(np.concatenate([[0, 0, 0], [1.0, 0, 0, 0], np.zeros(6)]), (N + 1, 1))
    states = np.hstack([xr, np.zeros((N + 1, 4))])
    u0 = np.array([9.0, 0.5, -0.25, 1.0])
    R, Rd = np.array(cost["R"]), np.array(cost["R_d"])
    assert orc.trajectory_cost(cost, states, np.tile(u0, (N, 1)), xr) == pytest.approx(N * u0 @ (R * u0), rel=1e-13)
    a = np.array([0.1, -0.2, 0.3, 0.05])
    only_rd = dict(cost, R=(0, 0, 0, 0))
    ramp = u0 + np.arange(N)[:, None] * a
    assert orc.trajectory_cost(only_rd, states, ramp, xr) == pytest.approx((N - 1) * a @ (Rd * a), rel=1e-12)
    # sum_j (u0 + j a)^2 via power sums sum_j j and sum_j j^2
    s1, s2 = N * (N - 1) / 2, (N - 1) * N * (2 * N - 1) / 6
    want = np.sum(R * (N * u0 * u0 + 2 * u0 * a * s1 + a * a * s2)) + (N - 1) * a @ (Rd * a)
    assert orc.trajectory_cost(cost, states, ramp, xr) == pytest.approx(want, rel=1e-12)
    # every state j = 0..N is scored: offsetting one state's position adds c_p |dp|^2
    for j in (0, N):
        s2_ = states.copy(); s2_[j, 0] += 0.5
        only_track = dict(cost, R=(0, 0, 0, 0), R_d=(0, 0, 0, 0))
        assert orc.trajectory_cost(only_track, s2_, ramp, xr) == pytest.approx(400 * 0.25, rel=1e-13)


# ---------------------------------------------------------------------------
# P10: weights (Eq. (4)) and the update (Eq. (5))
# ---------------------------------------------------------------------------

def test_weights_properties(orc):
    rng = np.random.default_rng(0)
    S = rng.uniform(100, 200, 500)
    w, diag = orc.weights(S, 3.0)
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    assert diag[0] == S.min() and diag[3] == np.argmin(S)
    assert diag[2] == pytest.approx(1.0 / np.sum(w * w), rel=1e-14)
    w2, _ = orc.weights(S + 1e4, 3.0)                # shift invariance (rho subtraction)
    np.testing.assert_allclose(w2, w, rtol=1e-9, atol=1e-300)
    ref = np.exp(-(S - S.min()) / 3.0 - np.log(np.sum(np.exp(-(S - S.min()) / 3.0))))
    np.testing.assert_allclose(w, ref, rtol=1e-12)
    w0, _ = orc.weights(S, 1e-9)                     # lambda -> 0: one-hot at argmin
    assert w0[np.argmin(S)] == 1.0 and np.sum(w0) == 1.0
    wi, d = orc.weights(S, 1e12)                     # lambda -> inf: uniform, ESS = K
    np.testing.assert_allclose(wi, 1.0 / S.size, rtol=1e-9)
    assert d[2] == pytest.approx(S.size, rel=1e-8)


def test_weights_nonfinite_and_ties(orc):
    S = np.array([5.0, np.nan, 5.0, np.inf, 7.0])
    w, diag = orc.weights(S, 1e-12)
    np.testing.assert_array_equal(w, [0.5, 0.0, 0.5, 0.0, 0.0])   # ties share the limit
    with pytest.raises(FloatingPointError):
        orc.weights(np.array([np.nan, np.inf]), 1.0)


def test_weighted_update_limits(orc):
    rng = np.random.default_rng(1)
    K, N = 64, 5
    du = rng.normal(size=(K, N, 4))
    u = rng.normal(size=(N, 4))
    np.testing.assert_allclose(orc.weighted_update(np.full(K, 1.0 / K), du, u), u + du.mean(axis=0),
                               rtol=1e-13, atol=1e-14)
    onehot = np.zeros(K); onehot[17] = 1.0
    np.testing.assert_array_equal(orc.weighted_update(onehot, du, u), u + du[17])


def test_apply_and_shift(orc):
    veh = W.vehicle_benchmark()
    N = 6
    u = np.arange(N * 4, dtype=float).reshape(N, 4)
    u_init = np.array([9.81, 0, 0, 0])
    ua, us = orc.apply_shift(veh, 0.01, hover_state(veh), u, u_init)
    np.testing.assert_array_equal(ua[:4], u[0])
    np.testing.assert_array_equal(us[:-1], u[1:])
    np.testing.assert_array_equal(us[-1], u_init)


def test_update_single_sample_is_brute_force(orc):
    """K = 1: the weight is 1, so the new sequence is u_nom + du^1, shifted."""
    sc = W.c1_plain(K=1, N=6)
    s = sc.solve(3)
    r = orc.update(sc.veh, sc.cost, s, sc.x0, sc.u_nom0(), sc.x_ref(3))
    du = orc.noise(1, 6, s["sigma"], s["seed"], s["vehicle_id"], s["t"])[0]
    new = sc.u_nom0() + du
    np.testing.assert_array_equal(r["w"], [1.0])
    np.testing.assert_allclose(r["u_apply"][:4], new[0], rtol=1e-15)
    np.testing.assert_allclose(r["u_nom"][:-1], new[1:], rtol=1e-15)
    np.testing.assert_array_equal(r["u_nom"][-1], sc.u_init)


def test_zero_noise_rollouts_are_deterministic(orc):
    """sigma = 0: every rollout is the noise-free integration of u_nom, every weight
    is 1/K exactly and the update leaves u_nom unchanged before the shift."""
    sc = W.c2_line(K=16, N=12)
    s = sc.solve(0); s["sigma"] = np.zeros(4)
    un = sc.u_nom0() + np.linspace(0, 1, 12)[:, None] * [0.5, 0.1, -0.1, 0.05]
    states, du, S = orc.rollouts(sc.veh, sc.cost, s, sc.x0, un, sc.x_ref(0), sc.obstacles, True)
    assert np.all(du == 0.0) and np.all(S == S[0])
    x = sc.x0.copy()
    for j in range(12):
        x = orc.model_step(sc.veh, x, un[j], sc.dt)
        np.testing.assert_array_equal(states[:, j + 1], np.tile(x, (16, 1)))
    r = orc.update(sc.veh, sc.cost, s, sc.x0, un, sc.x_ref(0), sc.obstacles)
    np.testing.assert_array_equal(r["w"], np.full(16, 1.0 / 16))
    np.testing.assert_array_equal(r["u_apply"][:4], un[0])
    np.testing.assert_array_equal(r["u_nom"][:-1], un[1:])


def test_rollout_uses_its_own_noise_and_cost(orc):
    """Each rollout's cost equals the trajectory cost of its own perturbed inputs
    and states (Eq. (3)), and its first state is the estimate x_hat."""
    sc = W.c2_line(K=6, N=9)
    s = sc.solve(2)
    states, du, S = orc.rollouts(sc.veh, sc.cost, s, sc.x0, sc.u_nom0(), sc.x_ref(2), sc.obstacles, True)
    np.testing.assert_array_equal(du, orc.noise(6, 9, s["sigma"], s["seed"], 0, 2))
    for k in range(6):
        np.testing.assert_array_equal(states[k, 0], sc.x0)
        uk = sc.u_nom0() + du[k]
        assert S[k] == orc.trajectory_cost(sc.cost, states[k], uk, sc.x_ref(2), sc.obstacles)
        x = sc.x0.copy()
        for j in range(9):
            x = orc.model_step(sc.veh, x, uk[j], sc.dt)
        np.testing.assert_array_equal(states[k, -1], x)


# ---------------------------------------------------------------------------
# Control input interpolation (Sec. IV-B) and delay compensation (Sec. IV-E)
# ---------------------------------------------------------------------------

def test_advance_by_a_whole_step_is_the_shift(orc):
    """alpha = 1 is Algorithm 1's shift: u_j <- u_{j+1}, u_{N-1} <- u_init, exactly."""
    rng = np.random.default_rng(7)
    u, ui = rng.normal(size=(9, 4)), rng.normal(size=4)
    np.testing.assert_array_equal(orc.advance(u, ui, 1.0), np.vstack([u[1:], ui]))


@pytest.mark.parametrize("alpha", [0.1, 0.25, 0.5, 0.999])
def test_advance_is_linear_interpolation(orc, alpha):
    """Knot j takes the value at j + alpha of the piecewise-linear interpolant through
    u_0..u_{N-1}, u_N = u_init (numpy.interp per input dimension)."""
    rng = np.random.default_rng(8)
    N = 15
    u, ui = rng.normal(size=(N, 4)), rng.normal(size=4)
    knots = np.vstack([u, ui])
    want = np.stack([np.interp(np.arange(N) + alpha, np.arange(N + 1), knots[:, d])
                     for d in range(4)], axis=1)
    np.testing.assert_allclose(orc.advance(u, ui, alpha), want, rtol=0, atol=1e-14)


def test_advance_of_a_linear_sequence_is_exact(orc):
    """A sequence linear in j (continued by u_init) moves along its line, and n
    advances by 1/n equal one whole shift on the knots that the fixed refill u_init
    has not reached (each advance carries its influence one knot back)."""
    N, n = 30, 10
    a, b = np.array([9.0, 0.3, -0.2, 0.1]), np.array([0.5, -0.05, 0.02, 0.01])
    u = a + b * np.arange(N)[:, None]
    ui = a + b * N
    np.testing.assert_allclose(orc.advance(u, ui, 0.3), a + b * (np.arange(N)[:, None] + 0.3),
                               atol=1e-13)
    v = u.copy()
    for _ in range(n):
        v = orc.advance(v, ui, 1.0 / n)
    np.testing.assert_allclose(v[:N - n + 1], u[1:N - n + 2], atol=1e-12)
    assert np.abs(v[-1] - ui).max() > 1e-3          # the refill is approached, not reached


def test_update_with_interpolation(orc):
    """dt_ctrl = dt / 10: the same update, then an advance by 1/10 of a step instead
    of the shift; u_apply is unchanged."""
    sc = W.c2_line(K=32, N=15)
    s = sc.solve(1)
    un = sc.u_nom0() + np.linspace(0, 1, 15)[:, None] * [0.5, 0.1, -0.1, 0.05]
    r1 = orc.update(sc.veh, sc.cost, s, sc.x0, un, sc.x_ref(1), sc.obstacles)
    s2 = dict(s, dt_ctrl=sc.dt / 10)
    r2 = orc.update(sc.veh, sc.cost, s2, sc.x0, un, sc.x_ref(1), sc.obstacles)
    np.testing.assert_array_equal(r1["u_apply"], r2["u_apply"])
    updated = orc.weighted_update(r1["w"], r1["du"], un)
    np.testing.assert_allclose(r1["u_nom"], np.vstack([updated[1:], sc.u_init]), rtol=1e-15)
    np.testing.assert_allclose(r2["u_nom"], 0.9 * updated + 0.1 * np.vstack([updated[1:], sc.u_init]),
                               rtol=1e-14, atol=1e-14)


def test_predict_zero_delay_and_one_step(orc):
    """No delay returns the estimate; a delay of one step dt is one model step."""
    veh = W.vehicle_benchmark()
    rng = np.random.default_rng(9)
    x = hover_state(veh, p=(1.0, 2.0, 3.0))
    x[3:7] = quat_axis_angle(rng.normal(size=3), 0.4)
    x[7:13] = rng.normal(size=6)
    u = np.array([11.0, 0.4, -0.3, 0.2])
    np.testing.assert_array_equal(orc.predict(veh, 0.01, 0.0, x, u), x)
    np.testing.assert_array_equal(orc.predict(veh, 0.01, 0.01, x, u), orc.model_step(veh, x, u, 0.01))


@pytest.mark.parametrize("tau_m", [0.0, 0.03])
def test_predict_hover_and_free_fall(orc, tau_m):
    """Hover is kept over any delay; zero thrust falls as p0 + v0 t - g t^2 / 2 e_z
    over several sub-steps (exact for RK4), spinning freely about body z with
    q(t) = q0 (x) exp(Omega t / 2) when J_x = J_y."""
    veh = W.vehicle_benchmark()
    veh["tau_m"] = tau_m
    x = hover_state(veh, p=(0.5, 0.0, 2.0))
    np.testing.assert_allclose(orc.predict(veh, 0.01, 0.037, x, W.hover_control(veh)), x, atol=1e-13)
    Om, t = 3.0, 0.025                                   # 3 sub-steps of t / 3
    x[7:10] = [1.0, -2.0, 0.5]
    x[10:13] = [0.0, 0.0, Om]
    x[13:17] = 0.0
    y = orc.predict(veh, 0.01, t, x, [0.0, 0.0, 0.0, Om])
    np.testing.assert_allclose(y[0:3], x[0:3] + x[7:10] * t - [0, 0, 0.5 * 9.81 * t * t], atol=1e-13)
    np.testing.assert_allclose(y[7:10], x[7:10] - [0, 0, 9.81 * t], atol=1e-13)
    np.testing.assert_allclose(y[3:7], quat_axis_angle([0, 0, 1], Om * t), atol=1e-10)
    np.testing.assert_allclose(y[10:17], x[10:17], atol=1e-13)
