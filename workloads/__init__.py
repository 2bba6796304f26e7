"""Seeded synthetic inputs for the MPPI update (arXiv 2407.09812).

This module produces *inputs only* -- vehicle and cost parameters, state estimates,
reference trajectories, obstacle sets, batch and arrival mixes -- shared by the FP64
oracle and the GPU path.  It holds none of the method's arithmetic (no sampling,
dynamics, cost, weights or update).  The paper flies on the MRS simulator with
MPC-generated references and hand-built scenes, none of which is available; the
generators below stand in for them with the shapes, speeds and obstacle densities
of the benchmark configurations.

Layouts: state (17) = [p(3), q(4) w-first, v(3), omega(3), T(4)];
reference rows (13) = [p, q, v, omega]; obstacle rows (5) = [type, cx, cy, cz, r]
(type 0 = sphere, 1 = vertical cylinder); control (4) = [F_t, omega_d(3)].
"""
from __future__ import annotations

import math

import numpy as np

SPHERE, VCYL = 0, 1
G = 9.81


# ---------------------------------------------------------------------------
# Parameter presets
# ---------------------------------------------------------------------------

def vehicle_benchmark() -> dict:
    """Vehicle of the benchmark configurations: 1 kg, J = diag(0.01, 0.01, 0.02),
    rotor limits [0, 8] N with a 30 ms first-order lag; arm length and torque
    constant from the paper's Table I."""
    return dict(mass=1.0, J=(0.01, 0.01, 0.02), arm_l=0.15, c_tf=0.012, g=G,
                T_min=0.0, T_max=8.0, tau_m=0.03, k_rate=0.0, w_xy_max=0.0, w_z_max=0.0)


def vehicle_paper(real: bool = False) -> dict:
    """The paper's vehicle (Table I): algebraic rotor model (no lag)."""
    return dict(mass=1.21, J=(7.06e-3, 7.06e-3, 13.6e-3), arm_l=0.15, c_tf=0.012, g=G,
                T_min=0.3, T_max=8.0 if real else 19.0, tau_m=0.0, k_rate=0.0,
                w_xy_max=6.0 if real else 10.0, w_z_max=0.5 if real else 2.0)


def cost_benchmark() -> dict:
    """Table II tracking and input weights; obstacle margin 0.3 m, quadratic
    margin weight 1e3 and collision constant 1e4."""
    return dict(c_p=400.0, c_v=40.0, c_q=20.0, c_w=20.0,
                R=(0.01, 0.05, 0.05, 0.10), R_d=(0.05, 0.10, 0.10, 0.30),
                obs_margin=0.3, obs_w=1.0e3, obs_collision=1.0e4)


def cost_paper() -> dict:
    """Table II weights with the paper's indicator-only obstacle term (c_obs = 1e6)."""
    c = cost_benchmark()
    c.update(obs_margin=0.0, obs_w=0.0, obs_collision=1.0e6)
    return c


def hover_control(veh: dict) -> np.ndarray:
    """u_init: zero body rates and the collective thrust that holds hover."""
    return np.array([veh["mass"] * veh["g"], 0.0, 0.0, 0.0])


# ---------------------------------------------------------------------------
# Rotations used to build references (not part of the method), vectorised
# ---------------------------------------------------------------------------

def _quats_from_frames(xb, yb, zb):
    """Unit quaternions [n, 4] (w first, w >= 0) of the rotation matrices whose
    columns are xb, yb, zb [n, 3] (Shepperd's method, best-conditioned branch)."""
    R = np.stack([xb, yb, zb], axis=2)                 # R[:, i, j] = column j, row i
    r00, r11, r22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    t = np.stack([1 + r00 + r11 + r22, 1 + r00 - r11 - r22,
                  1 - r00 + r11 - r22, 1 - r00 - r11 + r22], axis=1)
    k = np.argmax(t, axis=1)
    s = 2.0 * np.sqrt(np.maximum(t[np.arange(len(k)), k], 1e-300))
    q = np.empty((len(k), 4))
    d21, d02, d10 = R[:, 2, 1] - R[:, 1, 2], R[:, 0, 2] - R[:, 2, 0], R[:, 1, 0] - R[:, 0, 1]
    s01, s02, s12 = R[:, 0, 1] + R[:, 1, 0], R[:, 0, 2] + R[:, 2, 0], R[:, 1, 2] + R[:, 2, 1]
    cases = [np.stack([0.25 * s, d21 / s, d02 / s, d10 / s], 1),
             np.stack([d21 / s, 0.25 * s, s01 / s, s02 / s], 1),
             np.stack([d02 / s, s01 / s, 0.25 * s, s12 / s], 1),
             np.stack([d10 / s, s02 / s, s12 / s, 0.25 * s], 1)]
    for c in range(4):
        q[k == c] = cases[c][k == c]
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return np.where(q[:, :1] < 0.0, -q, q)


def _attitudes(acc: np.ndarray, yaw: float = 0.0) -> np.ndarray:
    """Differential flatness: body z along acc + g e_z, heading `yaw` ([n, 3] -> [n, 4])."""
    zb = acc + np.array([0.0, 0.0, G])
    zb = zb / np.linalg.norm(zb, axis=1, keepdims=True)
    xc = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    yb = np.cross(zb, xc)
    yb /= np.linalg.norm(yb, axis=1, keepdims=True)
    xb = np.cross(yb, zb)
    return _quats_from_frames(xb, yb, zb)


def _body_rates(q_prev, q_next, h):
    """Body rates [n, 3] carrying q_prev to q_next over time h (finite difference)."""
    w1, v1 = q_prev[:, 0], -q_prev[:, 1:]
    w2, v2 = q_next[:, 0], q_next[:, 1:]
    dw = w1 * w2 - np.sum(v1 * v2, axis=1)
    dv = w1[:, None] * v2 + w2[:, None] * v1 + np.cross(v1, v2)
    sign = np.where(dw < 0.0, -1.0, 1.0)
    dw, dv = dw * sign, dv * sign[:, None]
    n = np.linalg.norm(dv, axis=1)
    ang = 2.0 * np.arctan2(n, dw)
    scale = np.where(n < 1e-15, 0.0, ang / np.maximum(n, 1e-300) / h)
    return dv * scale[:, None]


# ---------------------------------------------------------------------------
# References: rows for times t0 + j*dt, j = 0..N
# ---------------------------------------------------------------------------

class Reference:
    """Position, velocity and acceleration as functions of time (vectorised over
    an array of times); attitude by differential flatness with zero yaw, body rates
    by central differences of the attitude."""

    def pva(self, tau: np.ndarray):
        raise NotImplementedError

    def yaw(self) -> float:
        return 0.0

    def rows_at(self, taus, h: float = 1e-3) -> np.ndarray:
        taus = np.asarray(taus, dtype=np.float64)
        p, v, a = self.pva(taus)
        q = _attitudes(a, self.yaw())
        q_prev = _attitudes(self.pva(taus - h)[2], self.yaw())
        q_next = _attitudes(self.pva(taus + h)[2], self.yaw())
        w = _body_rates(q_prev, q_next, 2.0 * h)
        return np.concatenate([p, q, v, w], axis=1)

    def row(self, tau: float) -> np.ndarray:
        return self.rows_at([tau])[0]

    def rows(self, t0: float, N: int, dt: float) -> np.ndarray:
        return self.rows_at(t0 + dt * np.arange(N + 1))

    def thrust(self, tau: float, mass: float) -> float:
        a = self.pva(np.array([tau]))[2][0]
        return mass * float(np.linalg.norm(a + np.array([0.0, 0.0, G])))


class PointReference(Reference):
    def __init__(self, point):
        self.point = np.asarray(point, dtype=np.float64)

    def pva(self, tau):
        n = np.size(tau)
        return np.tile(self.point, (n, 1)), np.zeros((n, 3)), np.zeros((n, 3))


class LineReference(Reference):
    def __init__(self, start, velocity):
        self.start = np.asarray(start, dtype=np.float64)
        self.vel = np.asarray(velocity, dtype=np.float64)

    def pva(self, tau):
        tau = np.atleast_1d(tau)[:, None]
        return self.start + self.vel * tau, np.tile(self.vel, (tau.shape[0], 1)), \
            np.zeros((tau.shape[0], 3))


class CircleReference(Reference):
    def __init__(self, centre, radius, speed, phase=0.0):
        self.c = np.asarray(centre, dtype=np.float64)
        self.r = float(radius)
        self.om = float(speed) / float(radius)
        self.phase = float(phase)

    def pva(self, tau):
        a = self.phase + self.om * np.atleast_1d(tau)
        ca, sa, z = np.cos(a), np.sin(a), np.zeros_like(a)
        p = self.c + self.r * np.stack([ca, sa, z], 1)
        v = self.r * self.om * np.stack([-sa, ca, z], 1)
        acc = -self.r * self.om ** 2 * np.stack([ca, sa, z], 1)
        return p, v, acc


class SlantedCircleReference(Reference):
    """Circle in a plane tilted by `tilt` about the world x axis:
    p = c + r (cos a, sin a cos(tilt), sin a sin(tilt)), a = phase + (v / r) t."""

    def __init__(self, centre, radius, speed, tilt, phase=0.0):
        self.c = np.asarray(centre, dtype=np.float64)
        self.r = float(radius)
        self.om = float(speed) / float(radius)
        self.ct, self.st = math.cos(tilt), math.sin(tilt)
        self.phase = float(phase)

    def pva(self, tau):
        a = self.phase + self.om * np.atleast_1d(tau)
        ca, sa = np.cos(a), np.sin(a)
        p = self.c + self.r * np.stack([ca, sa * self.ct, sa * self.st], 1)
        v = self.r * self.om * np.stack([-sa, ca * self.ct, ca * self.st], 1)
        acc = -self.r * self.om ** 2 * np.stack([ca, sa * self.ct, sa * self.st], 1)
        return p, v, acc


def state_on_reference(ref: Reference, tau: float, veh: dict) -> np.ndarray:
    """A state estimate sitting on the reference, rotors at the reference thrust."""
    row = ref.row(tau)
    T = ref.thrust(tau, veh["mass"]) / 4.0
    return np.concatenate([row, np.full(4, T)])


# ---------------------------------------------------------------------------
# Obstacles
# ---------------------------------------------------------------------------

def spheres_in_box(rng: np.random.Generator, M: int, lo, hi, r_lo=0.3, r_hi=1.0) -> np.ndarray:
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    c = rng.uniform(lo, hi, size=(M, 3))
    r = rng.uniform(r_lo, r_hi, size=M)
    return np.column_stack([np.full(M, SPHERE), c, r]).astype(np.float64)


def cylinders_off_circle(rng: np.random.Generator, M: int, area_lo, area_hi, centre, radius,
                         r_lo=0.2, r_hi=0.6, clearance=1.0) -> np.ndarray:
    """Vertical cylinders uniform in an area, rejected while they lie on the circle."""
    out = []
    centre = np.asarray(centre, float)
    while len(out) < M:
        cxy = rng.uniform(area_lo, area_hi, size=2)
        r = rng.uniform(r_lo, r_hi)
        if abs(np.linalg.norm(cxy - centre[:2]) - radius) < r + clearance:
            continue
        out.append([VCYL, cxy[0], cxy[1], 0.0, r])
    return np.array(out, dtype=np.float64).reshape(-1, 5)


def cylinders_off_path(rng: np.random.Generator, M: int, area_lo, area_hi, path_xy,
                       r_lo=0.2, r_hi=0.6, clearance=1.0) -> np.ndarray:
    """Vertical cylinders uniform in an area, rejected while closer than r + clearance
    to any of the path's sampled xy points."""
    out = []
    path_xy = np.asarray(path_xy, float)
    while len(out) < M:
        cxy = rng.uniform(area_lo, area_hi, size=2)
        r = rng.uniform(r_lo, r_hi)
        if np.min(np.linalg.norm(path_xy - cxy, axis=1)) < r + clearance:
            continue
        out.append([VCYL, cxy[0], cxy[1], 0.0, r])
    return np.array(out, dtype=np.float64).reshape(-1, 5)


# ---------------------------------------------------------------------------
# Benchmark configurations
# ---------------------------------------------------------------------------

class Scenario:
    """One vehicle's MPPI problem: parameters, reference, obstacles, start."""

    def __init__(self, name, veh, cost, K, N, dt, lam, sigma, seed, vehicle_id, ref, obstacles,
                 updates, x0=None, dt_ctrl=0.0):
        self.name, self.veh, self.cost = name, veh, cost
        self.K, self.N, self.dt, self.lam = int(K), int(N), float(dt), float(lam)
        self.dt_ctrl = float(dt_ctrl)            # time between updates; 0: dt
        self.sigma = np.asarray(sigma, dtype=np.float64)
        self.seed, self.vehicle_id = int(seed), int(vehicle_id)
        self.ref = ref
        self.obstacles = np.asarray(obstacles, dtype=np.float64).reshape(-1, 5)
        self.updates = int(updates)
        self.x0 = state_on_reference(ref, 0.0, veh) if x0 is None else np.asarray(x0, float)
        self.u_init = hover_control(veh)

    @property
    def M(self):
        return self.obstacles.shape[0]

    @property
    def period(self) -> float:
        """Time between consecutive updates (the closed loop's plant step)."""
        return self.dt_ctrl if self.dt_ctrl > 0 else self.dt

    def solve(self, t: int = 0) -> dict:
        return dict(K=self.K, N=self.N, dt=self.dt, lam=self.lam, sigma=self.sigma,
                    seed=self.seed, vehicle_id=self.vehicle_id, t=int(t), u_init=self.u_init,
                    dt_ctrl=self.dt_ctrl)

    def x_ref(self, t: int = 0) -> np.ndarray:
        """Reference rows at the prediction steps from the time of update t."""
        return self.ref.rows(t * self.period, self.N, self.dt)

    def u_nom0(self) -> np.ndarray:
        return np.tile(self.u_init, (self.N, 1))


def c1_plain(K=256, N=20) -> Scenario:
    """Hover-to-point 2 m away, no obstacles, 50 closed-loop updates, seed 0."""
    veh = vehicle_benchmark()
    x0 = np.concatenate([np.zeros(3), [1.0, 0, 0, 0], np.zeros(6),
                         np.full(4, veh["mass"] * veh["g"] / 4.0)])
    return Scenario("c1_plain", veh, cost_benchmark(), K, N, 0.01, 1.0, (1.0, 1.0, 1.0, 1.0),
                    seed=0, vehicle_id=0, ref=PointReference([2.0, 0.0, 0.0]),
                    obstacles=np.zeros((0, 5)), updates=50, x0=x0)


def c2_line(K=4096, N=100, seed=2) -> Scenario:
    """Straight line at 12 m/s with 20 spheres in a 20 x 20 x 5 m box."""
    rng = np.random.default_rng(seed)
    obs = spheres_in_box(rng, 20, (0.0, -10.0, 0.0), (20.0, 10.0, 5.0))
    ref = LineReference([0.0, 0.0, 2.5], [12.0, 0.0, 0.0])
    return Scenario("c2_line", vehicle_benchmark(), cost_benchmark(), K, N, 0.01, 1.0,
                    (1.0, 1.0, 1.0, 1.0), seed=seed, vehicle_id=0, ref=ref, obstacles=obs,
                    updates=200)


def c3_agile(K=16384, N=200, seed=3) -> Scenario:
    """Circle of radius 8 m at 12.2 m/s (about 19 m/s^2) with 200 vertical cylinders
    in a 30 x 30 m area, rejected near the circle."""
    rng = np.random.default_rng(seed)
    centre = (15.0, 15.0, 2.0)
    obs = cylinders_off_circle(rng, 200, 0.0, 30.0, centre, 8.0)
    ref = CircleReference(centre, 8.0, 12.2)
    return Scenario("c3_agile", vehicle_benchmark(), cost_benchmark(), K, N, 0.01, 1.0,
                    (1.0, 1.0, 1.0, 1.0), seed=seed, vehicle_id=0, ref=ref, obstacles=obs,
                    updates=200)


def paper_preset(K=896, N=15, seed=6) -> Scenario:
    """The paper's own setting: Table I vehicle (simulation limits, no rotor lag),
    Table II parameters (prediction step 0.1 s, K = 896, N = 15, lambda = 1e-4,
    Sigma = diag(0.60, 0.15, 0.15, 0.05) read as variances), updates every 10 ms with
    the warm start advanced by interpolation (Sec. IV-B, n = 10), and the
    indicator-only obstacle cost with c_obs = 1e6 (Sec. IV-D).  The path is a circle
    of radius 6.04 m tilted by 30 degrees at 5.65 m/s (5.29 m/s^2, the speed and
    acceleration of the slanted-circle trajectory in Table III) among 40 pillar-like
    vertical cylinders kept 1 m off its ground track."""
    rng = np.random.default_rng(seed)
    centre = (0.0, 0.0, 4.0)
    ref = SlantedCircleReference(centre, 6.04, 5.65, math.radians(30.0))
    track = ref.pva(np.linspace(0.0, 2 * math.pi / ref.om, 400))[0][:, :2]
    obs = cylinders_off_path(rng, 40, -12.0, 12.0, track, r_lo=0.3, r_hi=0.8)
    veh = vehicle_paper()
    return Scenario("paper_preset", veh, cost_paper(), K, N, 0.1, 1e-4,
                    np.sqrt([0.60, 0.15, 0.15, 0.05]), seed=seed, vehicle_id=0, ref=ref,
                    obstacles=obs, updates=300, dt_ctrl=0.01)


K_SET = (1024, 2048, 4096, 8192, 16384)


def random_vehicle(rng: np.random.Generator, vehicle_id: int, seed: int,
                   K=None, N=None, M=None) -> Scenario:
    """One vehicle of the batched/served mixes: K from the power-of-two set,
    N uniform in [50, 200], a random line or circle at U[2, 12] m/s, and 0-200
    spheres placed around its start."""
    K = int(rng.choice(K_SET)) if K is None else int(K)
    N = int(rng.integers(50, 201)) if N is None else int(N)
    M = int(rng.integers(0, 201)) if M is None else int(M)
    speed = rng.uniform(2.0, 12.0)
    heading = rng.uniform(0.0, 2.0 * math.pi)
    start = np.array([rng.uniform(-50, 50), rng.uniform(-50, 50), rng.uniform(1.0, 5.0)])
    if rng.uniform() < 0.5:
        ref = LineReference(start, speed * np.array([math.cos(heading), math.sin(heading), 0.0]))
    else:
        radius = max(rng.uniform(4.0, 10.0), speed * speed / 19.0)
        centre = start - radius * np.array([math.cos(heading), math.sin(heading), 0.0])
        ref = CircleReference(centre, radius, speed, phase=heading)
    obs = spheres_in_box(rng, M, start + np.array([0.0, -10.0, -2.5]),
                         start + np.array([20.0, 10.0, 2.5]))
    return Scenario(f"vehicle{vehicle_id}", vehicle_benchmark(), cost_benchmark(), K, N, 0.01,
                    1.0, (1.0, 1.0, 1.0, 1.0), seed=seed, vehicle_id=vehicle_id, ref=ref,
                    obstacles=obs, updates=1)


def c4_batch(n_vehicles=256, seed=4) -> list:
    """256 independent vehicles with uneven K, N and obstacle counts."""
    rng = np.random.default_rng(seed)
    return [random_vehicle(rng, i, seed) for i in range(n_vehicles)]


def c5_arrivals(rate_hz=2000.0, duration_s=60.0, n_vehicles=512, seed=5):
    """Poisson request arrivals: (time_s, vehicle_id, K, N) tuples, plus the
    per-vehicle scenarios.  Each request draws its own K and N."""
    rng = np.random.default_rng(seed)
    fleet = [random_vehicle(rng, i, seed, K=16384, N=200) for i in range(n_vehicles)]
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        out.append((t, int(rng.integers(0, n_vehicles)), int(rng.choice(K_SET)),
                    int(rng.integers(50, 201))))
    return fleet, out


CONFIGS = {"c1": c1_plain, "c2": c2_line, "c3": c3_agile, "paper": paper_preset}
