"""FP64 CPU oracle for one MPPI update (arXiv 2407.09812) -- TEST INFRASTRUCTURE.

This package is the plain, slow, obviously-correct reference that the HIP path is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product package never does.

The arithmetic lives in ``mppi_oracle.c`` (double precision, no fast-math, no FMA
contraction); this module only marshals numpy arrays through ctypes.

Parameter dictionaries (plain numbers, produced by ``workloads``):
  vehicle: mass, J (3), arm_l, c_tf, g, T_min, T_max, tau_m, k_rate, w_xy_max, w_z_max
  cost:    c_p, c_v, c_q, c_w, R (4), R_d (4), obs_margin, obs_w, obs_collision
Arrays: state x (17) = [p, q (w first), v, omega, T]; control u (4) = [F_t, omega_d];
reference x_ref [(N+1), 13] = [p, q, v, omega]; obstacles [M, 5] = [type, cx, cy, cz, r]
with type 0 = sphere, 1 = vertical cylinder.

Every function follows the paper (Algorithm 1, Sec. III-A Eqs. (2)-(5),
Sec. III-B Eqs. (6)-(15), Sec. IV-C Eqs. (16)-(21), Sec. IV-D Eq. (22)); see the
header of ``mppi_oracle.c`` for the readings taken where the paper is silent.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

NX = 17
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB) or (
            os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
        _build.build()
    lib = C.CDLL(_build.LIB)
    dp = C.POINTER(C.c_double)
    up = C.POINTER(C.c_uint32)
    ip = C.POINTER(C.c_int32)
    i32, u32, u64, f64 = C.c_int, C.c_uint32, C.c_uint64, C.c_double
    sig = {
        "orc_philox4x32_10": (None, [up, up, up]),
        "orc_uniform": (f64, [u32]),
        "orc_noise_one": (None, [i32, i32, dp, u64, u32, u32, dp]),
        "orc_noise": (None, [i32, i32, dp, u64, u32, u32, dp]),
        "orc_allocation": (None, [dp, dp]),
        "orc_allocation_inverse": (i32, [dp, dp]),
        "orc_controller": (None, [dp, dp, dp, f64, dp]),
        "orc_dynamics": (None, [dp, dp, dp, dp]),
        "orc_rk4_step": (None, [dp, dp, dp, f64, dp]),
        "orc_model_step": (None, [dp, dp, dp, f64, dp]),
        "orc_applied_input": (None, [dp, dp, dp, f64, dp]),
        "orc_quat_distance": (f64, [dp, dp]),
        "orc_tracking_cost": (f64, [dp, dp, dp]),
        "orc_obstacle_cost": (f64, [dp, dp, dp, i32]),
        "orc_trajectory_cost": (f64, [dp, i32, dp, dp, dp, dp, i32]),
        "orc_rollouts": (None, [dp, dp, i32, i32, f64, dp, u64, u32, u32,
                                dp, dp, dp, dp, i32, dp, dp, dp]),
        "orc_rollouts_subset": (None, [dp, dp, i32, ip, i32, f64, dp, u64, u32, u32,
                                       dp, dp, dp, dp, i32, dp, dp, dp]),
        "orc_philox_many": (None, [i32, up, up, up]),
        "orc_num_threads": (i32, []),
        "orc_set_num_threads": (None, [i32]),
        "orc_weights": (i32, [i32, dp, f64, dp, dp]),
        "orc_weighted_update": (None, [i32, i32, dp, dp, dp]),
        "orc_advance": (None, [i32, f64, dp, dp]),
        "orc_apply_shift": (None, [dp, i32, f64, f64, dp, dp, dp, dp]),
        "orc_predict": (None, [dp, f64, f64, dp, dp, dp]),
        "orc_update": (i32, [dp, dp, i32, i32, f64, f64, dp, u64, u32, u32,
                             dp, f64, dp, dp, dp, dp, i32, dp, dp, dp, dp, dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a, n=None):
    """Contiguous float64 array (kept alive by the caller) and its pointer."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def vehicle_array(veh: dict) -> np.ndarray:
    J = veh["J"]
    return np.array([veh["mass"], J[0], J[1], J[2], veh["arm_l"], veh["c_tf"], veh["g"],
                     veh["T_min"], veh["T_max"], veh["tau_m"], veh.get("k_rate", 0.0),
                     veh.get("w_xy_max", 0.0), veh.get("w_z_max", 0.0)], dtype=np.float64)


def cost_array(cost: dict) -> np.ndarray:
    return np.array([cost["c_p"], cost["c_v"], cost["c_q"], cost["c_w"], *cost["R"],
                     *cost["R_d"], cost["obs_margin"], cost["obs_w"],
                     cost["obs_collision"]], dtype=np.float64)


def obstacle_array(obs) -> np.ndarray:
    if obs is None:
        return np.zeros((0, 5))
    a = np.ascontiguousarray(obs, dtype=np.float64).reshape(-1, 5)
    return a


# --- noise ---------------------------------------------------------------

def philox4x32_10(ctr, key):
    lib = _load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def num_threads() -> int:
    """Threads the oracle's per-sample loop uses."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int):
    """Threads of the per-sample loop from now on (OpenMP)."""
    _load().orc_set_num_threads(int(n))


def philox_many(ctr, key):
    """Philox4x32-10 of n counters [n, 4] with keys [n, 2] (uint32) -> [n, 4]."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    up = C.POINTER(C.c_uint32)
    _load().orc_philox_many(ctr.shape[0], ctr.ctypes.data_as(up), key.ctypes.data_as(up),
                            out.ctypes.data_as(up))
    return out


def uniform(w: int) -> float:
    return _load().orc_uniform(int(w) & 0xFFFFFFFF)


def noise(K, N, sigma, seed, vehicle_id=0, t=0):
    """delta_u for all samples and steps, [K, N, 4]."""
    lib = _load()
    s = _d(sigma, 4)
    out = np.empty((K, N, 4))
    lib.orc_noise(K, N, _p(s), int(seed), int(vehicle_id), int(t), _p(out))
    return out


# --- model ---------------------------------------------------------------

def allocation(veh):
    v = vehicle_array(veh)
    G = np.empty(16)
    _load().orc_allocation(_p(v), _p(G))
    return G.reshape(4, 4)


def allocation_inverse(veh):
    v = vehicle_array(veh)
    G = np.empty(16)
    if _load().orc_allocation_inverse(_p(v), _p(G)) != 0:
        raise ValueError("allocation matrix is singular")
    return G.reshape(4, 4)


def controller(veh, x, u, dt):
    v, x, u = vehicle_array(veh), _d(x, NX), _d(u, 4)
    out = np.empty(4)
    _load().orc_controller(_p(v), _p(x), _p(u), dt, _p(out))
    return out


def dynamics(veh, x, T_cmd):
    v, x, T = vehicle_array(veh), _d(x, NX), _d(T_cmd, 4)
    out = np.empty(NX)
    _load().orc_dynamics(_p(v), _p(x), _p(T), _p(out))
    return out


def rk4_step(veh, x, T_cmd, dt):
    v, x, T = vehicle_array(veh), _d(x, NX), _d(T_cmd, 4)
    out = np.empty(NX)
    _load().orc_rk4_step(_p(v), _p(x), _p(T), dt, _p(out))
    return out


def model_step(veh, x, u, dt):
    v, x, u = vehicle_array(veh), _d(x, NX), _d(u, 4)
    out = np.empty(NX)
    _load().orc_model_step(_p(v), _p(x), _p(u), dt, _p(out))
    return out


def applied_input(veh, x, u, dt):
    v, x, u = vehicle_array(veh), _d(x, NX), _d(u, 4)
    out = np.empty(4)
    _load().orc_applied_input(_p(v), _p(x), _p(u), dt, _p(out))
    return out


# --- cost ----------------------------------------------------------------

def quat_distance(q1, q2):
    a, b = _d(q1, 4), _d(q2, 4)
    return _load().orc_quat_distance(_p(a), _p(b))


def tracking_cost(cost, x, xr):
    c, x, xr = cost_array(cost), _d(x, NX), _d(xr, 13)
    return _load().orc_tracking_cost(_p(c), _p(x), _p(xr))


def obstacle_cost(cost, p, obs):
    c, p = cost_array(cost), _d(p, 3)
    o = obstacle_array(obs)
    return _load().orc_obstacle_cost(_p(c), _p(p), _p(o), o.shape[0])


def trajectory_cost(cost, states, u, x_ref, obs=None):
    u = _d(u).reshape(-1, 4)
    N = u.shape[0]
    c = cost_array(cost)
    s = _d(states, (N + 1) * NX)
    xr = _d(x_ref, (N + 1) * 13)
    o = obstacle_array(obs)
    return _load().orc_trajectory_cost(_p(c), N, _p(s), _p(u), _p(xr), _p(o), o.shape[0])


# --- the MPPI iteration ---------------------------------------------------

def rollouts(veh, cost, solve, x_hat, u_nom, x_ref, obs=None, want_states=False):
    """Returns (states [K, N+1, 17] or None, du [K, N, 4], S [K])."""
    K, N = int(solve["K"]), int(solve["N"])
    v, c = vehicle_array(veh), cost_array(cost)
    s = _d(solve["sigma"], 4)
    xh, un, xr = _d(x_hat, NX), _d(u_nom, N * 4), _d(x_ref, (N + 1) * 13)
    o = obstacle_array(obs)
    states = np.empty((K, N + 1, NX)) if want_states else None
    du = np.empty((K, N, 4))
    S = np.empty(K)
    _load().orc_rollouts(_p(v), _p(c), K, N, float(solve["dt"]), _p(s), int(solve["seed"]),
                         int(solve.get("vehicle_id", 0)), int(solve.get("t", 0)),
                         _p(xh), _p(un), _p(xr), _p(o), o.shape[0], _p(states), _p(du), _p(S))
    return states, du, S


def rollouts_subset(veh, cost, solve, ks, x_hat, u_nom, x_ref, obs=None, want_states=True):
    """Rollouts of the sample indices ks only: (states [n, N+1, 17] or None,
    du [n, N, 4], S [n])."""
    N = int(solve["N"])
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    v, c = vehicle_array(veh), cost_array(cost)
    s = _d(solve["sigma"], 4)
    xh, un, xr = _d(x_hat, NX), _d(u_nom, N * 4), _d(x_ref, (N + 1) * 13)
    o = obstacle_array(obs)
    n = ks.size
    states = np.empty((n, N + 1, NX)) if want_states else None
    du = np.empty((n, N, 4))
    S = np.empty(n)
    _load().orc_rollouts_subset(_p(v), _p(c), n, ks.ctypes.data_as(C.POINTER(C.c_int32)), N,
                                float(solve["dt"]), _p(s), int(solve["seed"]),
                                int(solve.get("vehicle_id", 0)), int(solve.get("t", 0)),
                                _p(xh), _p(un), _p(xr), _p(o), o.shape[0], _p(states), _p(du),
                                _p(S))
    return states, du, S


def weights(S, lam):
    """Softmin weights (Eq. (4)); returns (w [K], diag = [rho, eta, ess, argmin])."""
    S = _d(S)
    w = np.empty(S.size)
    diag = np.empty(4)
    if _load().orc_weights(S.size, _p(S), float(lam), _p(w), _p(diag)) != 0:
        raise FloatingPointError("every rollout cost is non-finite")
    return w, diag


def weighted_update(w, du, u_nom):
    """u_nom + sum_k w_k du^k (Eq. (5)); du is [K, N, 4]."""
    w = _d(w)
    du = _d(du)
    K, N = du.shape[0], du.shape[1]
    out = _d(u_nom, N * 4).copy()
    _load().orc_weighted_update(K, N, _p(w), _p(du), _p(out))
    return out.reshape(N, 4)


def apply_shift(veh, dt, x_hat, u_nom, u_init, alpha=1.0):
    """Returns (u_apply [8], u_nom [N, 4] advanced by alpha of a step; 1 = shift)."""
    un = _d(u_nom).reshape(-1, 4).copy()
    v, xh, ui = vehicle_array(veh), _d(x_hat, NX), _d(u_init, 4)
    ua = np.empty(8)
    _load().orc_apply_shift(_p(v), un.shape[0], float(dt), float(alpha), _p(xh), _p(ui),
                            _p(un), _p(ua))
    return ua, un


def advance(u_nom, u_init, alpha):
    """The warm start advanced by alpha in (0, 1] of a step (Sec. IV-B)."""
    un = _d(u_nom).reshape(-1, 4).copy()
    ui = _d(u_init, 4)
    _load().orc_advance(un.shape[0], float(alpha), _p(ui), _p(un))
    return un


def predict(veh, dt, delay, x, u_hold):
    """State after `delay` s with u_hold held (Sec. IV-E), steps of at most dt."""
    v, x, u = vehicle_array(veh), _d(x, NX), _d(u_hold, 4)
    out = np.empty(NX)
    _load().orc_predict(_p(v), float(dt), float(delay), _p(x), _p(u), _p(out))
    return out


def update(veh, cost, solve, x_hat, u_nom, x_ref, obs=None):
    """One loop body of Algorithm 1.  Returns a dict with the new (shifted) u_nom,
    u_apply [8], diag [rho, eta, ess, argmin], du [K, N, 4], S [K] and w [K]."""
    K, N = int(solve["K"]), int(solve["N"])
    v, c = vehicle_array(veh), cost_array(cost)
    s, ui = _d(solve["sigma"], 4), _d(solve["u_init"], 4)
    xh, xr = _d(x_hat, NX), _d(x_ref, (N + 1) * 13)
    un = _d(u_nom, N * 4).copy()
    o = obstacle_array(obs)
    ua, diag = np.empty(8), np.empty(4)
    du, S, w = np.empty((K, N, 4)), np.empty(K), np.empty(K)
    rc = _load().orc_update(_p(v), _p(c), K, N, float(solve["dt"]), float(solve["lam"]), _p(s),
                            int(solve["seed"]), int(solve.get("vehicle_id", 0)),
                            int(solve.get("t", 0)), _p(ui), float(solve.get("dt_ctrl", 0.0)),
                            _p(xh), _p(un), _p(xr), _p(o),
                            o.shape[0],
                            _p(ua), _p(diag), _p(du), _p(S), _p(w))
    if rc != 0:
        raise FloatingPointError("every rollout cost is non-finite")
    return {"u_nom": un.reshape(N, 4), "u_apply": ua, "diag": diag, "du": du, "S": S, "w": w}
