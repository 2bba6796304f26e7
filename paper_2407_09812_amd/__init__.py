"""Python binding of libmppi, the MI355X (gfx950) MPPI update library.

Argument marshalling only: every step of the update runs in the HIP kernels behind
the C ABI declared in ``include/mppi.h``.  PyTorch supplies device memory and
streams.  Importing this package loads ``libmppi.so`` from the package directory and
raises if it is missing -- there is no CPU fallback.

Function names follow the C ABI (``mppi_update``, ``mppi_rollout``, ...).
Parameter dictionaries use the keys of ``include/mppi.h``'s structs:
  vehicle: mass, J, arm_l, c_tf, g, T_min, T_max, tau_m, k_rate, w_xy_max, w_z_max
  cost:    c_p, c_v, c_q, c_w, R, R_d, obs_margin, obs_w, obs_collision
  solve:   K, N, dt, lam, sigma, u_init, seed, vehicle_id, t
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmppi.so")

MPPI_OK = 0
STATUS = {0: "MPPI_OK", -1: "MPPI_E_INVALID_ARG", -2: "MPPI_E_NONFINITE_INPUT",
          -3: "MPPI_E_ALL_NONFINITE", -4: "MPPI_E_BUDGET", -5: "MPPI_E_OOM", -6: "MPPI_E_HIP",
          -7: "MPPI_E_PENDING", -8: "MPPI_E_CAPACITY"}
NX, NU, NREF = 17, 4, 13
N_MAX, M_MAX = 4096, 2048
SPHERE, VCYLINDER = 0, 1


class MPPIError(RuntimeError):
    def __init__(self, status, where, detail=""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} {detail}".strip())


# --- C structs (layouts of include/mppi.h) ----------------------------------

class Vehicle(C.Structure):
    _fields_ = [("mass", C.c_float), ("J", C.c_float * 3), ("arm_l", C.c_float),
                ("c_tf", C.c_float), ("g", C.c_float), ("T_min", C.c_float), ("T_max", C.c_float),
                ("tau_m", C.c_float), ("k_rate", C.c_float), ("w_xy_max", C.c_float),
                ("w_z_max", C.c_float)]


class Cost(C.Structure):
    _fields_ = [("c_p", C.c_float), ("c_v", C.c_float), ("c_q", C.c_float), ("c_w", C.c_float),
                ("R", C.c_float * 4), ("R_d", C.c_float * 4), ("obs_margin", C.c_float),
                ("obs_w", C.c_float), ("obs_collision", C.c_float)]


class Solve(C.Structure):
    _fields_ = [("K", C.c_int32), ("N", C.c_int32), ("dt", C.c_float), ("lam", C.c_float),
                ("sigma", C.c_float * 4), ("u_init", C.c_float * 4), ("seed", C.c_uint64),
                ("vehicle_id", C.c_uint32), ("t", C.c_uint32), ("dt_ctrl", C.c_float),
                ("reserved", C.c_uint32)]


class Diag(C.Structure):
    _fields_ = [("rho", C.c_float), ("eta", C.c_float), ("ess", C.c_float),
                ("argmin", C.c_int32), ("n_finite", C.c_int32), ("status", C.c_int32),
                ("lanes", C.c_int32), ("reserved", C.c_float)]


class LaunchConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("lanes", C.c_int32), ("unroll", C.c_int32),
                ("fused", C.c_int32), ("pipe", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("veh", Vehicle), ("cost", Cost), ("solve", Solve), ("x_hat", C.c_void_p),
                ("x_ref", C.c_void_p), ("obs", C.c_void_p), ("M", C.c_int32),
                ("u_nom", C.c_void_p), ("u_apply", C.c_void_p), ("diag", C.c_void_p)]


class BatchConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("lanes", C.c_int32), ("unroll", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32)]


class ServerCfg(C.Structure):
    _fields_ = [("device", C.c_int32), ("n_vehicles", C.c_int32), ("K_max", C.c_int32),
                ("N_max", C.c_int32), ("M_max", C.c_int32), ("n_streams", C.c_int32),
                ("max_batch", C.c_int32), ("reserved", C.c_int32), ("budget_bytes", C.c_int64),
                ("veh", Vehicle), ("cost", Cost), ("u_init", C.c_float * 4)]


class ServerRequest(C.Structure):
    _fields_ = [("vehicle_id", C.c_uint32), ("K", C.c_int32), ("N", C.c_int32), ("M", C.c_int32),
                ("dt", C.c_float), ("lam", C.c_float), ("sigma", C.c_float * 4),
                ("dt_ctrl", C.c_float), ("delay", C.c_float),
                ("seed", C.c_uint64), ("x_hat", C.c_void_p), ("x_ref", C.c_void_p),
                ("obs", C.c_void_p)]


class ServerResult(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("vehicle_id", C.c_uint32), ("t", C.c_uint32),
                ("u_apply", C.c_float * 8), ("diag", Diag), ("submit_s", C.c_double),
                ("launch_s", C.c_double), ("done_s", C.c_double), ("K", C.c_int32),
                ("N", C.c_int32), ("delay", C.c_float), ("pipe", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("rejected", C.c_int64), ("rollout_steps", C.c_int64),
                ("max_in_flight", C.c_int64), ("busy_s", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("updates", C.c_int64), ("rollout_ms", C.c_double), ("sum_ms", C.c_double),
                ("batches", C.c_int64),
                ("batch_rollout_ms", C.c_double), ("batch_rest_ms", C.c_double),
                ("obstacle_tests", C.c_int64)]


OBSTACLE_DTYPE = np.dtype([("type", "<i4"), ("c", "<f4", (3,)), ("r", "<f4")])
assert OBSTACLE_DTYPE.itemsize == 20 and C.sizeof(Diag) == 32

# --- library ------------------------------------------------------------------

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (hipcc, gfx950); there is no fallback path")
_lib = C.CDLL(LIB_PATH)

_vp, _i32, _f32 = C.c_void_p, C.c_int32, C.c_float
_PV, _PC, _PS = C.POINTER(Vehicle), C.POINTER(Cost), C.POINTER(Solve)
_SIGS = {
    "mppi_create": [C.c_int, C.POINTER(_vp)],
    "mppi_destroy": [_vp],
    "mppi_reserve": [_vp, _i32, _i32, _i32],
    "mppi_validate": [_PV, _PC, _PS, _i32],
    "mppi_update": [_vp, _vp, _PV, _PC, _PS, _vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "mppi_update_static": [_vp, _vp, _PV, _PC, _PS, _vp, _vp, _vp, _i32, _vp, _vp, _vp],
    "mppi_rollout": [_vp, _vp, _PV, _PC, _PS, _vp, _vp, _vp, _i32, _vp, _vp, _i32, _vp, _vp],
    "mppi_weights": [_vp, _vp, _i32, _vp, _f32, _vp, _vp],
    "mppi_weighted_sum": [_vp, _vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _vp],
    "mppi_apply_shift": [_vp, _vp, _PV, _PS, _vp, _vp, _vp, _vp],
    "mppi_noise": [_vp, _vp, _PS, _vp, _i32],
    "mppi_philox": [_vp, _vp, _i32, _vp, _vp, _vp],
    "mppi_plant_step": [_vp, _vp, _PV, _f32, _vp, _vp, _vp],
    "mppi_predict": [_vp, _vp, _PV, _f32, _f32, _vp, _vp, _vp],
    "mppi_get_config": [_vp, _i32, _i32, _i32, C.POINTER(LaunchConfig)],
    "mppi_set_config": [_vp, _i32, _i32, _i32, C.POINTER(LaunchConfig)],
    "mppi_autotune": [_vp, _vp, _PV, _PC, _PS, _vp, _vp, _vp, _i32, _vp, _i32,
                      C.POINTER(LaunchConfig)],
    "mppi_batch_reserve": [_vp, C.POINTER(Request), _i32],
    "mppi_batch_update": [_vp, _vp, C.POINTER(Request), _i32],
    "mppi_batch_autotune": [_vp, _vp, C.POINTER(Request), _i32, _i32, C.POINTER(BatchConfig)],
    "mppi_batch_get_config": [_vp, C.POINTER(BatchConfig)],
    "mppi_batch_set_config": [_vp, C.POINTER(BatchConfig)],
    "mppi_server_create": [C.POINTER(ServerCfg), C.POINTER(_vp)],
    "mppi_server_destroy": [_vp],
    "mppi_server_set_batch_config": [_vp, C.POINTER(BatchConfig)],
    "mppi_server_submit": [_vp, C.POINTER(ServerRequest), C.POINTER(C.c_uint64)],
    "mppi_server_poll": [_vp, C.c_uint64, C.POINTER(ServerResult)],
    "mppi_server_wait": [_vp, C.c_uint64, C.POINTER(ServerResult)],
    "mppi_server_drain": [_vp],
    "mppi_server_stats_get": [_vp, C.POINTER(ServerStats)],
    "mppi_server_snapshot": [_vp, _vp, C.POINTER(C.c_size_t)],
    "mppi_server_restore": [_vp, _vp, C.c_size_t],
    "mppi_profile_enable": [_vp, _i32],
    "mppi_profile_read": [_vp, C.POINTER(Profile)],
    "mppi_device_address": [_vp, C.POINTER(_vp)],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int32
_lib.mppi_status_str.argtypes = [C.c_int32]
_lib.mppi_status_str.restype = C.c_char_p
_lib.mppi_last_error.argtypes = [_vp]
_lib.mppi_last_error.restype = C.c_char_p
_lib.mppi_server_clock.argtypes = [_vp]
_lib.mppi_server_clock.restype = C.c_double


def exported_symbols():
    """Names of the C ABI entry points this binding resolves."""
    return sorted(list(_SIGS) + ["mppi_status_str", "mppi_last_error", "mppi_server_clock"])


# --- marshalling ----------------------------------------------------------------

def vehicle(d) -> Vehicle:
    """mppi_vehicle from a dict (a Vehicle is passed through, so that a caller in a
    control loop can build it once)."""
    if isinstance(d, Vehicle):
        return d
    v = Vehicle()
    v.mass = d["mass"]; v.J = (C.c_float * 3)(*d["J"]); v.arm_l = d["arm_l"]; v.c_tf = d["c_tf"]
    v.g = d["g"]; v.T_min = d["T_min"]; v.T_max = d["T_max"]; v.tau_m = d["tau_m"]
    v.k_rate = d.get("k_rate", 0.0); v.w_xy_max = d.get("w_xy_max", 0.0)
    v.w_z_max = d.get("w_z_max", 0.0)
    return v


def cost(d) -> Cost:
    """mppi_cost from a dict (a Cost is passed through)."""
    if isinstance(d, Cost):
        return d
    c = Cost()
    c.c_p, c.c_v, c.c_q, c.c_w = d["c_p"], d["c_v"], d["c_q"], d["c_w"]
    c.R = (C.c_float * 4)(*d["R"]); c.R_d = (C.c_float * 4)(*d["R_d"])
    c.obs_margin, c.obs_w, c.obs_collision = d["obs_margin"], d["obs_w"], d["obs_collision"]
    return c


def solve(d) -> Solve:
    """mppi_solve from a dict (a Solve is passed through)."""
    if isinstance(d, Solve):
        return d
    s = Solve()
    s.K, s.N, s.dt, s.lam = int(d["K"]), int(d["N"]), float(d["dt"]), float(d["lam"])
    s.sigma = (C.c_float * 4)(*[float(v) for v in d["sigma"]])
    s.u_init = (C.c_float * 4)(*[float(v) for v in d["u_init"]])
    s.seed = int(d["seed"]) & 0xFFFFFFFFFFFFFFFF
    s.vehicle_id = int(d.get("vehicle_id", 0)) & 0xFFFFFFFF
    s.t = int(d.get("t", 0)) & 0xFFFFFFFF
    s.dt_ctrl = float(d.get("dt_ctrl", 0.0))
    return s


def obstacles_to_device(obs, device="cuda") -> torch.Tensor:
    """[M, 5] rows (type, cx, cy, cz, r) -> device buffer of mppi_obstacle structs."""
    obs = np.asarray(obs, dtype=np.float64).reshape(-1, 5)
    rec = np.zeros(obs.shape[0], dtype=OBSTACLE_DTYPE)
    rec["type"] = obs[:, 0].astype(np.int32)
    rec["c"] = obs[:, 1:4].astype(np.float32)
    rec["r"] = obs[:, 4].astype(np.float32)
    raw = np.frombuffer(rec.tobytes(), dtype=np.uint8).copy()
    if raw.size == 0:
        raw = np.zeros(4, dtype=np.uint8)
    return torch.from_numpy(raw).to(device)


_mapped = {}


def device_address(t: torch.Tensor) -> int:
    """Device address of a pinned host tensor (mppi_device_address), cached per
    allocation."""
    host = t.data_ptr()
    if host not in _mapped:
        d = _vp()
        st = _lib.mppi_device_address(_vp(host), C.byref(d))
        if st != MPPI_OK or not d.value:
            raise MPPIError(st, "mppi_device_address: not pinned host memory")
        _mapped[host] = d.value
    return _mapped[host]


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if t.is_cuda:
        return C.c_void_p(t.data_ptr())
    if t.is_pinned():                     # host memory the device reaches directly
        return C.c_void_p(device_address(t))
    raise ValueError("tensors must be device tensors or pinned host tensors")


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def diag_from_tensor(t: torch.Tensor) -> dict:
    raw = t.detach().cpu().numpy().tobytes()
    d = Diag.from_buffer_copy(raw[:C.sizeof(Diag)])
    return dict(rho=d.rho, eta=d.eta, ess=d.ess, argmin=d.argmin, n_finite=d.n_finite,
                status=d.status, lanes=d.lanes)


def new_diag(device="cuda") -> torch.Tensor:
    return torch.zeros(C.sizeof(Diag), dtype=torch.uint8, device=device)


# --- entry points ---------------------------------------------------------------

class Context:
    """An mppi_ctx on one device (owns the update's scratch)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = _lib.mppi_create(int(device), C.byref(h))
        if st != MPPI_OK:
            raise MPPIError(st, "mppi_create")
        self.handle = h
        self.device = device

    def check(self, st, where):
        if st != MPPI_OK:
            raise MPPIError(st, where, _lib.mppi_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            _lib.mppi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mppi_create(device: int = 0) -> Context:
    return Context(device)


def mppi_destroy(ctx: Context):
    ctx.close()


def mppi_reserve(ctx: Context, K: int, N: int, M: int):
    ctx.check(_lib.mppi_reserve(ctx.handle, int(K), int(N), int(M)), "mppi_reserve")


def mppi_validate(veh: dict, cst: dict, slv: dict, M: int) -> int:
    """Host-only argument check; returns the status code."""
    v, c, s = vehicle(veh), cost(cst), solve(slv)
    return int(_lib.mppi_validate(C.byref(v), C.byref(c), C.byref(s), int(M)))


def mppi_update(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, u_apply, diag=None,
                stream=None):
    v, c, s = vehicle(veh), cost(cst), solve(slv)
    ctx.check(_lib.mppi_update(ctx.handle, _stream(stream), C.byref(v), C.byref(c), C.byref(s),
                               _ptr(x_hat), _ptr(x_ref), _ptr(obs_dev) if M > 0 else None, int(M),
                               _ptr(u_nom), _ptr(u_apply), _ptr(diag)), "mppi_update")


def mppi_update_static(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, u_apply, diag=None,
                       stream=None):
    """mppi_update with its scratch in the library's static device array (no allocation,
    no mppi_reserve needed; stored form)."""
    v, c, s = vehicle(veh), cost(cst), solve(slv)
    ctx.check(_lib.mppi_update_static(ctx.handle, _stream(stream), C.byref(v), C.byref(c),
                                      C.byref(s), _ptr(x_hat), _ptr(x_ref),
                                      _ptr(obs_dev) if M > 0 else None, int(M), _ptr(u_nom),
                                      _ptr(u_apply), _ptr(diag)), "mppi_update_static")


class PreparedUpdate:
    """mppi_update with its arguments marshalled once: calling it (no arguments) runs
    the update on the same buffers, for a control loop that holds its per-step inputs in
    fixed device buffers, as a C caller holds its pointers.  The buffers' contents may
    change between calls; the tensors must stay alive."""

    def __init__(self, ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, u_apply, diag=None,
                 stream=None):
        self._ctx = ctx
        self._keep = (vehicle(veh), cost(cst), solve(slv), x_hat, x_ref, obs_dev, u_nom, u_apply, diag)
        v, c, s = self._keep[:3]
        self._args = (ctx.handle, _stream(stream), C.byref(v), C.byref(c), C.byref(s), _ptr(x_hat),
                      _ptr(x_ref), _ptr(obs_dev) if M > 0 else None, int(M), _ptr(u_nom),
                      _ptr(u_apply), _ptr(diag))

    def __call__(self):
        st = _lib.mppi_update(*self._args)
        if st != MPPI_OK:
            self._ctx.check(st, "mppi_update")


def prepare_update(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, u_apply, diag=None,
                   stream=None) -> PreparedUpdate:
    return PreparedUpdate(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, u_apply, diag, stream)


def mppi_rollout(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, du, ld, S, states=None,
                 stream=None):
    v, c, s = vehicle(veh), cost(cst), solve(slv)
    ctx.check(_lib.mppi_rollout(ctx.handle, _stream(stream), C.byref(v), C.byref(c), C.byref(s),
                                _ptr(x_hat), _ptr(x_ref), _ptr(obs_dev) if M > 0 else None,
                                int(M), _ptr(u_nom), _ptr(du), int(ld), _ptr(S), _ptr(states)),
              "mppi_rollout")


def mppi_weights(ctx, K, S, lam, w, diag, stream=None):
    ctx.check(_lib.mppi_weights(ctx.handle, _stream(stream), int(K), _ptr(S), float(lam), _ptr(w),
                                _ptr(diag)), "mppi_weights")


def mppi_weighted_sum(ctx, K, N, w, du, ld, u_in, u_out, diag=None, stream=None):
    ctx.check(_lib.mppi_weighted_sum(ctx.handle, _stream(stream), int(K), int(N), _ptr(w), _ptr(du),
                                     int(ld), _ptr(u_in), _ptr(u_out), _ptr(diag)),
              "mppi_weighted_sum")


def mppi_apply_shift(ctx, veh, slv, x_hat, u_upd, u_nom, u_apply, stream=None):
    v, s = vehicle(veh), solve(slv)
    ctx.check(_lib.mppi_apply_shift(ctx.handle, _stream(stream), C.byref(v), C.byref(s),
                                    _ptr(x_hat), _ptr(u_upd), _ptr(u_nom), _ptr(u_apply)),
              "mppi_apply_shift")


def mppi_noise(ctx, slv, du, ld, stream=None):
    s = solve(slv)
    ctx.check(_lib.mppi_noise(ctx.handle, _stream(stream), C.byref(s), _ptr(du), int(ld)),
              "mppi_noise")


def mppi_philox(ctx, ctr, key, out, stream=None):
    n = ctr.shape[0]
    ctx.check(_lib.mppi_philox(ctx.handle, _stream(stream), int(n), _ptr(ctr), _ptr(key), _ptr(out)),
              "mppi_philox")


def mppi_plant_step(ctx, veh, dt, x, u, x_out, stream=None):
    v = vehicle(veh)
    ctx.check(_lib.mppi_plant_step(ctx.handle, _stream(stream), C.byref(v), float(dt), _ptr(x),
                                   _ptr(u), _ptr(x_out)), "mppi_plant_step")


def mppi_predict(ctx, veh, dt, delay, x_hat, u_hold, x_out, stream=None):
    v = vehicle(veh)
    ctx.check(_lib.mppi_predict(ctx.handle, _stream(stream), C.byref(v), float(dt), float(delay),
                                _ptr(x_hat), _ptr(u_hold), _ptr(x_out)), "mppi_predict")


def mppi_get_config(ctx, K, N, M) -> dict:
    c = LaunchConfig()
    ctx.check(_lib.mppi_get_config(ctx.handle, int(K), int(N), int(M), C.byref(c)), "mppi_get_config")
    return dict(block=c.block, lanes=c.lanes, unroll=c.unroll, fused=c.fused, pipe=c.pipe)


def mppi_set_config(ctx, K, N, M, block, lanes, unroll, fused=0, pipe=0):
    c = LaunchConfig(int(block), int(lanes), int(unroll), int(fused), int(pipe))
    ctx.check(_lib.mppi_set_config(ctx.handle, int(K), int(N), int(M), C.byref(c)), "mppi_set_config")


def mppi_autotune(ctx, veh, cst, slv, x_hat, x_ref, obs_dev, M, u_nom, reps=3, stream=None) -> dict:
    v, c, s = vehicle(veh), cost(cst), solve(slv)
    best = LaunchConfig()
    ctx.check(_lib.mppi_autotune(ctx.handle, _stream(stream), C.byref(v), C.byref(c), C.byref(s),
                                 _ptr(x_hat), _ptr(x_ref), _ptr(obs_dev) if M > 0 else None,
                                 int(M), _ptr(u_nom), int(reps), C.byref(best)), "mppi_autotune")
    return dict(block=best.block, lanes=best.lanes, unroll=best.unroll, fused=best.fused,
                pipe=best.pipe)


def make_requests(items) -> C.Array:
    """items: dicts with veh, cost, solve (parameter dicts) and device tensors x_hat,
    x_ref, obs (may be None when M = 0), M, u_nom, u_apply and optionally diag."""
    arr = (Request * len(items))()
    for r, it in zip(arr, items):
        r.veh, r.cost, r.solve = vehicle(it["veh"]), cost(it["cost"]), solve(it["solve"])
        r.x_hat, r.x_ref = it["x_hat"].data_ptr(), it["x_ref"].data_ptr()
        r.M = int(it["M"])
        r.obs = it["obs"].data_ptr() if r.M > 0 else None
        r.u_nom, r.u_apply = it["u_nom"].data_ptr(), it["u_apply"].data_ptr()
        d = it.get("diag")
        r.diag = d.data_ptr() if d is not None else None
    return arr


def mppi_batch_reserve(ctx, reqs):
    ctx.check(_lib.mppi_batch_reserve(ctx.handle, reqs, len(reqs)), "mppi_batch_reserve")


def mppi_batch_update(ctx, reqs, stream=None):
    ctx.check(_lib.mppi_batch_update(ctx.handle, _stream(stream), reqs, len(reqs)),
              "mppi_batch_update")


def _batch_cfg_dict(c):
    return dict(block=c.block, lanes=c.lanes, unroll=c.unroll, blocks_per_cu=c.blocks_per_cu,
                use_graph=c.use_graph)


def mppi_batch_autotune(ctx, reqs, reps=2, stream=None) -> dict:
    best = BatchConfig()
    ctx.check(_lib.mppi_batch_autotune(ctx.handle, _stream(stream), reqs, len(reqs), int(reps),
                                       C.byref(best)), "mppi_batch_autotune")
    return _batch_cfg_dict(best)


def mppi_batch_get_config(ctx) -> dict:
    c = BatchConfig()
    ctx.check(_lib.mppi_batch_get_config(ctx.handle, C.byref(c)), "mppi_batch_get_config")
    return _batch_cfg_dict(c)


def mppi_batch_set_config(ctx, block, lanes, unroll, blocks_per_cu, use_graph=True):
    c = BatchConfig(int(block), int(lanes), int(unroll), int(blocks_per_cu), 1 if use_graph else 0)
    ctx.check(_lib.mppi_batch_set_config(ctx.handle, C.byref(c)), "mppi_batch_set_config")


def mppi_profile_enable(ctx, on=True):
    ctx.check(_lib.mppi_profile_enable(ctx.handle, 1 if on else 0), "mppi_profile_enable")


def mppi_profile_read(ctx) -> dict:
    p = Profile()
    ctx.check(_lib.mppi_profile_read(ctx.handle, C.byref(p)), "mppi_profile_read")
    return dict(updates=p.updates, rollout_ms=p.rollout_ms, sum_ms=p.sum_ms, batches=p.batches,
                batch_rollout_ms=p.batch_rollout_ms, batch_rest_ms=p.batch_rest_ms,
                obstacle_tests=p.obstacle_tests)


def mppi_status_str(st: int) -> str:
    return _lib.mppi_status_str(int(st)).decode()


# --- serving --------------------------------------------------------------------

def _result_dict(r: ServerResult) -> dict:
    return dict(ticket=r.ticket, vehicle_id=r.vehicle_id, t=r.t, u_apply=np.array(r.u_apply[:]),
                status=r.diag.status, rho=r.diag.rho, eta=r.diag.eta, ess=r.diag.ess,
                argmin=r.diag.argmin,
                lanes=r.diag.lanes,
                submit_s=r.submit_s, launch_s=r.launch_s, done_s=r.done_s, K=r.K, N=r.N,
                delay=r.delay, pipe=r.pipe, latency_s=r.done_s - r.submit_s)


class Server:
    """mppi_server: continuous batching of MPPI updates for many vehicles."""

    def __init__(self, veh, cst, u_init, n_vehicles, K_max, N_max, M_max, n_streams=2,
                 max_batch=256, budget_bytes=2 << 30, device=0):
        c = ServerCfg()
        c.device, c.n_vehicles, c.K_max, c.N_max, c.M_max = device, n_vehicles, K_max, N_max, M_max
        c.n_streams, c.max_batch, c.budget_bytes = n_streams, max_batch, int(budget_bytes)
        c.veh, c.cost = vehicle(veh), cost(cst)
        c.u_init = (C.c_float * 4)(*[float(v) for v in u_init])
        h = C.c_void_p()
        st = _lib.mppi_server_create(C.byref(c), C.byref(h))
        if st != MPPI_OK:
            raise MPPIError(st, "mppi_server_create")
        self.handle = h

    def _check(self, st, where):
        if st != MPPI_OK:
            raise MPPIError(st, where)

    def set_batch_config(self, block, lanes, unroll, blocks_per_cu, use_graph=True):
        c = BatchConfig(int(block), int(lanes), int(unroll), int(blocks_per_cu), 1 if use_graph else 0)
        self._check(_lib.mppi_server_set_batch_config(self.handle, C.byref(c)),
                    "mppi_server_set_batch_config")

    def submit(self, vehicle_id, K, N, dt, lam, sigma, seed, x_hat, x_ref, obs=None,
               dt_ctrl=0.0, delay=0.0) -> int:
        """x_hat [17], x_ref [(N+1), 13] host arrays; obs an OBSTACLE_DTYPE array;
        dt_ctrl the time between updates (0: dt); delay the seconds to predict x_hat
        forward (< 0: the server's median latency)."""
        r = ServerRequest()
        r.vehicle_id, r.K, r.N = int(vehicle_id), int(K), int(N)
        r.dt, r.lam = float(dt), float(lam)
        r.dt_ctrl, r.delay = float(dt_ctrl), float(delay)
        r.sigma = (C.c_float * 4)(*[float(v) for v in sigma])
        r.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        xh = np.ascontiguousarray(x_hat, dtype=np.float32)
        xr = np.ascontiguousarray(x_ref, dtype=np.float32)
        if xh.size != 17 or xr.size != 13 * (int(N) + 1):
            raise ValueError("x_hat must hold 17 values and x_ref (N+1) x 13")
        r.x_hat, r.x_ref = xh.ctypes.data, xr.ctypes.data
        if obs is not None and len(obs) > 0:
            ob = np.ascontiguousarray(obs, dtype=OBSTACLE_DTYPE)
            r.M, r.obs = ob.shape[0], ob.ctypes.data
        else:
            r.M, r.obs = 0, None
        t = C.c_uint64()
        self._check(_lib.mppi_server_submit(self.handle, C.byref(r), C.byref(t)), "mppi_server_submit")
        return t.value

    def poll(self, ticket):
        r = ServerResult()
        st = _lib.mppi_server_poll(self.handle, int(ticket), C.byref(r))
        if st == -7:
            return None
        self._check(st, "mppi_server_poll")
        return _result_dict(r)

    def wait(self, ticket) -> dict:
        r = ServerResult()
        self._check(_lib.mppi_server_wait(self.handle, int(ticket), C.byref(r)), "mppi_server_wait")
        return _result_dict(r)

    def drain(self):
        self._check(_lib.mppi_server_drain(self.handle), "mppi_server_drain")

    def stats(self) -> dict:
        s = ServerStats()
        self._check(_lib.mppi_server_stats_get(self.handle, C.byref(s)), "mppi_server_stats_get")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def clock(self) -> float:
        return _lib.mppi_server_clock(self.handle)

    def snapshot(self) -> bytes:
        n = C.c_size_t(0)
        self._check(_lib.mppi_server_snapshot(self.handle, None, C.byref(n)), "mppi_server_snapshot")
        buf = C.create_string_buffer(n.value)
        self._check(_lib.mppi_server_snapshot(self.handle, buf, C.byref(n)), "mppi_server_snapshot")
        return buf.raw

    def restore(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        self._check(_lib.mppi_server_restore(self.handle, buf, len(data)), "mppi_server_restore")

    def close(self):
        if self.handle:
            _lib.mppi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def obstacles_host(obs) -> np.ndarray:
    """[M, 5] rows (type, cx, cy, cz, r) -> host array of mppi_obstacle structs."""
    obs = np.asarray(obs, dtype=np.float64).reshape(-1, 5)
    rec = np.zeros(obs.shape[0], dtype=OBSTACLE_DTYPE)
    rec["type"] = obs[:, 0].astype(np.int32)
    rec["c"] = obs[:, 1:4].astype(np.float32)
    rec["r"] = obs[:, 4].astype(np.float32)
    return rec
