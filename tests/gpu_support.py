"""Helpers shared by the GPU parity tests: device copies of a scenario, the
binary32-rounded inputs the oracle is given, and the relative-error measure.

Relative error: |gpu - oracle| / max(|oracle|, floor) with floors 1 m (position),
1 (quaternion), 1 m/s (velocity), 1 rad/s (body rate), 1 N (thrust), sigma (noise
and controls) -- the scale of each quantity, so that values near zero are not held
to a relative bound they cannot meet in binary32.
"""
import numpy as np
import torch

TOL = 1e-4
STATE_FLOOR = np.array([1.0] * 17)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def f32_params(d: dict) -> dict:
    """Round every number of a parameter dict to binary32, as the device sees it."""
    out = {}
    for k, v in d.items():
        if isinstance(v, (list, tuple, np.ndarray)):
            out[k] = tuple(float(np.float32(x)) for x in np.asarray(v).ravel())
        elif isinstance(v, float):
            out[k] = float(np.float32(v))
        else:
            out[k] = v
    return out


def rel_err(gpu, ref, floor):
    gpu, ref = np.asarray(gpu, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), floor)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


class DeviceProblem:
    """Device-resident inputs of one update of a scenario, and the same inputs
    rounded to binary32 for the oracle."""

    def __init__(self, lib, sc, t=0, x_hat=None, u_nom=None, solve=None):
        self.sc = sc
        self.solve = dict(sc.solve(t) if solve is None else solve)
        self.N, self.K, self.M = self.solve["N"], self.solve["K"], sc.M
        x_hat = sc.x0 if x_hat is None else x_hat
        u_nom = sc.u_nom0()[: self.N] if u_nom is None else u_nom
        x_ref = sc.ref.rows(t * sc.period, self.N, sc.dt)
        self.x_hat, self.u_nom, self.x_ref = dev(x_hat), dev(u_nom), dev(x_ref)
        self.obs = lib.obstacles_to_device(sc.obstacles)
        # what the oracle is given: the binary32 values the device holds
        self.o_x_hat, self.o_u_nom, self.o_x_ref = f32(x_hat), f32(u_nom), f32(x_ref)
        self.o_obs = sc.obstacles.copy()
        self.o_obs[:, 1:] = f32(self.o_obs[:, 1:])
        self.o_veh, self.o_cost = f32_params(sc.veh), f32_params(sc.cost)
        self.o_solve = f32_params(self.solve)


def collision_counts(states, obstacles):
    """Per sample, the number of states inside some obstacle (binary64, from the
    given positions): the states the collision constant is charged on."""
    if obstacles.shape[0] == 0:
        return np.zeros(states.shape[0], dtype=np.int64), np.full(states.shape[:2], np.inf)
    p = states[:, :, None, 0:3]                      # [n, N+1, 1, 3]
    d = p - obstacles[None, None, :, 1:4]
    zmask = (obstacles[:, 0] == 0).astype(np.float64)[None, None, :]
    dist = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2 + (d[..., 2] * zmask) ** 2)
    gap = dist - obstacles[None, None, :, 4]
    inside = (gap < 0).any(axis=2)
    return inside.sum(axis=1), np.abs(gap).min(axis=2)


def check_costs(S_gpu, S_orc, st_gpu, st_orc, obstacles, c_col, tol):
    """Costs agree to tol, except where a state sits on an obstacle surface closer
    than the two trajectories differ: there the collision indicator may flip, and
    the costs must then differ by an integer multiple of the collision constant.
    Returns (max relative error over the unambiguous samples, number of flips)."""
    n_g, _ = collision_counts(st_gpu, obstacles)
    n_o, gap_o = collision_counts(st_orc, obstacles)
    dp = np.linalg.norm(st_gpu[:, :, 0:3] - st_orc[:, :, 0:3], axis=2)
    ambiguous = ((gap_o < 2.0 * dp + 1e-6).any(axis=1)) | (n_g != n_o)
    err = np.abs(S_gpu - S_orc) / np.maximum(np.abs(S_orc), 1.0)
    e_clean = err[~ambiguous].max() if (~ambiguous).any() else 0.0
    if ambiguous.any() and c_col > 0:
        r = (S_gpu[ambiguous] - S_orc[ambiguous]) / c_col
        resid = np.abs(r - np.round(r)) * c_col / np.maximum(np.abs(S_orc[ambiguous]), 1.0)
        assert resid.max() <= tol, f"ambiguous samples differ by a non-multiple of c_col: {resid.max()}"
    return e_clean, int(ambiguous.sum())


def check_cost_flips(S_gpu, S_orc, c_col, tol, gap_orc=None, reach=None):
    """Costs without the device's trajectories: a sample whose cost differs by at
    least half the collision constant counts as a collision-indicator flip, and must
    differ by an integer multiple of it (residual within tol of the cost); when the
    oracle's closest approach to an obstacle surface per sample (gap_orc) is given,
    a flip is allowed only where that approach is within `reach` (the distance the
    binary32 trajectory may lie from the binary64 one) of a surface.  Returns (max
    relative error over the other samples, number of flips)."""
    S_gpu, S_orc = np.asarray(S_gpu, np.float64), np.asarray(S_orc, np.float64)
    err = np.abs(S_gpu - S_orc) / np.maximum(np.abs(S_orc), 1.0)
    if c_col > 0:
        r = (S_gpu - S_orc) / c_col
        flip = np.abs(r) >= 0.5
    else:
        r, flip = np.zeros_like(S_gpu), np.zeros(S_gpu.shape, bool)
    if flip.any():
        resid = np.abs(r[flip] - np.round(r[flip])) * c_col / np.maximum(np.abs(S_orc[flip]), 1.0)
        assert resid.max() <= tol, f"flipped samples differ by a non-multiple of c_col: {resid.max()}"
        if gap_orc is not None:
            far = np.asarray(gap_orc)[flip] > np.asarray(reach)[flip]
            assert not far.any(), f"{int(far.sum())} flipped samples are nowhere near a surface"
    e_clean = err[~flip].max() if (~flip).any() else 0.0
    return e_clean, int(flip.sum())


def surface_gap(states, obstacles):
    """Per sample, the smallest |distance - radius| over its states and the obstacles
    (binary64), and a reach 2 TOL max(|p|, 1) the binary32 positions may differ by."""
    _, gap = collision_counts(states, obstacles)
    reach = 2.0 * TOL * np.maximum(np.linalg.norm(states[:, :, 0:3], axis=2), 1.0)
    return gap.min(axis=1), (reach + 1e-6).max(axis=1)
