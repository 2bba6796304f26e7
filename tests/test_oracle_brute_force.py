"""A third implementation of one MPPI update, written out by hand for K = 2 samples
and N = 2 steps in plain Python scalars, against which the FP64 oracle's whole
update is pinned (Algorithm 1's loop body).

Nothing here calls the oracle's model, cost, weights or update: only its noise,
which the Philox known-answer vectors and the Gaussian statistics pin separately.
The allocation is the matrix printed in Eq. (11) and its inverse in closed form
(its rows are orthogonal: Gamma^-1 = Gamma^T diag(1/4, 1/(2 l^2), 1/(2 l^2),
1/(4 c^2))), where the oracle eliminates; RK4's four stages, the quaternion
product and the rotation's third column are expanded term by term; the two-sample
softmin and the weighted sums are written out.

Citations are to arXiv 2407.09812.
"""
import math

import numpy as np
import pytest

import workloads as W

K, N = 2, 2


def rotor_command(veh, x, u, dt):
    """Eqs. (8)-(12): body-rate P law, desired torque, allocation, clip."""
    Jx, Jy, Jz = veh["J"]
    l, c = veh["arm_l"], veh["c_tf"]
    kw = veh["k_rate"] if veh["k_rate"] > 0 else 1.0 / dt
    wx, wy, wz = x[10], x[11], x[12]
    # omega x (J omega), component by component
    gx = wy * (Jz * wz) - wz * (Jy * wy)
    gy = wz * (Jx * wx) - wx * (Jz * wz)
    gz = wx * (Jy * wy) - wy * (Jx * wx)
    tx = Jx * (kw * (u[1] - wx)) + gx
    ty = Jy * (kw * (u[2] - wy)) + gy
    tz = Jz * (kw * (u[3] - wz)) + gz
    s = l / math.sqrt(2.0)
    a, b, e, f = u[0] / 4.0, tx / (2 * l * l), ty / (2 * l * l), tz / (4 * c * c)
    Td = [a - s * b - s * e - c * f,       # column 1 of Eq. (11): (1, -s, -s, -c)
          a + s * b + s * e - c * f,       # column 2: (1,  s,  s, -c)
          a + s * b - s * e + c * f,       # column 3: (1,  s, -s,  c)
          a - s * b + s * e + c * f]       # column 4: (1, -s,  s,  c)
    return [min(max(T, veh["T_min"]), veh["T_max"]) for T in Td]


def wrench(veh, T):
    """Eq. (13): [F; tau] = Gamma T with the printed matrix."""
    s = veh["arm_l"] / math.sqrt(2.0)
    c = veh["c_tf"]
    return (T[0] + T[1] + T[2] + T[3],
            s * (-T[0] + T[1] + T[2] - T[3]),
            s * (-T[0] + T[1] - T[2] + T[3]),
            c * (-T[0] - T[1] + T[2] + T[3]))


def derivative(veh, x, Tc):
    """Eq. (6) with the rotor lag (T' = (T_cmd - T) / tau_m) when tau_m > 0."""
    lag = veh["tau_m"] > 0
    T = x[13:17] if lag else Tc
    F, tx, ty, tz = wrench(veh, T)
    Jx, Jy, Jz = veh["J"]
    m, g = veh["mass"], veh["g"]
    qw, qx, qy, qz = x[3], x[4], x[5], x[6]
    wx, wy, wz = x[10], x[11], x[12]
    d = [0.0] * 17
    d[0], d[1], d[2] = x[7], x[8], x[9]
    d[3] = 0.5 * (-qx * wx - qy * wy - qz * wz)
    d[4] = 0.5 * (qw * wx + qy * wz - qz * wy)
    d[5] = 0.5 * (qw * wy - qx * wz + qz * wx)
    d[6] = 0.5 * (qw * wz + qx * wy - qy * wx)
    d[7] = 2.0 * (qx * qz + qw * qy) * F / m
    d[8] = 2.0 * (qy * qz - qw * qx) * F / m
    d[9] = (1.0 - 2.0 * (qx * qx + qy * qy)) * F / m - g
    d[10] = (tx - (wy * (Jz * wz) - wz * (Jy * wy))) / Jx
    d[11] = (ty - (wz * (Jx * wx) - wx * (Jz * wz))) / Jy
    d[12] = (tz - (wx * (Jy * wy) - wy * (Jx * wx))) / Jz
    for i in range(4):
        d[13 + i] = (Tc[i] - x[13 + i]) / veh["tau_m"] if lag else 0.0
    return d


def step(veh, x, u, dt):
    """Eq. (2), last line: controller held over one classic RK4 step, then q / |q|."""
    Tc = rotor_command(veh, x, u, dt)
    k1 = derivative(veh, x, Tc)
    k2 = derivative(veh, [x[i] + 0.5 * dt * k1[i] for i in range(17)], Tc)
    k3 = derivative(veh, [x[i] + 0.5 * dt * k2[i] for i in range(17)], Tc)
    k4 = derivative(veh, [x[i] + dt * k3[i] for i in range(17)], Tc)
    y = [x[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]) for i in range(17)]
    n = math.sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5] + y[6] * y[6])
    y[3], y[4], y[5], y[6] = y[3] / n, y[4] / n, y[5] / n, y[6] / n
    if veh["tau_m"] <= 0:
        y[13:17] = Tc
    return y


def state_cost(cost, x, r, obs):
    """Eq. (18) with d_q of Eq. (21), plus the obstacle term (Eq. (22) with the
    quadratic margin; strict inside test)."""
    ep = sum((x[i] - r[i]) ** 2 for i in range(3))
    ev = sum((x[7 + i] - r[7 + i]) ** 2 for i in range(3))
    ew = sum((x[10 + i] - r[10 + i]) ** 2 for i in range(3))
    ip = x[3] * r[3] + x[4] * r[4] + x[5] * r[5] + x[6] * r[6]
    dq = 1.0 - ip * ip
    s = cost["c_p"] * ep + cost["c_q"] * dq * dq + cost["c_v"] * ev + cost["c_w"] * ew
    hit, pen = False, 0.0
    for typ, cx, cy, cz, rad in obs:
        dz2 = 0.0 if int(typ) == W.VCYL else (x[2] - cz) ** 2
        dist = math.sqrt((x[0] - cx) ** 2 + (x[1] - cy) ** 2 + dz2)
        hit = hit or dist < rad
        gap = rad + cost["obs_margin"] - dist
        pen += gap * gap if gap > 0 else 0.0
    return s + (cost["obs_collision"] if hit else 0.0) + cost["obs_w"] * pen


def feasible(veh, x, u, dt):
    """Eqs. (12)-(15): [F_clip, w_clip] with the optional rate limits."""
    F, tx, ty, tz = wrench(veh, rotor_command(veh, x, u, dt))
    Jx, Jy, Jz = veh["J"]
    wx, wy, wz = x[10], x[11], x[12]
    out = [F,
           wx + (tx - (wy * (Jz * wz) - wz * (Jy * wy))) / Jx * dt,
           wy + (ty - (wz * (Jx * wx) - wx * (Jz * wz))) / Jy * dt,
           wz + (tz - (wx * (Jy * wy) - wy * (Jx * wx))) / Jz * dt]
    for i, lim in ((1, veh["w_xy_max"]), (2, veh["w_xy_max"]), (3, veh["w_z_max"])):
        if lim > 0:
            out[i] = min(max(out[i], -lim), lim)
    return out


def brute_force_update(veh, cost, dt, lam, alpha, u_init, x_hat, u_nom, x_ref, obs, du):
    """Algorithm 1's loop body for K = 2, N = 2, every sum written out."""
    x_hat = [float(v) for v in x_hat]
    S = []
    for k in range(K):
        u0 = [u_nom[0][d] + du[k][0][d] for d in range(4)]
        u1 = [u_nom[1][d] + du[k][1][d] for d in range(4)]
        x1 = step(veh, x_hat, u0, dt)
        x2 = step(veh, x1, u1, dt)
        R, Rd = cost["R"], cost["R_d"]
        s = sum(R[d] * (u0[d] * u0[d] + u1[d] * u1[d]) for d in range(4))       # Eq. (16)
        s += sum(Rd[d] * (u1[d] - u0[d]) ** 2 for d in range(4))
        s += state_cost(cost, x_hat, x_ref[0], obs)
        s += state_cost(cost, x1, x_ref[1], obs)
        s += state_cost(cost, x2, x_ref[2], obs)
        S.append(s)
    rho = min(S[0], S[1])                                                      # Eq. (4)
    e0, e1 = math.exp(-(S[0] - rho) / lam), math.exp(-(S[1] - rho) / lam)
    eta = e0 + e1
    w0, w1 = e0 / eta, e1 / eta
    upd = [[u_nom[j][d] + (w0 * du[0][j][d] + w1 * du[1][j][d]) for d in range(4)]
           for j in range(N)]                                                  # Eq. (5)
    u_apply = upd[0] + feasible(veh, x_hat, upd[0], dt)
    nxt = [upd[1], list(u_init)]
    new = [[(1 - alpha) * upd[j][d] + alpha * nxt[j][d] for d in range(4)] for j in range(N)]
    return dict(S=S, rho=rho, eta=eta, ess=1.0 / (w0 * w0 + w1 * w1),
                argmin=0 if S[0] <= S[1] else 1, u_apply=u_apply, u_nom=new)


def case(name):
    rng = np.random.default_rng({"lag": 31, "paper": 32}[name])
    if name == "lag":
        veh, cost = W.vehicle_benchmark(), W.cost_benchmark()
        sigma, dt, alpha = np.array([6.0, 3.0, 3.0, 2.0]), 0.01, 1.0
    else:
        veh, cost = W.vehicle_paper(), W.cost_paper()
        cost["obs_w"], cost["obs_margin"] = 500.0, 0.25        # both obstacle terms active
        sigma, dt, alpha = np.sqrt([0.60, 0.15, 0.15, 0.05]) * 8, 0.02, 0.4
    x_hat = np.concatenate([[1.0, -0.5, 2.0], [0.9, 0.1, -0.3, 0.2], [2.0, -1.0, 0.5],
                            [0.7, -0.4, 1.1], rng.uniform(1.0, 4.0, 4)])
    x_hat[3:7] /= np.linalg.norm(x_hat[3:7])
    u_nom = np.array([[12.0, 0.5, -0.2, 0.3], [10.0, -0.4, 0.6, -0.1]])
    x_ref = np.concatenate([rng.normal(size=(N + 1, 3)) + x_hat[:3],
                            np.tile([0.8, 0.0, 0.6, 0.0], (N + 1, 1)),
                            rng.normal(size=(N + 1, 6))], axis=1)
    obs = np.array([[W.SPHERE, 1.45, -0.5, 2.1, 0.3],       # inside the margin, outside r
                    [W.VCYL, 0.95, -0.35, 0.0, 0.25]])       # the state sits inside
    solve = dict(K=K, N=N, dt=dt, lam=1.0, sigma=sigma, seed=(7 << 32) | 99, vehicle_id=5, t=3,
                 u_init=W.hover_control(veh), dt_ctrl=alpha * dt if alpha < 1 else 0.0)
    return veh, cost, solve, alpha, x_hat, u_nom, x_ref, obs


@pytest.mark.parametrize("name", ["lag", "paper"])
def test_update_equals_hand_expanded_brute_force(orc, name):
    veh, cost, solve, alpha, x_hat, u_nom, x_ref, obs = case(name)
    du = orc.noise(K, N, solve["sigma"], solve["seed"], solve["vehicle_id"], solve["t"]).tolist()
    ref = [list(r) for r in x_ref]
    un = [list(r) for r in u_nom]
    first = brute_force_update(veh, cost, solve["dt"], 1.0, alpha, solve["u_init"], x_hat, un,
                               ref, obs.tolist(), du)
    # a temperature of the order of the cost gap keeps both weights well away from 0 and 1
    lam = max(abs(first["S"][0] - first["S"][1]), 1e-3)
    solve["lam"] = lam
    want = brute_force_update(veh, cost, solve["dt"], lam, alpha, solve["u_init"], x_hat, un,
                              ref, obs.tolist(), du)
    got = orc.update(veh, cost, solve, x_hat, u_nom, x_ref, obs)

    np.testing.assert_allclose(got["S"], want["S"], rtol=1e-12)
    assert got["diag"][3] == want["argmin"]
    # The exponent (S_k - rho) / lambda inherits the costs' rounding, a few units of
    # 2^-53 |S| each (summation order differs): relative to lambda that is the
    # conditioning of Eq. (4), and it bounds how far the weights, eta, the ESS and
    # the update can agree.
    tol = 1e-12 + 64 * 2.0 ** -53 * max(abs(s) for s in want["S"]) / lam
    np.testing.assert_allclose(got["diag"][:3], [want["rho"], want["eta"], want["ess"]], rtol=tol)
    assert 0.1 < got["w"].min() < got["w"].max() < 0.9
    np.testing.assert_allclose(got["u_apply"], want["u_apply"], rtol=tol, atol=tol)
    np.testing.assert_allclose(got["u_nom"], want["u_nom"], rtol=tol, atol=tol)


@pytest.mark.parametrize("name", ["lag", "paper"])
def test_brute_force_case_exercises_every_term(orc, name):
    """The hand-expanded case is not degenerate: some rotor saturates, the obstacle
    collision and margin terms both contribute, and with the lag the thrust state
    differs from its command."""
    veh, cost, solve, alpha, x_hat, u_nom, x_ref, obs = case(name)
    du = orc.noise(K, N, solve["sigma"], solve["seed"], solve["vehicle_id"], solve["t"])
    clipped = 0
    for k in range(K):
        T = rotor_command(veh, list(x_hat), list(u_nom[0] + du[k][0]), solve["dt"])
        clipped += sum(t in (veh["T_min"], veh["T_max"]) for t in T)
    assert clipped > 0
    c = state_cost(cost, list(x_hat), list(x_ref[0]), obs.tolist())
    no_obs = state_cost(cost, list(x_hat), list(x_ref[0]), [])
    margin_only = state_cost(cost, list(x_hat), list(x_ref[0]), obs[:1].tolist())
    assert c - no_obs > cost["obs_collision"] and margin_only > no_obs
