/*
 * FP64 CPU oracle for one MPPI update of a quadrotor (arXiv 2407.09812).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant generator with the HIP library.
 *
 * Everything is computed in IEEE double precision, compiled without fast-math
 * and without FMA contraction, step by step in the order of the paper:
 *   Algorithm 1 (the MPPI iteration), Eqs. (2)-(5) of Sec. III-A,
 *   the quadrotor model, Eqs. (6)-(15) of Sec. III-B,
 *   the tracking cost, Eqs. (16)-(18) and (21) of Sec. IV-C,
 *   the obstacle term, Eq. (22) of Sec. IV-D.
 *
 * Readings of the paper that this file takes (where the text is silent):
 *  - State x = [p(3), q(4) w-first, v(3), omega(3), T(4)]: the paper's 13-dim
 *    state plus the four rotor thrusts of a first-order rotor lag with time
 *    constant tau_m.  tau_m = 0 gives the paper's algebraic model, where the
 *    clipped thrusts act at once (Eq. (13)); the T slots then hold T_cmd.
 *  - The body-rate controller (Eqs. (8)-(12)) runs once per step from x_j and
 *    its clipped command is held over the RK4 step (zero-order hold).
 *  - Hamilton quaternion product, body-to-world rotation, omega in the body
 *    frame, world z up, gravity (0, 0, -g).  q is renormalised after each step.
 *  - R(q) uses the unit-quaternion formula also at the RK4 stage points.
 *  - Cost sums: controls over j = 0..N-1, control changes over j = 0..N-2,
 *    states (tracking and obstacles) over j = 0..N.  The attitude term is
 *    c_q * d_q^2 with d_q = 1 - <q, q_ref>^2, as printed in Eq. (18).
 *  - Obstacle term: c_col * [any obstacle has d < r] plus
 *    w_obs * sum_i max(0, r_i + margin - d_i)^2; sphere d = |p - c|, vertical
 *    cylinder d = |(p - c)_xy|.  With w_obs = 0 this is Eq. (22).
 *  - Noise: counter-based Philox4x32-10 (Salmon et al., SC'11, "Parallel
 *    random numbers: as easy as 1, 2, 3"), key = (seed_lo, vehicle_id),
 *    counter = (k, j, t, seed_hi); uniforms u = (floor(w / 2^9) + 1/2) 2^-23;
 *    Box-Muller pairs (u0, u1) and (u2, u3); delta_u = sigma * z, sigma being
 *    the per-dimension standard deviation.
 *  - Non-finite rollout costs get weight 0; all non-finite is an error and
 *    leaves u_nom unchanged.
 *  - The last slot after the shift is refilled with u_init, an input of
 *    Algorithm 1 (hover, (m g, 0, 0, 0), in the paper).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Parameter blocks, passed in as flat double arrays so that a foreign      */
/* caller needs no struct layout.                                           */
/* ------------------------------------------------------------------------ */

enum { ORC_NX = 17 };

/* vehicle: [mass, Jxx, Jyy, Jzz, arm_l, c_tf, g, T_min, T_max, tau_m, k_rate,
 *           w_xy_max, w_z_max]  (k_rate = 0 -> 1/dt; w_*_max = 0 -> off)   */
typedef struct {
    double m, J[3], l, c_tf, g, T_min, T_max, tau_m, k_rate, w_xy_max, w_z_max;
} orc_vehicle;

/* cost: [c_p, c_v, c_q, c_w, R0..R3, Rd0..Rd3, obs_margin, obs_w, obs_col] */
typedef struct {
    double c_p, c_v, c_q, c_w, R[4], Rd[4], margin, w_obs, c_col;
} orc_cost;

static orc_vehicle unpack_vehicle(const double *a)
{
    orc_vehicle v;
    v.m = a[0]; v.J[0] = a[1]; v.J[1] = a[2]; v.J[2] = a[3];
    v.l = a[4]; v.c_tf = a[5]; v.g = a[6]; v.T_min = a[7]; v.T_max = a[8];
    v.tau_m = a[9]; v.k_rate = a[10]; v.w_xy_max = a[11]; v.w_z_max = a[12];
    return v;
}

static orc_cost unpack_cost(const double *a)
{
    orc_cost c;
    c.c_p = a[0]; c.c_v = a[1]; c.c_q = a[2]; c.c_w = a[3];
    for (int i = 0; i < 4; ++i) { c.R[i] = a[4 + i]; c.Rd[i] = a[8 + i]; }
    c.margin = a[12]; c.w_obs = a[13]; c.c_col = a[14];
    return c;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011).                                      */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {              /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0, 1) from the top 23 bits; exact in binary32 and binary64. */
double orc_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * ldexp(1.0, -23);
}

/* delta_u_j^k ~ N(0, diag(sigma^2))  (Sec. III-A, Eq. (2), first line). */
void orc_noise_one(int k, int j, const double sigma[4], uint64_t seed,
                   uint32_t vehicle_id, uint32_t t, double du[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t ctr[4] = { (uint32_t)k, (uint32_t)j, t, (uint32_t)(seed >> 32) };
    uint32_t key[2] = { (uint32_t)seed, vehicle_id };
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u0 = orc_uniform(w[0]), u1 = orc_uniform(w[1]);
    double u2 = orc_uniform(w[2]), u3 = orc_uniform(w[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    double z[4];
    z[0] = r0 * cos(two_pi * u1);
    z[1] = r0 * sin(two_pi * u1);
    z[2] = r1 * cos(two_pi * u3);
    z[3] = r1 * sin(two_pi * u3);
    for (int d = 0; d < 4; ++d) du[d] = sigma[d] * z[d];
}

/* n independent Philox calls: ctr [n][4], key [n][2], out [n][4]. */
void orc_philox_many(int n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * (size_t)i, key + 2 * (size_t)i, out + 4 * (size_t)i);
}

/* du laid out [K][N][4]. */
void orc_noise(int K, int N, const double sigma[4], uint64_t seed,
               uint32_t vehicle_id, uint32_t t, double *du)
{
    for (int k = 0; k < K; ++k)
        for (int j = 0; j < N; ++j)
            orc_noise_one(k, j, sigma, seed, vehicle_id, t, du + ((size_t)k * N + j) * 4);
}

/* ------------------------------------------------------------------------ */
/* Quadrotor model (Sec. III-B).                                            */
/* ------------------------------------------------------------------------ */

/* Allocation matrix Gamma, Eq. (11), row-major 4x4: [F; tau] = Gamma T. */
void orc_allocation(const double *veh, double G[16])
{
    orc_vehicle v = unpack_vehicle(veh);
    double s = v.l / sqrt(2.0), c = v.c_tf;
    const double rows[16] = {
        1.0, 1.0, 1.0, 1.0,
        -s,  s,   s,  -s,
        -s,  s,  -s,   s,
        -c, -c,   c,   c,
    };
    memcpy(G, rows, sizeof rows);
}

/* Gamma^{-1} by Gauss-Jordan elimination with partial pivoting. */
int orc_allocation_inverse(const double *veh, double Ginv[16])
{
    double A[4][8];
    double G[16];
    orc_allocation(veh, G);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 8; ++c)
            A[r][c] = c < 4 ? G[r * 4 + c] : (c - 4 == r ? 1.0 : 0.0);
    for (int col = 0; col < 4; ++col) {
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int c = 0; c < 8; ++c) { double tmp = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = tmp; }
        double inv = 1.0 / A[col][col];
        for (int c = 0; c < 8; ++c) A[col][c] *= inv;
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            double f = A[r][col];
            for (int c = 0; c < 8; ++c) A[r][c] -= f * A[col][c];
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) Ginv[r * 4 + c] = A[r][c + 4];
    return 0;
}

static void matvec4(const double M[16], const double x[4], double y[4])
{
    for (int r = 0; r < 4; ++r)
        y[r] = M[r * 4 + 0] * x[0] + M[r * 4 + 1] * x[1] + M[r * 4 + 2] * x[2] + M[r * 4 + 3] * x[3];
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Hamilton product r = a (x) b, quaternions w-first. */
static void quat_mul(const double a[4], const double b[4], double r[4])
{
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    r[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* Rotation matrix R(q) (body to world) for a unit quaternion, row-major. */
static void quat_to_rot(const double q[4], double Rm[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    Rm[0] = 1.0 - 2.0 * (y * y + z * z); Rm[1] = 2.0 * (x * y - w * z);       Rm[2] = 2.0 * (x * z + w * y);
    Rm[3] = 2.0 * (x * y + w * z);       Rm[4] = 1.0 - 2.0 * (x * x + z * z); Rm[5] = 2.0 * (y * z - w * x);
    Rm[6] = 2.0 * (x * z - w * y);       Rm[7] = 2.0 * (y * z + w * x);       Rm[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Body-rate controller and saturation, Eqs. (8)-(12): u = [F_t, w_d] -> T_cmd. */
void orc_controller(const double *veh, const double x[ORC_NX], const double u[4],
                    double dt, double T_cmd[4])
{
    orc_vehicle v = unpack_vehicle(veh);
    double Ginv[16];
    orc_allocation_inverse(veh, Ginv);
    const double *w = x + 10;
    double k_w = v.k_rate > 0.0 ? v.k_rate : 1.0 / dt;
    double wdot_d[3], Jw[3], wxJw[3], wrench[4], T_d[4];
    for (int i = 0; i < 3; ++i) {
        wdot_d[i] = k_w * (u[1 + i] - w[i]);                 /* Eq. (8) */
        Jw[i] = v.J[i] * w[i];
    }
    cross3(w, Jw, wxJw);
    wrench[0] = u[0];
    for (int i = 0; i < 3; ++i) wrench[1 + i] = v.J[i] * wdot_d[i] + wxJw[i];   /* Eq. (9) */
    matvec4(Ginv, wrench, T_d);                              /* Eq. (10) */
    for (int i = 0; i < 4; ++i)                              /* Eq. (12) */
        T_cmd[i] = T_d[i] < v.T_min ? v.T_min : (T_d[i] > v.T_max ? v.T_max : T_d[i]);
}

/* Continuous dynamics, Eq. (6), driven by the rotor thrusts (Eq. (13)), plus
 * the first-order rotor lag T' = (T_cmd - T) / tau_m when tau_m > 0. */
void orc_dynamics(const double *veh, const double x[ORC_NX], const double T_cmd[4],
                  double xdot[ORC_NX])
{
    orc_vehicle v = unpack_vehicle(veh);
    double G[16], T[4], wrench[4];
    orc_allocation(veh, G);
    for (int i = 0; i < 4; ++i) T[i] = v.tau_m > 0.0 ? x[13 + i] : T_cmd[i];
    matvec4(G, T, wrench);                                   /* Eq. (13) */
    const double *q = x + 3, *vel = x + 7, *w = x + 10;

    for (int i = 0; i < 3; ++i) xdot[i] = vel[i];            /* p' = v */

    double w_quat[4] = { 0.0, w[0], w[1], w[2] }, qw[4];
    quat_mul(q, w_quat, qw);                                 /* q' = 1/2 q (x) [0, w] */
    for (int i = 0; i < 4; ++i) xdot[3 + i] = 0.5 * qw[i];

    double Rm[9];
    quat_to_rot(q, Rm);                                      /* v' = R(q)[0,0,F]/m + g */
    for (int i = 0; i < 3; ++i) xdot[7 + i] = Rm[i * 3 + 2] * wrench[0] / v.m;
    xdot[9] -= v.g;

    double Jw[3], wxJw[3];
    for (int i = 0; i < 3; ++i) Jw[i] = v.J[i] * w[i];
    cross3(w, Jw, wxJw);                                     /* w' = J^-1 (tau - w x Jw) */
    for (int i = 0; i < 3; ++i) xdot[10 + i] = (wrench[1 + i] - wxJw[i]) / v.J[i];

    for (int i = 0; i < 4; ++i)
        xdot[13 + i] = v.tau_m > 0.0 ? (T_cmd[i] - x[13 + i]) / v.tau_m : 0.0;
}

/* Classic RK4 with the command held, then q <- q / |q|  (Eq. (2), last line). */
void orc_rk4_step(const double *veh, const double x[ORC_NX], const double T_cmd[4],
                  double dt, double x_next[ORC_NX])
{
    orc_vehicle v = unpack_vehicle(veh);
    double k1[ORC_NX], k2[ORC_NX], k3[ORC_NX], k4[ORC_NX], xs[ORC_NX];
    orc_dynamics(veh, x, T_cmd, k1);
    for (int i = 0; i < ORC_NX; ++i) xs[i] = x[i] + 0.5 * dt * k1[i];
    orc_dynamics(veh, xs, T_cmd, k2);
    for (int i = 0; i < ORC_NX; ++i) xs[i] = x[i] + 0.5 * dt * k2[i];
    orc_dynamics(veh, xs, T_cmd, k3);
    for (int i = 0; i < ORC_NX; ++i) xs[i] = x[i] + dt * k3[i];
    orc_dynamics(veh, xs, T_cmd, k4);
    for (int i = 0; i < ORC_NX; ++i)
        x_next[i] = x[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    double nq = sqrt(x_next[3] * x_next[3] + x_next[4] * x_next[4] +
                     x_next[5] * x_next[5] + x_next[6] * x_next[6]);
    for (int i = 3; i < 7; ++i) x_next[i] /= nq;
    if (!(v.tau_m > 0.0))
        for (int i = 0; i < 4; ++i) x_next[13 + i] = T_cmd[i];
}

/* One model step x_{j+1} = x_j + f_RK4(x_j, u_j, dt): controller, then RK4. */
void orc_model_step(const double *veh, const double x[ORC_NX], const double u[4],
                    double dt, double x_next[ORC_NX])
{
    double T_cmd[4];
    orc_controller(veh, x, u, dt, T_cmd);
    orc_rk4_step(veh, x, T_cmd, dt, x_next);
}

/* Feasible input sent to the low-level controller, Eqs. (12)-(15):
 * out = [F_clip, w_clip], w_clip = w + J^-1(tau_clip - w x Jw) dt, with the
 * optional body-rate safety limits applied to w_clip only. */
void orc_applied_input(const double *veh, const double x[ORC_NX], const double u[4],
                       double dt, double out[4])
{
    orc_vehicle v = unpack_vehicle(veh);
    double T_cmd[4], G[16], wrench[4], Jw[3], wxJw[3];
    orc_controller(veh, x, u, dt, T_cmd);
    orc_allocation(veh, G);
    matvec4(G, T_cmd, wrench);
    const double *w = x + 10;
    for (int i = 0; i < 3; ++i) Jw[i] = v.J[i] * w[i];
    cross3(w, Jw, wxJw);
    out[0] = wrench[0];
    for (int i = 0; i < 3; ++i)
        out[1 + i] = w[i] + (wrench[1 + i] - wxJw[i]) / v.J[i] * dt;
    double lim[3] = { v.w_xy_max, v.w_xy_max, v.w_z_max };
    for (int i = 0; i < 3; ++i)
        if (lim[i] > 0.0) {
            if (out[1 + i] > lim[i]) out[1 + i] = lim[i];
            if (out[1 + i] < -lim[i]) out[1 + i] = -lim[i];
        }
}

/* ------------------------------------------------------------------------ */
/* Cost (Sec. IV-C and IV-D).                                               */
/* ------------------------------------------------------------------------ */

/* d_q(q1, q2) = 1 - <q1, q2>^2, Eq. (21). */
double orc_quat_distance(const double q1[4], const double q2[4])
{
    double ip = q1[0] * q2[0] + q1[1] * q2[1] + q1[2] * q2[2] + q1[3] * q2[3];
    return 1.0 - ip * ip;
}

/* rho_ref(x, x_ref), Eq. (18).  x_ref rows are [p, q, v, w] (13 values). */
double orc_tracking_cost(const double *cost, const double x[ORC_NX], const double xr[13])
{
    orc_cost c = unpack_cost(cost);
    double ep = 0.0, ev = 0.0, ew = 0.0;
    for (int i = 0; i < 3; ++i) {
        ep += (x[i] - xr[i]) * (x[i] - xr[i]);
        ev += (x[7 + i] - xr[7 + i]) * (x[7 + i] - xr[7 + i]);
        ew += (x[10 + i] - xr[10 + i]) * (x[10 + i] - xr[10 + i]);
    }
    double dq = orc_quat_distance(x + 3, xr + 3);
    return c.c_p * ep + c.c_q * dq * dq + c.c_v * ev + c.c_w * ew;
}

/* Obstacle term for one position, Eq. (22) with the quadratic margin.
 * obs rows are [type, cx, cy, cz, r], type 0 = sphere, 1 = vertical cylinder. */
double orc_obstacle_cost(const double *cost, const double p[3], const double *obs, int M)
{
    orc_cost c = unpack_cost(cost);
    int collide = 0;
    double pen = 0.0;
    for (int i = 0; i < M; ++i) {
        const double *o = obs + (size_t)i * 5;
        double dx = p[0] - o[1], dy = p[1] - o[2], dz = p[2] - o[3];
        double d = ((int)o[0] == 1) ? sqrt(dx * dx + dy * dy) : sqrt(dx * dx + dy * dy + dz * dz);
        if (d < o[4]) collide = 1;
        double gap = o[4] + c.margin - d;
        if (gap > 0.0) pen += gap * gap;
    }
    return (collide ? c.c_col : 0.0) + c.w_obs * pen;
}

/* S_k of one rollout: states [N+1][17], perturbed controls [N][4],
 * reference [N+1][13]  (Eqs. (16)-(18) and (22)). */
double orc_trajectory_cost(const double *cost, int N, const double *states, const double *u,
                           const double *x_ref, const double *obs, int M)
{
    orc_cost c = unpack_cost(cost);
    double S = 0.0;
    for (int j = 0; j < N; ++j)
        for (int d = 0; d < 4; ++d)
            S += c.R[d] * u[j * 4 + d] * u[j * 4 + d];
    for (int j = 0; j + 1 < N; ++j)
        for (int d = 0; d < 4; ++d) {
            double du = u[(j + 1) * 4 + d] - u[j * 4 + d];
            S += c.Rd[d] * du * du;
        }
    for (int j = 0; j <= N; ++j) {
        const double *x = states + (size_t)j * ORC_NX;
        S += orc_tracking_cost(cost, x, x_ref + (size_t)j * 13);
        S += orc_obstacle_cost(cost, x, obs, M);
    }
    return S;
}

/* ------------------------------------------------------------------------ */
/* The MPPI iteration (Algorithm 1).                                        */
/* ------------------------------------------------------------------------ */

/* Rollout k from x_hat (Eq. (2)) and its cost (Eq. (3)): du_k [N][4],
 * returns S_k; traj (may be NULL) receives the states [N+1][17]. */
double orc_rollout_one(const double *veh, const double *cost, int k, int N, double dt,
                       const double sigma[4], uint64_t seed, uint32_t vehicle_id, uint32_t t,
                       const double *x_hat, const double *u_nom, const double *x_ref,
                       const double *obs, int M, double *traj_out, double *du_k)
{
    double *traj = (double *)malloc(sizeof(double) * (size_t)(N + 1) * ORC_NX);
    double *uk = (double *)malloc(sizeof(double) * (size_t)N * 4);
    memcpy(traj, x_hat, sizeof(double) * ORC_NX);
    for (int j = 0; j < N; ++j) {
        orc_noise_one(k, j, sigma, seed, vehicle_id, t, du_k + j * 4);
        for (int d = 0; d < 4; ++d) uk[j * 4 + d] = u_nom[j * 4 + d] + du_k[j * 4 + d];
        orc_model_step(veh, traj + (size_t)j * ORC_NX, uk + j * 4, dt,
                       traj + (size_t)(j + 1) * ORC_NX);
    }
    double S = orc_trajectory_cost(cost, N, traj, uk, x_ref, obs, M);
    if (traj_out) memcpy(traj_out, traj, sizeof(double) * (size_t)(N + 1) * ORC_NX);
    free(uk);
    free(traj);
    return S;
}

/* K rollouts and their costs.  u_nom [N][4]; x_ref [N+1][13]; outputs du
 * [K][N][4], S [K] and, when not NULL, states [K][N+1][17].  Samples are
 * independent, so the loop over k may run on several threads without changing
 * any result. */
void orc_rollouts(const double *veh, const double *cost, int K, int N, double dt,
                  const double sigma[4], uint64_t seed, uint32_t vehicle_id, uint32_t t,
                  const double *x_hat, const double *u_nom, const double *x_ref,
                  const double *obs, int M, double *states, double *du, double *S)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < K; ++k)
        S[k] = orc_rollout_one(veh, cost, k, N, dt, sigma, seed, vehicle_id, t, x_hat, u_nom,
                               x_ref, obs, M, states ? states + (size_t)k * (N + 1) * ORC_NX : NULL,
                               du + (size_t)k * N * 4);
}

/* The rollouts of the listed sample indices only (outputs indexed like ks). */
void orc_rollouts_subset(const double *veh, const double *cost, int nk, const int *ks, int N,
                         double dt, const double sigma[4], uint64_t seed, uint32_t vehicle_id,
                         uint32_t t, const double *x_hat, const double *u_nom,
                         const double *x_ref, const double *obs, int M, double *states,
                         double *du, double *S)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < nk; ++i)
        S[i] = orc_rollout_one(veh, cost, ks[i], N, dt, sigma, seed, vehicle_id, t, x_hat, u_nom,
                               x_ref, obs, M, states ? states + (size_t)i * (N + 1) * ORC_NX : NULL,
                               du + (size_t)i * N * 4);
}

/* Softmin weights, Eq. (4).  Returns 0, or -1 when no cost is finite.
 * diag (may be NULL) receives [rho, eta, ess = 1 / sum w^2, argmin]. */
int orc_weights(int K, const double *S, double lambda, double *w, double diag[4])
{
    double rho = INFINITY;
    int argmin = -1;
    for (int k = 0; k < K; ++k)
        if (isfinite(S[k]) && S[k] < rho) { rho = S[k]; argmin = k; }
    if (argmin < 0) return -1;
    double eta = 0.0;
    for (int k = 0; k < K; ++k) {
        w[k] = isfinite(S[k]) ? exp(-(S[k] - rho) / lambda) : 0.0;
        eta += w[k];
    }
    double sw2 = 0.0;
    for (int k = 0; k < K; ++k) { w[k] /= eta; sw2 += w[k] * w[k]; }
    if (diag) { diag[0] = rho; diag[1] = eta; diag[2] = 1.0 / sw2; diag[3] = (double)argmin; }
    return 0;
}

/* u_nom_j += sum_k w_k du_j^k, Eq. (5).  du [K][N][4], u_nom [N][4] in place. */
void orc_weighted_update(int K, int N, const double *w, const double *du, double *u_nom)
{
    for (int j = 0; j < N; ++j)
        for (int d = 0; d < 4; ++d) {
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc += w[k] * du[((size_t)k * N + j) * 4 + d];
            u_nom[j * 4 + d] += acc;
        }
}

/* Advance of the warm start by a fraction alpha in (0, 1] of a prediction step
 * (Sec. IV-B, control input interpolation).  The sequence is read as the piecewise-
 * linear function of the step index through the knots u_0..u_{N-1} and
 * u_N = u_init (the refill of Algorithm 1); knot j takes that function's value at
 * j + alpha.  alpha = 1 is Algorithm 1's shift; with the prediction step n times the
 * time between updates, alpha = 1/n. */
void orc_advance(int N, double alpha, const double u_init[4], double *u_nom)
{
    for (int j = 0; j < N; ++j) {            /* knot j + 1 is still the old value */
        const double *next = j + 1 < N ? u_nom + (j + 1) * 4 : u_init;
        for (int d = 0; d < 4; ++d)
            u_nom[j * 4 + d] = (1.0 - alpha) * u_nom[j * 4 + d] + alpha * next[d];
    }
}

/* Apply and advance (Algorithm 1, after the update): u_apply[0..3] = u_nom_0,
 * u_apply[4..7] = feasible [F_clip, w_clip] at x_hat; then the sequence advances by
 * alpha of a step (orc_advance; alpha = 1: u_j <- u_{j+1}, u_{N-1} <- u_init, where
 * Algorithm 1 takes u_init as an input; hover in the paper). */
void orc_apply_shift(const double *veh, int N, double dt, double alpha, const double *x_hat,
                     const double u_init[4], double *u_nom, double u_apply[8])
{
    for (int d = 0; d < 4; ++d) u_apply[d] = u_nom[d];
    orc_applied_input(veh, x_hat, u_nom, dt, u_apply + 4);
    orc_advance(N, alpha, u_init, u_nom);
}

/* Delay compensation by prediction (Sec. IV-E): the state the vehicle reaches after
 * `delay` seconds while the previous command u_hold is executed, from the model with
 * that command held: ceil(delay / dt) equal steps of h <= dt, each the controller of
 * Eqs. (8)-(12) at the step's start (gain from the prediction step dt) followed by one
 * RK4 step of length h.  delay = 0 returns x. */
void orc_predict(const double *veh, double dt, double delay, const double x[ORC_NX],
                 const double u_hold[4], double x_out[ORC_NX])
{
    double cur[ORC_NX], nxt[ORC_NX], T_cmd[4];
    for (int i = 0; i < ORC_NX; ++i) cur[i] = x[i];
    int n = delay > 0.0 ? (int)ceil(delay / dt) : 0;
    double h = n > 0 ? delay / n : 0.0;
    for (int s = 0; s < n; ++s) {
        orc_controller(veh, cur, u_hold, dt, T_cmd);
        orc_rk4_step(veh, cur, T_cmd, h, nxt);
        for (int i = 0; i < ORC_NX; ++i) cur[i] = nxt[i];
    }
    for (int i = 0; i < ORC_NX; ++i) x_out[i] = cur[i];
}

/* One full iteration of Algorithm 1's loop body for a given state estimate.
 * u_nom [N][4] is updated in place (warm start); dt_ctrl is the time between updates
 * (0: one prediction step dt), the warm start advancing by dt_ctrl / dt of a step.  du_out [K][N][4], S_out [K],
 * w_out [K] may be NULL.  Returns 0, or -1 (u_nom untouched) when every
 * rollout cost is non-finite. */
int orc_update(const double *veh, const double *cost, int K, int N, double dt, double lambda,
               const double sigma[4], uint64_t seed, uint32_t vehicle_id, uint32_t t,
               const double u_init[4], double dt_ctrl, const double *x_hat, double *u_nom,
               const double *x_ref, const double *obs, int M, double u_apply[8], double diag[4],
               double *du_out, double *S_out, double *w_out)
{
    double *du = du_out ? du_out : (double *)malloc(sizeof(double) * (size_t)K * N * 4);
    double *S = S_out ? S_out : (double *)malloc(sizeof(double) * (size_t)K);
    double *w = w_out ? w_out : (double *)malloc(sizeof(double) * (size_t)K);
    orc_rollouts(veh, cost, K, N, dt, sigma, seed, vehicle_id, t, x_hat, u_nom, x_ref,
                 obs, M, NULL, du, S);
    int rc = orc_weights(K, S, lambda, w, diag);
    if (rc == 0) {
        orc_weighted_update(K, N, w, du, u_nom);
        double alpha = dt_ctrl > 0.0 ? dt_ctrl / dt : 1.0;   /* Sec. IV-B */
        orc_apply_shift(veh, N, dt, alpha, x_hat, u_init, u_nom, u_apply);
    }
    if (!du_out) free(du);
    if (!S_out) free(S);
    if (!w_out) free(w);
    return rc;
}

/* Threads the per-sample loop runs on (OpenMP; OMP_NUM_THREADS). */
int orc_num_threads(void)
{
    return omp_get_max_threads();
}

/* Set the threads of the per-sample loop (timing runs: one thread, or all cores). */
void orc_set_num_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}
