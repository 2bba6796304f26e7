// Device-side quadrotor model, noise and cost for the MPPI rollouts (gfx950).
//
// Everything here runs per lane in binary32 registers:
//   - counter-based Philox4x32-10 (Salmon et al., SC'11) and Box-Muller, giving
//     the perturbations delta_u ~ N(0, diag(sigma^2)) of Sec. III-A, Eq. (2);
//   - the body-rate controller, allocation and rotor saturation of Sec. III-B,
//     Eqs. (8)-(12), evaluated once per step and held over the step;
//   - the rigid-body dynamics of Eq. (6) driven by the rotor thrusts through the
//     allocation matrix (Eq. (13)), with an optional first-order rotor lag;
//   - one classic RK4 step followed by quaternion renormalisation (Eq. (2));
//   - the per-state tracking cost of Eq. (18) with the quaternion distance of
//     Eq. (21), and the obstacle term of Eq. (22) with a quadratic margin.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

// Vehicle constants, derived on the host from mppi_vehicle for one call.
struct ModelParams {
    float m_inv, g;
    float J[3], J_inv[3];
    // omega x (J omega) = (G0 wy wz, G1 wz wx, G2 wx wy), G = (Jz-Jy, Jx-Jz, Jy-Jx)
    float G[3];
    // Gamma rows 1..3 are s(-1,1,1,-1), s(-1,1,-1,1), c(-1,-1,1,1) with s = l/sqrt(2);
    // Gamma's rows are orthogonal, so Gamma^-1 = Gamma^T diag(1/4, 1/(4s^2), 1/(4s^2), 1/(4c^2)).
    float s, c, inv_4s, inv_4c;
    float T_min, T_max;
    float tau_inv;   // 1 / tau_m (rotor lag); unused when lag == 0
    int lag;         // 0: thrusts equal the clipped command (Eq. (13))
    // RK4 applied to the linear lag T' = (T_cmd - T)/tau_m with T_cmd held gives the
    // thrusts T + c (T_cmd - T) at RK4 stages 2, 3, 4 (c = lag_c[0..2]) and at the end
    // of the step (c = lag_c[3]); with z = dt/tau_m: c1 = z/2, c2 = c1 (1 - c1),
    // c3 = z (1 - c2), c4 = z (6 - 2 c1 - 2 c2 - c3)/6 = 1 - R(-z), R the RK4
    // stability polynomial.
    float lag_c[4];
    float k_w;       // rate-controller gain (1/dt in Eq. (8))
    float dt;
    float w_xy_max, w_z_max;
};

struct CostParams {
    float c_p, c_v, c_q, c_w;
    float R[4], Rd[4];
    float margin, w_obs, c_col;
};

struct NoiseParams {
    float sigma[4];
    uint32_t key0, key1;    // seed low word, vehicle id
    uint32_t t, seed_hi;    // counter words 2 and 3
};

// Scalar parameters of one instance's rollout launch.  obs_tests, when not null,
// accumulates the number of obstacle tests the launch performed (profiling).
struct RolloutParams {
    ModelParams mp;
    CostParams cp;
    NoiseParams np;
    int M, K, N, ld;
    unsigned long long* obs_tests;
};

constexpr int kWeightsThreads = 1024;   // one workgroup computes one instance's weights
constexpr int kSumThreads = 256;        // one workgroup reduces one delta_u row

// 17 state values held in registers.
// Per-wave partial results of the single-pass update (written by the rollout
// kernel's epilogue, read by the merge).
struct WaveStat {
    float rho;            // minimum finite cost of the wave (+inf if none)
    float eta_s, eta_c;   // compensated sum of exp(-(S_k - rho) / lambda)
    float q;              // sum of their squares
    int argmin;           // first sample attaining rho (-1 if none)
    int n;                // finite costs
    int skipped;          // 1: every weight underflows, no partial sums written
    int pad;
};

constexpr int kMergeThreads = 256;   // single-pass sum workgroup: 64 columns x 4 waves
constexpr float kSkipLog2 = 160.0f;  // waves whose weights are all below 2^-160 skip

struct State {
    float px, py, pz;
    float qw, qx, qy, qz;
    float vx, vy, vz;
    float wx, wy, wz;
    float T0, T1, T2, T3;
};

// ---------------------------------------------------------------------------
// Noise
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;   // one v_mad_u64_u32 each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// ((w >> 9) + 0.5) * 2^-23 in (0, 1): the bit pattern 1.m minus (1 - 2^-24) is
// exact because the result (2m + 1) 2^-24 is representable.
__device__ __forceinline__ float unit_uniform(uint32_t w)
{
    return __uint_as_float((w >> 9) | 0x3F800000u) - 0.99999994f;
}

// v as computed, in a register of its own: the empty asm statement hides how v was
// produced, so the compiler cannot fuse its producing multiply into a consumer.  Values
// that the kernels hand over between waves or lanes pass through it everywhere, so
// that every launch shape computes them -- and what follows -- the same way.
__device__ __forceinline__ float opaque(float v)
{
    asm("" : "+v"(v));
    return v;
}

// delta_u for sample k, step j: Philox counter (k, j, t, seed_hi), Box-Muller on
// (u0, u1) and (u2, u3).  v_sin/v_cos take revolutions, so sin(2 pi u) is one op.
__device__ __forceinline__ void draw_noise(const NoiseParams& np, uint32_t k, uint32_t j,
                                           float du[4])
{
    const uint4 w = philox4x32_10(make_uint4(k, j, np.t, np.seed_hi), np.key0, np.key1);
    const float u0 = unit_uniform(w.x), u1 = unit_uniform(w.y);
    const float u2 = unit_uniform(w.z), u3 = unit_uniform(w.w);
    const float neg2ln2 = -1.38629436112f;   // -2 ln 2: ln u = ln 2 * log2 u
    const float r0 = __builtin_amdgcn_sqrtf(neg2ln2 * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(neg2ln2 * __builtin_amdgcn_logf(u2));
    du[0] = opaque(np.sigma[0] * (r0 * __builtin_amdgcn_cosf(u1)));
    du[1] = opaque(np.sigma[1] * (r0 * __builtin_amdgcn_sinf(u1)));
    du[2] = opaque(np.sigma[2] * (r1 * __builtin_amdgcn_cosf(u3)));
    du[3] = opaque(np.sigma[3] * (r1 * __builtin_amdgcn_sinf(u3)));
}

// ---------------------------------------------------------------------------
// Controller and allocation (Eqs. (8)-(12))
// ---------------------------------------------------------------------------

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return fminf(fmaxf(v, lo), hi);
}

// u = [F_t, omega_d]; returns the clipped rotor command.
__device__ __forceinline__ void rate_controller(const ModelParams& P, float wx, float wy, float wz,
                                                const float u[4], float Tc[4])
{
    // Eq. (8): omega_dot_d = k_w (omega_d - omega); Eq. (9): tau_d = J omega_dot_d + omega x J omega
    const float tx = fmaf(P.J[0], P.k_w * (u[1] - wx), P.G[0] * (wy * wz));
    const float ty = fmaf(P.J[1], P.k_w * (u[2] - wy), P.G[1] * (wz * wx));
    const float tz = fmaf(P.J[2], P.k_w * (u[3] - wz), P.G[2] * (wx * wy));
    // Eq. (10) with Gamma^-1 = Gamma^T D^-1
    const float a0 = 0.25f * u[0], a1 = tx * P.inv_4s, a2 = ty * P.inv_4s, a3 = tz * P.inv_4c;
    const float p = a0 - a3, m = a0 + a3;
    Tc[0] = clampf(p - a1 - a2, P.T_min, P.T_max);   // Eq. (12)
    Tc[1] = clampf(p + a1 + a2, P.T_min, P.T_max);
    Tc[2] = clampf(m + a1 - a2, P.T_min, P.T_max);
    Tc[3] = clampf(m - a1 + a2, P.T_min, P.T_max);
}

// ---------------------------------------------------------------------------
// Dynamics (Eq. (6)) and RK4 (Eq. (2))
// ---------------------------------------------------------------------------

// Collective thrust and body torques of four rotor thrusts, Eq. (13): [F; tau] = Gamma T.
struct Wrench {
    float F, tx, ty, tz;
};

__device__ __forceinline__ Wrench allocate(const ModelParams& P, float T0, float T1, float T2,
                                           float T3)
{
    const float s01 = T0 + T1, s23 = T2 + T3, d10 = T1 - T0, d23 = T2 - T3;
    return Wrench{s01 + s23, P.s * (d10 + d23), P.s * (d10 - d23), P.c * (s23 - s01)};
}

// Attitude, velocity and body rate: the part of the state the right-hand side of
// Eq. (6) depends on (it does not depend on the position).
// Accelerations v' at the four RK4 stage points of one step.
struct StageAccel {
    float x[4], y[4], z[4];
};

// One step x <- x + f_RK4(x, Tc, dt) with the command held, then q <- q / |q|.
// This is classic RK4 on the 17-value state, arranged to skip work that is known in
// closed form: the wrench at each stage point comes from the stage thrusts of the
// linear lag (W(T) + c_s W(T_cmd - T), exact since the allocation is linear), and
// since nothing depends on the position its update is p + h v + h^2/6 (a1 + a2 + a3),
// which is what RK4's four stage velocities sum to.  Nothing in the rotational part
// (q, omega, T) depends on p or v, and omega' depends on omega and the thrusts only,
// so the step splits into three chains: rk4_rates (omega, T), rk4_attitude (q, given
// the stage rates and thrusts, with the stage accelerations) and rk4_translational
// (p, v from the stage accelerations).  Values handed from one chain to the next go
// through opaque(), so every kernel that splits them across waves computes the same.

// Body rates, stage by stage: omega at the four RK4 stage points and the collective
// thrust there (the rates part of rk4_rotational; omega' depends on omega and the
// thrusts only).
struct RateStages {
    float wx[4], wy[4], wz[4], F[4];
};

template <bool kLag>
__device__ __forceinline__ void rk4_rates(const ModelParams& P, State& x, const float Tc[4],
                                          RateStages& R)
{
    const float h = P.dt, h2 = 0.5f * P.dt, h6 = P.dt * (1.0f / 6.0f);
    Wrench Ws[4];
    float D0 = 0.0f, D1 = 0.0f, D2 = 0.0f, D3 = 0.0f;
    if (kLag) {
        D0 = Tc[0] - x.T0; D1 = Tc[1] - x.T1; D2 = Tc[2] - x.T2; D3 = Tc[3] - x.T3;
        const Wrench W0 = allocate(P, x.T0, x.T1, x.T2, x.T3);
        const Wrench dW = allocate(P, D0, D1, D2, D3);
        Ws[0] = W0;
#define MPPI_STAGE_WRENCH(Wd, c) \
        Wd = Wrench{fmaf(c, dW.F, W0.F), fmaf(c, dW.tx, W0.tx), fmaf(c, dW.ty, W0.ty), fmaf(c, dW.tz, W0.tz)};
        MPPI_STAGE_WRENCH(Ws[1], P.lag_c[0])
        MPPI_STAGE_WRENCH(Ws[2], P.lag_c[1])
        MPPI_STAGE_WRENCH(Ws[3], P.lag_c[2])
#undef MPPI_STAGE_WRENCH
    } else {
        Ws[0] = Ws[1] = Ws[2] = Ws[3] = allocate(P, Tc[0], Tc[1], Tc[2], Tc[3]);
    }
    const float bx = x.wx, by = x.wy, bz = x.wz;
    float sx = bx, sy = by, sz = bz, ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        sx = opaque(sx); sy = opaque(sy); sz = opaque(sz);
        R.wx[s] = sx; R.wy[s] = sy; R.wz[s] = sz;
        R.F[s] = opaque(Ws[s].F);
        // omega' = J^-1 (tau - omega x J omega)
        const float kx = (Ws[s].tx - P.G[0] * (sy * sz)) * P.J_inv[0];
        const float ky = (Ws[s].ty - P.G[1] * (sz * sx)) * P.J_inv[1];
        const float kz = (Ws[s].tz - P.G[2] * (sx * sy)) * P.J_inv[2];
        if (s == 0) {
            ax = kx; ay = ky; az = kz;
            sx = fmaf(h2, kx, bx); sy = fmaf(h2, ky, by); sz = fmaf(h2, kz, bz);
        } else if (s == 1) {
            ax = fmaf(2.0f, kx, ax); ay = fmaf(2.0f, ky, ay); az = fmaf(2.0f, kz, az);
            sx = fmaf(h2, kx, bx); sy = fmaf(h2, ky, by); sz = fmaf(h2, kz, bz);
        } else if (s == 2) {
            ax = fmaf(2.0f, kx, ax); ay = fmaf(2.0f, ky, ay); az = fmaf(2.0f, kz, az);
            sx = fmaf(h, kx, bx); sy = fmaf(h, ky, by); sz = fmaf(h, kz, bz);
        } else {
            x.wx = fmaf(h6, ax + kx, bx); x.wy = fmaf(h6, ay + ky, by); x.wz = fmaf(h6, az + kz, bz);
        }
    }
    if (kLag) {
        x.T0 = fmaf(P.lag_c[3], D0, x.T0); x.T1 = fmaf(P.lag_c[3], D1, x.T1);
        x.T2 = fmaf(P.lag_c[3], D2, x.T2); x.T3 = fmaf(P.lag_c[3], D3, x.T3);
    } else {
        x.T0 = Tc[0]; x.T1 = Tc[1]; x.T2 = Tc[2]; x.T3 = Tc[3];
    }
}

// Attitude over one step from the stage rates and thrusts of rk4_rates, with the stage
// accelerations v' = R(q) [0, 0, F] / m + [0, 0, -g]; then q <- q / |q|.
__device__ __forceinline__ void rk4_attitude(const ModelParams& P, State& x, const RateStages& R,
                                             StageAccel& A)
{
    const float h = P.dt, h2 = 0.5f * P.dt, h6 = P.dt * (1.0f / 6.0f);
    const float bw = x.qw, bx = x.qx, by = x.qy, bz = x.qz;
    float qw = bw, qx = bx, qy = by, qz = bz;
    float aw = 0.0f, ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        // q' = 1/2 q (x) [0, omega]
        const float hx = 0.5f * R.wx[s], hy = 0.5f * R.wy[s], hz = 0.5f * R.wz[s];
        const float kw = -(qx * hx + qy * hy + qz * hz);
        const float kx = qw * hx + qy * hz - qz * hy;
        const float ky = qw * hy - qx * hz + qz * hx;
        const float kz = qw * hz + qx * hy - qy * hx;
        // third column of R(q)
        const float fm = R.F[s] * P.m_inv, f2 = fm + fm;
        A.x[s] = opaque(f2 * (qx * qz + qw * qy));
        A.y[s] = opaque(f2 * (qy * qz - qw * qx));
        A.z[s] = opaque(fm - f2 * (qx * qx + qy * qy) - P.g);
        if (s == 0) {
            aw = kw; ax = kx; ay = ky; az = kz;
            qw = fmaf(h2, kw, bw); qx = fmaf(h2, kx, bx); qy = fmaf(h2, ky, by); qz = fmaf(h2, kz, bz);
        } else if (s == 1) {
            aw = fmaf(2.0f, kw, aw); ax = fmaf(2.0f, kx, ax); ay = fmaf(2.0f, ky, ay); az = fmaf(2.0f, kz, az);
            qw = fmaf(h2, kw, bw); qx = fmaf(h2, kx, bx); qy = fmaf(h2, ky, by); qz = fmaf(h2, kz, bz);
        } else if (s == 2) {
            aw = fmaf(2.0f, kw, aw); ax = fmaf(2.0f, kx, ax); ay = fmaf(2.0f, ky, ay); az = fmaf(2.0f, kz, az);
            qw = fmaf(h, kw, bw); qx = fmaf(h, kx, bx); qy = fmaf(h, ky, by); qz = fmaf(h, kz, bz);
        } else {
            x.qw = fmaf(h6, aw + kw, bw); x.qx = fmaf(h6, ax + kx, bx);
            x.qy = fmaf(h6, ay + ky, by); x.qz = fmaf(h6, az + kz, bz);
        }
    }
    const float n2 = x.qw * x.qw + x.qx * x.qx + x.qy * x.qy + x.qz * x.qz;
    const float inv = __builtin_amdgcn_rsqf(n2);
    x.qw *= inv; x.qx *= inv; x.qy *= inv; x.qz *= inv;
}

// The rotational half of the step: body rates and thrusts, then the attitude.
template <bool kLag>
__device__ __forceinline__ void rk4_rotational(const ModelParams& P, State& x, const float Tc[4],
                                               StageAccel& A)
{
    RateStages R;
    rk4_rates<kLag>(P, x, Tc, R);
    rk4_attitude(P, x, R, A);
}

// p and v over the step from the stage accelerations of rk4_rotational.
__device__ __forceinline__ void rk4_translational(const ModelParams& P, State& x, const StageAccel& A)
{
    const float h = P.dt, h6 = P.dt * (1.0f / 6.0f), hh6 = h * h6;
    const float ax = (A.x[0] + A.x[1]) + A.x[2];
    const float ay = (A.y[0] + A.y[1]) + A.y[2];
    const float az = (A.z[0] + A.z[1]) + A.z[2];
    x.px = fmaf(hh6, ax, fmaf(h, x.vx, x.px));
    x.py = fmaf(hh6, ay, fmaf(h, x.vy, x.py));
    x.pz = fmaf(hh6, az, fmaf(h, x.vz, x.pz));
    x.vx = fmaf(h6, fmaf(2.0f, A.x[2], fmaf(2.0f, A.x[1], A.x[0])) + A.x[3], x.vx);
    x.vy = fmaf(h6, fmaf(2.0f, A.y[2], fmaf(2.0f, A.y[1], A.y[0])) + A.y[3], x.vy);
    x.vz = fmaf(h6, fmaf(2.0f, A.z[2], fmaf(2.0f, A.z[1], A.z[0])) + A.z[3], x.vz);
}

template <bool kLag>
__device__ __forceinline__ void rk4_step(const ModelParams& P, State& x, const float Tc[4])
{
    StageAccel A;
    rk4_rotational<kLag>(P, x, Tc, A);
    rk4_translational(P, x, A);
}

// ---------------------------------------------------------------------------
// Cost (Eqs. (16)-(22))
// ---------------------------------------------------------------------------

// rho_ref (Eq. (18)) for a state against a reference row [p, q, v, omega]; the
// reference position is given relative to the frame origin of the state.
__device__ __forceinline__ float tracking_cost(const CostParams& C, const State& x,
                                               float rpx, float rpy, float rpz, const float* ref)
{
    const float dx = x.px - rpx, dy = x.py - rpy, dz = x.pz - rpz;
    const float ip = x.qw * ref[3] + x.qx * ref[4] + x.qy * ref[5] + x.qz * ref[6];
    const float dq = fmaf(-ip, ip, 1.0f);                        // Eq. (21)
    const float ex = x.vx - ref[7], ey = x.vy - ref[8], ez = x.vz - ref[9];
    const float ox = x.wx - ref[10], oy = x.wy - ref[11], oz = x.wz - ref[12];
    float c = C.c_p * (dx * dx + dy * dy + dz * dz);
    c = fmaf(C.c_q, dq * dq, c);
    c = fmaf(C.c_v, ex * ex + ey * ey + ez * ez, c);
    c = fmaf(C.c_w, ox * ox + oy * oy + oz * oz, c);
    return c;
}

// Sum / OR over the L consecutive lanes that share one sample: DPP quad permutations
// (xor 1, xor 2), then for eight lanes the half-row mirror, which pairs each lane of
// one quad with a lane of the other (both quads already hold their sums).  Every lane
// of the group ends with the same value (the additions pair the same operands).
__device__ __forceinline__ float dpp_xor1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_xor2(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}

template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    if (L >= 2) v += dpp_xor1(v);
    if (L >= 4) v += dpp_xor2(v);
    if (L >= 8)
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
    return v;
}

// Minimum and maximum over the 64 lanes of the wave (all lanes active), returned in
// scalar registers.  The values are mapped to integer keys that order like the floats
// (the sign flips the magnitude bits), so that each butterfly step within a row of 16
// (quad permutations, half-row and row mirrors) is one DPP integer min or max; the row
// broadcasts 15 and 31 then fold the rows into lane 63, which alone is read (rows a
// broadcast does not write keep values that never reach lane 63).  A NaN lane enters
// the minimum as -inf and the maximum as +inf: it widens the range of the others and
// never shrinks it.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kCtrl, kRowMask, 0xF, false));
}

__device__ __forceinline__ int order_key(float f)
{
    const int b = __float_as_int(f);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float from_order_key(int k)
{
    return __int_as_float(k ^ ((k >> 31) & 0x7fffffff));
}

template <int D, int kCtrl, int kRowMask>
__device__ __forceinline__ void key_range_step(int (&lo)[D], int (&hi)[D])
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = min(lo[d], __builtin_amdgcn_mov_dpp(lo[d], kCtrl, kRowMask, 0xF, true));
        hi[d] = max(hi[d], __builtin_amdgcn_mov_dpp(hi[d], kCtrl, kRowMask, 0xF, true));
    }
}

// A lane's key range of value v, merged into (lo, hi): NaN keys lie beyond the
// infinities, so a NaN widens the range to an infinity and never narrows it.
__device__ __forceinline__ void key_range_of(float v, int& lo, int& hi)
{
    const int k = order_key(v);
    lo = min(lo, max(k, order_key(-INFINITY)));
    hi = max(hi, min(k, order_key(INFINITY)));
}

// The ranges (lo, hi) of each lane merged over each group of G consecutive lanes (G =
// 8, 16, 32 or 64), in every lane of the group (G = 64: read from lane 63, uniform).
template <int D, int G>
__device__ __forceinline__ void key_ranges_merge(int (&lo)[D], int (&hi)[D])
{
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "group of 8, 16, 32 or 64 lanes");
    key_range_step<D, 0xB1, 0xF>(lo, hi);              // quad_perm [1, 0, 3, 2]
    key_range_step<D, 0x4E, 0xF>(lo, hi);              // quad_perm [2, 3, 0, 1]
    key_range_step<D, 0x141, 0xF>(lo, hi);             // row_half_mirror: 8 lanes
    if (G >= 16) key_range_step<D, 0x140, 0xF>(lo, hi);  // row_mirror: 16 lanes
    if (G >= 32) key_range_step<D, 0x142, 0xA>(lo, hi);  // row_bcast:15 into rows 1 and 3
    if (G == 64) {
        key_range_step<D, 0x143, 0xC>(lo, hi);         // row_bcast:31 into rows 2 and 3
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = __builtin_amdgcn_readlane(lo[d], 63);
            hi[d] = __builtin_amdgcn_readlane(hi[d], 63);
        }
    } else if (G == 32) {
        const bool low = (__lane_id() & 32) == 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int l0 = __builtin_amdgcn_readlane(lo[d], 31), l1 = __builtin_amdgcn_readlane(lo[d], 63);
            const int h0 = __builtin_amdgcn_readlane(hi[d], 31), h1 = __builtin_amdgcn_readlane(hi[d], 63);
            lo[d] = low ? l0 : l1;
            hi[d] = low ? h0 : h1;
        }
    }
}

// Key ranges of D values per lane over each group of G consecutive lanes.
template <int D, int G>
__device__ __forceinline__ void key_ranges(const float (&v)[D], int (&lo)[D], int (&hi)[D])
{
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = order_key(INFINITY) + 1;    // above every key key_range_of keeps
        hi[d] = order_key(-INFINITY) - 1;
        key_range_of(v[d], lo[d], hi[d]);
    }
    key_ranges_merge<D, G>(lo, hi);
}

__device__ __forceinline__ void wave_range(float v, float& lo, float& hi)
{
    const float vv[1] = {v};
    int l[1], h[1];
    key_ranges<1, 64>(vv, l, h);
    lo = from_order_key(l[0]);
    hi = from_order_key(h[0]);
}

// Minimum and maximum over each group of G consecutive lanes (G = 8, 16, 32 or 64),
// returned in every lane of the group.  NaN lanes are handled as in wave_range.
template <int G>
__device__ __forceinline__ void group_range(float v, float& lo, float& hi)
{
    const float vv[1] = {v};
    int l[1], h[1];
    key_ranges<1, G>(vv, l, h);
    lo = from_order_key(l[0]);
    hi = from_order_key(h[0]);
}

// Obstacles in LDS, one block per workgroup (see stage_obstacles):
//   float4 header (x0, 1 / bin width, R_max + slack, culling on)
//   kObsBins + 1 bin starts (int, padded to 68): first obstacle with x >= x0 + b w;
//     int kObsSphereSlot of the padding: 1 if any obstacle is a sphere, else 0
//   two float4 per obstacle, sorted by x:
//     a = (cx, cy, cz, zmask)  centre relative to the frame origin; zmask 0 for a
//                              vertical cylinder (ignore z), 1 for a sphere
//     b = (r^2, (r + margin)^2, r + margin, 0)
//   then kObsPad padding entries a = 0, b = (-inf, -inf, 0, 0), which no distance is
//   below: obstacle_cost reads up to 2 L max(U, 2) - 1 entries past the last obstacle.
constexpr int kObsBins = 64;
constexpr int kObsHeaderFloat4 = 1 + 68 / 4;        // header + padded bin table
constexpr int kObsSphereSlot = kObsBins + 1;        // bin-table int: any sphere in the block
constexpr int kObsPad = 64;                         // >= 2 L max(U, 2) - 1, L <= 8, U <= 4
constexpr int kCullMin = 16, kCullMax = 512;       // sorted and culled for M in this range
constexpr int kCullKeysInLds = 64;                 // from this M the sort ranks keys in LDS
constexpr float kCullSlack = 1.0e-3f;              // m, covers rounding of the x tests

// float4 slots of the obstacle block (header, bins, obstacles, padding).
__host__ __device__ constexpr int obstacle_lds_float4(int M)
{
    return kObsHeaderFloat4 + 2 * ((M > 0 ? M : 0) + kObsPad);
}
__host__ __device__ constexpr size_t obstacle_lds_bytes(int M)
{
    return sizeof(float4) * (size_t)obstacle_lds_float4(M);
}

// Obstacle term of Eq. (22) (with the quadratic margin) for this lane's position; h is
// the block's header.  Lane q of a sample's L lanes tests obstacles q, q + L, ...; the partial penalties and
// hit flags are combined over the group.  With culling on, the wave first takes the
// x-range of all its lanes' positions and tests only obstacles whose centre lies
// within R_max + slack of that range: every other obstacle is farther than its
// r + margin from every lane, so it adds exactly zero to the penalty and to the hit.
// Every lane runs the same number of tests, ceil(window / L) rounded up to R = max(U,
// 2); the indices past the window reach obstacles outside it or the padding, which add
// exactly zero, so the result is that of testing the window alone, in the same order.
// The culling window [i0, i1) for the positions px of the wave's lanes (all active),
// from the block's header h (read once by the caller).  obstacle_bins_of issues the
// bin reads for a given x-range [lo, hi] of positions and leaves their values in
// registers, so that a caller can do other work before it uses them; obstacle_bins
// takes the range of the whole wave.
__device__ __forceinline__ void obstacle_bins_of(const float4 h, const float4* __restrict__ blk,
                                                 float lo, float hi, int& v0, int& v1)
{
    const int* bins = reinterpret_cast<const int*>(blk + 1);
    lo -= h.z;
    hi += h.z;
    const float b0 = fminf(fmaxf(floorf((lo - h.x) * h.y), 0.0f), (float)kObsBins);
    const float b1 = fminf(fmaxf(floorf((hi - h.x) * h.y) + 1.0f, 0.0f), (float)kObsBins);
    v0 = bins[(int)b0];
    v1 = bins[(int)b1];
}

__device__ __forceinline__ void obstacle_bins(const float4 h, const float4* __restrict__ blk,
                                              float px, int M, int& v0, int& v1)
{
    v0 = 0;
    v1 = M;
    if (h.w != 0.0f) {
        float lo, hi;
        wave_range(px, lo, hi);
        obstacle_bins_of(h, blk, lo, hi, v0, v1);
    }
}

__device__ __forceinline__ void obstacle_window(const float4 h, const float4* __restrict__ blk,
                                                float px, int M, int& i0, int& i1)
{
    int v0, v1;
    obstacle_bins(h, blk, px, M, v0, v1);
    i0 = __builtin_amdgcn_readfirstlane(v0);
    i1 = __builtin_amdgcn_readfirstlane(v1);
}

// The tests of obstacles [i0, i1) (uniform over the wave): any window that contains the
// culling window of every lane in the wave gives the same result.
// kZ false: every obstacle of the block is a vertical cylinder (z is not read).
template <int L, int U, bool kZ = true>
__device__ __forceinline__ float obstacle_tests(const CostParams& C, float px, float py, float pz,
                                                const float4* __restrict__ blk, int i0, int i1, int q,
                                                int& tested)
{
    tested += i1 - i0;                     // obstacles each sample of this wave tests
    // R register slots, each holding one test's operands: a slot is scored, then
    // refilled with the test R further on, whose loads are in flight while the other
    // slots are scored.  Lane's test t reads o[2 L t] and o[2 L t + 1].
    constexpr int R = U < 2 ? 2 : U;
    const int n = (i1 - i0 + (L - 1)) / L;                      // tests per lane, uniform
    const float4* o = blk + kObsHeaderFloat4 + 2 * (i0 + q);
    // no scalar load may be outstanding when the loop starts: those return out of
    // order, and with one pending every wait in the loop would be for all LDS loads
    // rather than for the oldest slot's
    __builtin_amdgcn_s_waitcnt(0xC07F);                         // lgkmcnt(0) only
    float4 a[R], b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        a[r] = o[2 * L * r];
        b[r] = o[2 * L * r + 1];
        __builtin_amdgcn_sched_barrier(0);     // issued in slot order, as in the loop
    }
    float hits[R], pen = 0.0f;             // a hit flag per slot, so each slot's operands
#pragma unroll                             // are dead once it has been scored
    for (int r = 0; r < R; ++r) hits[r] = 0.0f;
    for (int t = 0; t < n; t += R) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = px - a[r].x, dy = py - a[r].y;
            float d2;
            if (kZ) {
                const float dz = (pz - a[r].z) * a[r].w;
                d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            } else {   // a cylinder's dz is 0 (zmask 0), and fma(dy, dy, 0) rounds as dy * dy
                d2 = fmaf(dx, dx, dy * dy);
            }
            hits[r] = d2 < b[r].x ? 1.0f : hits[r];
            if (d2 < b[r].y) {
                const float gap = b[r].z - __builtin_amdgcn_sqrtf(d2);
                pen = fmaf(gap, gap, pen);
            }
            a[r] = o[2 * L * (t + R + r)];            // index < M + 2 L R - 1 (padding)
            b[r] = o[2 * L * (t + R + r) + 1];
            // compiler-only barriers: without them the refill is folded into a load at
            // the top of the next iteration, or scheduled after the other slots' tests
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    float hit = hits[0];
#pragma unroll
    for (int r = 1; r < R; ++r) hit = hits[r] > 0.0f ? 1.0f : hit;
    if (L > 1) {
        pen = group_sum<L>(pen);
        hit = group_sum<L>(hit);
    }
    return fmaf(C.w_obs, pen, hit > 0.0f ? C.c_col : 0.0f);
}

// The box of the wave's positions (all lanes active), in scalar registers: the three
// ranges of wave_range, interleaved (a NaN coordinate widens the box, never shrinks it).
struct WaveBox {
    float xlo, xhi, ylo, yhi, zlo, zhi;
};

__device__ __forceinline__ WaveBox wave_box(float px, float py, float pz)
{
    const float v[3] = {px, py, pz};
    int lo[3], hi[3];
    key_ranges<3, 64>(v, lo, hi);
    return WaveBox{from_order_key(lo[0]), from_order_key(hi[0]), from_order_key(lo[1]),
                   from_order_key(hi[1]), from_order_key(lo[2]), from_order_key(hi[2])};
}

// Culling by the wave's box of positions.  Among obstacles [i0, i1) only those whose
// centre lies within R (the block's R_max + slack) of the box can reach a lane: the
// distance to a vertical cylinder is at least |dx| and |dy|, to a sphere at least |dx|,
// |dy| and |dz|, so every other obstacle is farther than its r + margin from every lane
// and adds exactly zero to the penalty and to the hit.  The near obstacles are found 64
// at a time, one per lane (near_block), then tested in increasing index order, the
// c-th of a block by lane c mod L of each sample (the L lanes of a sample divide its
// tests), with S register slots as in obstacle_tests: a slot is scored, then refilled
// with the candidate S rounds further on (near_tests).  Lanes left without a candidate
// test the padding entry at index M, which adds zero.  With L = 1 the penalty is summed
// in the order of obstacle_tests over the same window, term for term (the skipped
// obstacles add nothing there either).
struct NearLimits {
    float xl, xh, yl, yh, zl, zh;
};

__device__ __forceinline__ NearLimits near_limits(const WaveBox& bx, float R)
{
    return NearLimits{bx.xlo - R, bx.xhi + R, bx.ylo - R, bx.yhi + R, bx.zlo - R, bx.zhi + R};
}

// One block of 64 obstacles [base, min(base + 64, i1)): lane l's obstacle base + l, whose
// centre c the caller has loaded (o[2 min(base + l, ...)]; any entry past i1).  m: the
// near ones (bit l), cnt of them; with L > 1 a forward permute (ds_permute, no memory)
// also sends the index of the c-th near obstacle to lane c (the others send the padding
// index M to the lanes after the last candidate).
struct NearBlock {
    uint64_t m;
    int cnt, base, cand;
};

template <int L>
__device__ __forceinline__ NearBlock near_block(const float4 c, int base, int i1, int M,
                                                const NearLimits& lim)
{
    const int lane = __lane_id(), i = base + lane;
    const bool near = i < i1 && c.x >= lim.xl && c.x <= lim.xh && c.y >= lim.yl &&
                      c.y <= lim.yh && (c.w == 0.0f || (c.z >= lim.zl && c.z <= lim.zh));
    NearBlock nb;
    nb.m = __ballot(near);
    nb.cnt = __popcll(nb.m);
    nb.base = base;
    nb.cand = M;
    if (L > 1) {
        const int below = __builtin_amdgcn_mbcnt_hi((uint32_t)(nb.m >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)nb.m, 0u));
        const int dst = near ? below : nb.cnt + (lane - below);   // a permutation of the lanes
        nb.cand = __builtin_amdgcn_ds_permute(dst << 2, near ? i : M);
    }
    return nb;
}

// The near obstacles of block nb tested at this lane's position (lane q of its sample),
// accumulated into the slots' hit flags and the penalty.
template <int L, int U>
__device__ __forceinline__ void near_tests(const float4* __restrict__ o, NearBlock nb, int M, int q,
                                           float px, float py, float pz,
                                           float (&hits)[U < 2 ? 2 : U], float& pen)
{
    constexpr int S = U < 2 ? 2 : U;
    // the candidate of the next round for this lane: with L = 1 the lowest bit left in
    // the (uniform) mask; else lane L t + q of the permuted indices
    int round = 0;
    auto next = [&]() {
        int sel = M;
        if (L == 1) {
            if (nb.m != 0) {
                sel = nb.base + __builtin_ctzll(nb.m);
                nb.m &= nb.m - 1;
            }
        } else {
            const int src = L * round + q;
            const int v = __builtin_amdgcn_ds_bpermute(src << 2, nb.cand);
            sel = src < nb.cnt ? v : M;
        }
        ++round;
        return sel;
    };
    float4 a[S], b[S];
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const int sr = next();
        a[r] = o[2 * sr];
        b[r] = o[2 * sr + 1];
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int t = 0; t < nb.cnt; t += L * S) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const float dx = px - a[r].x, dy = py - a[r].y, dz = (pz - a[r].z) * a[r].w;
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            hits[r] = d2 < b[r].x ? 1.0f : hits[r];
            if (d2 < b[r].y) {
                const float gap = b[r].z - __builtin_amdgcn_sqrtf(d2);
                pen = fmaf(gap, gap, pen);
            }
            const int sr = next();
            a[r] = o[2 * sr];
            b[r] = o[2 * sr + 1];
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// near_tests for the C positions p[0..C) of this lane's sample (the steps of a chunk):
// each candidate's operands are loaded once and tested at every position; per position
// the hit flags and the penalty are accumulated as near_tests does for one (kZ false:
// a block of vertical cylinders only, whose z terms are 0).
template <int L, int U, bool kZ, int C>
__device__ __forceinline__ void near_tests_chunk(const float4* __restrict__ o, NearBlock nb, int M,
                                                 int q, const float4 (&p)[C],
                                                 float (&hits)[C][U < 2 ? 2 : U], float (&pen)[C])
{
    constexpr int S = U < 2 ? 2 : U;
    int round = 0;
    auto next = [&]() {
        int sel = M;
        if (L == 1) {
            if (nb.m != 0) {
                sel = nb.base + __builtin_ctzll(nb.m);
                nb.m &= nb.m - 1;
            }
        } else {
            const int src = L * round + q;
            const int v = __builtin_amdgcn_ds_bpermute(src << 2, nb.cand);
            sel = src < nb.cnt ? v : M;
        }
        ++round;
        return sel;
    };
    float4 a[S], b[S];
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const int sr = next();
        a[r] = o[2 * sr];
        b[r] = o[2 * sr + 1];
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int t = 0; t < nb.cnt; t += L * S) {
#pragma unroll
        for (int r = 0; r < S; ++r) {
#pragma unroll
            for (int s = 0; s < C; ++s) {
                const float dx = p[s].x - a[r].x, dy = p[s].y - a[r].y;
                float d2;
                if (kZ) {
                    const float dz = (p[s].z - a[r].z) * a[r].w;
                    d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                } else {
                    d2 = fmaf(dx, dx, dy * dy);
                }
                hits[s][r] = d2 < b[r].x ? 1.0f : hits[s][r];
                if (d2 < b[r].y) {
                    const float gap = b[r].z - __builtin_amdgcn_sqrtf(d2);
                    pen[s] = fmaf(gap, gap, pen[s]);
                }
            }
            const int sr = next();
            a[r] = o[2 * sr];
            b[r] = o[2 * sr + 1];
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The box of the wave's positions over the C steps of a chunk (each lane holds its
// sample's positions p[0..C)), uniform: the ranges of wave_box over all of them; with
// kZ false (vertical cylinders only) the z range is left infinite.
template <int C, bool kZ>
__device__ __forceinline__ WaveBox wave_box_steps(const float4 (&p)[C])
{
    constexpr int D = kZ ? 3 : 2;
    int lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = order_key(INFINITY) + 1;
        hi[d] = order_key(-INFINITY) - 1;
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
        key_range_of(p[s].x, lo[0], hi[0]);
        key_range_of(p[s].y, lo[1], hi[1]);
        if (kZ) key_range_of(p[s].z, lo[D - 1], hi[D - 1]);
    }
    key_ranges_merge<D, 64>(lo, hi);
    return WaveBox{from_order_key(lo[0]), from_order_key(hi[0]), from_order_key(lo[1]),
                   from_order_key(hi[1]), kZ ? from_order_key(lo[D - 1]) : -INFINITY,
                   kZ ? from_order_key(hi[D - 1]) : INFINITY};
}

// The obstacle term from the slots' hit flags and this lane's penalty share.
template <int L, int S>
__device__ __forceinline__ float near_total(const CostParams& C, const float (&hits)[S], float pen)
{
    float hit = hits[0];
#pragma unroll
    for (int r = 1; r < S; ++r) hit = hits[r] > 0.0f ? 1.0f : hit;
    if (L > 1) {
        pen = group_sum<L>(pen);
        hit = group_sum<L>(hit);
    }
    return fmaf(C.w_obs, pen, hit > 0.0f ? C.c_col : 0.0f);
}

// Obstacle term of Eq. (22) for this lane's position among the obstacles [i0, i1) near
// the wave's box bx.
template <int L, int U>
__device__ __forceinline__ float obstacle_tests_near(const CostParams& C, float px, float py, float pz,
                                                     const float4* __restrict__ blk, int i0, int i1,
                                                     int M, int q, float R, const WaveBox& bx,
                                                     int& tested)
{
    constexpr int S = U < 2 ? 2 : U;
    const float4* o = blk + kObsHeaderFloat4;
    const NearLimits lim = near_limits(bx, R);
    float hits[S], pen = 0.0f;
#pragma unroll
    for (int r = 0; r < S; ++r) hits[r] = 0.0f;
    for (int base = i0; base < i1; base += 64) {          // uniform
        const int i = base + __lane_id();
        const NearBlock nb = near_block<L>(o[2 * (i < i1 ? i : M)], base, i1, M, lim);
        tested += nb.cnt;                  // obstacles each sample of this wave tests
        near_tests<L, U>(o, nb, M, q, px, py, pz, hits, pen);
    }
    return near_total<L, S>(C, hits, pen);
}

// Obstacle term of Eq. (22) for this lane's position (h: the block's header).  Short
// lists (M < kCullMin) are tested whole; longer ones through the wave's box of
// positions: the x-sorted window of the box's x-range when the block is sorted, else the
// whole list, and within it the obstacles near the box (obstacle_tests_near).
template <int L, int U>
__device__ __forceinline__ float obstacle_cost(const CostParams& C, const float4 h, float px, float py,
                                               float pz, const float4* __restrict__ blk, int M, int q,
                                               int& tested)
{
    if (M < kCullMin) return obstacle_tests<L, U>(C, px, py, pz, blk, 0, M, q, tested);
    const WaveBox bx = wave_box(px, py, pz);
    int i0 = 0, i1 = M;
    if (h.w != 0.0f) {
        int v0, v1;
        obstacle_bins_of(h, blk, bx.xlo, bx.xhi, v0, v1);
        i0 = __builtin_amdgcn_readfirstlane(v0);
        i1 = __builtin_amdgcn_readfirstlane(v1);
    }
    return obstacle_tests_near<L, U>(C, px, py, pz, blk, i0, i1, M, q, h.z, bx, tested);
}

// Kahan-compensated accumulation of the rollout cost.
struct KahanSum {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
};

}  // namespace mppi
