// Device-side bodies of the MPPI stages, shared by the one-instance kernels
// (kernels.hip) and the batched persistent kernels (batch.hip), so that an instance
// computes bit-identical results alone and inside a batch.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "../../include/mppi.h"
#include "model.h"

namespace mppi {

// ---------------------------------------------------------------------------
// Rollouts and costs (Eqs. (2), (3), (16)-(22))
// ---------------------------------------------------------------------------

// Stage the obstacle list into the workgroup's LDS block (layout at obstacle_cost),
// centred on x_hat's position: the rollouts integrate positions relative to p_hat,
// which keeps binary32 rounding at the scale of the excursion rather than of the
// world frame.  For kCullMin <= M <= kCullMax the obstacles are placed in order of x
// (rank sort: each obstacle's rank is the number of obstacles before it in (x, index)
// order; short lists rank within one wave, lane j holding key j, long lists read the
// keys from LDS) and indexed by kObsBins bins; otherwise they keep their order and
// culling is off.  Contains barriers: every thread of the workgroup calls it; the caller
// synchronises again before reading the block.  The work is spread over thread indices
// shifted by tshift (mod the workgroup size), and every thread calls hook() once after
// the first barrier: a caller can keep one wave free of staging work and give it
// other work there.
static_assert(kCullKeysInLds <= 64, "short obstacle lists are ranked within one wave");

struct NoStageHook {
    __device__ void operator()() const {}
};

template <typename Hook = NoStageHook>
__device__ __forceinline__ void stage_obstacles(float4* blk, const mppi_obstacle* __restrict__ obs,
                                                int M, float phx, float phy, float phz, float margin,
                                                int tshift = 0, const Hook& hook = Hook())
{
    __shared__ unsigned int s_rmax, s_sph;
    const int t = (int)((threadIdx.x + (unsigned)tshift) % blockDim.x);
    float4* o_lds = blk + kObsHeaderFloat4;
    int* bins = reinterpret_cast<int*>(blk + 1);
    const bool cull = M >= kCullMin && M <= kCullMax;
    auto place = [&](const mppi_obstacle& o, int rank) {
        const float R = o.r + margin;
        o_lds[2 * rank] = make_float4(o.c[0] - phx, o.c[1] - phy, o.c[2] - phz,
                                      o.type == MPPI_VCYLINDER ? 0.0f : 1.0f);
        o_lds[2 * rank + 1] = make_float4(o.r * o.r, R * R, R, 0.0f);
        if (o.type != MPPI_VCYLINDER) s_sph = 1u;
    };
    auto put = [&](int i, int rank) {
        const mppi_obstacle o = obs[i];
        place(o, rank);
        atomicMax(&s_rmax, __float_as_uint(fmaxf(o.r + margin, 0.0f)));
    };
    if (t == 0) { s_rmax = 0u; s_sph = 0u; }
    if (cull && M >= kCullKeysInLds) {
        // long lists: the sort keys (x relative to p_hat) go to LDS first, where the
        // obstacles land afterwards, padded to whole float4 with +inf, and each rank
        // reads them four at a time (a global load per obstacle costs more)
        // Each thread loads its obstacles i = t + n blockDim once, keeps them in registers
        // for the placement, and writes their keys.
        float* keys = reinterpret_cast<float*>(o_lds);
        const int M4 = (M + 3) >> 2;
        mppi_obstacle mine[kCullMax / 64];
#pragma unroll
        for (int n = 0; n < kCullMax / 64; ++n) {
            const int i = t + n * blockDim.x;
            if (i < M) {
                mine[n] = obs[i];
                keys[i] = mine[n].c[0] - phx;
            }
        }
        for (int j = M + t; j < 4 * M4; j += blockDim.x) keys[j] = INFINITY;
        __syncthreads();
        hook();
        int ranks[kCullMax / 64];                       // blockDim >= 64
#pragma unroll
        for (int n = 0; n < kCullMax / 64; ++n) {
            const int i = t + n * blockDim.x;
            ranks[n] = 0;
            if (i < M) {
                const float key = keys[i];
                const float4* k4 = reinterpret_cast<const float4*>(keys);
                for (int m = 0; m < M4; ++m) {
                    const float4 kv = k4[m];
                    const int jj = 4 * m;
                    ranks[n] += (kv.x < key || (kv.x == key && jj < i)) ? 1 : 0;
                    ranks[n] += (kv.y < key || (kv.y == key && jj + 1 < i)) ? 1 : 0;
                    ranks[n] += (kv.z < key || (kv.z == key && jj + 2 < i)) ? 1 : 0;
                    ranks[n] += (kv.w < key || (kv.w == key && jj + 3 < i)) ? 1 : 0;
                }
            }
        }
        __syncthreads();                                // keys read; the obstacles land
        float rmax = 0.0f;
#pragma unroll
        for (int n = 0; n < kCullMax / 64; ++n) {
            const int i = t + n * blockDim.x;
            if (i < M) {
                place(mine[n], ranks[n]);
                rmax = fmaxf(rmax, fmaxf(mine[n].r + margin, 0.0f));
            }
        }
        float lo, hi;                                   // one atomic per wave
        wave_range(rmax, lo, hi);
        if ((threadIdx.x & 63) == 0) atomicMax(&s_rmax, __float_as_uint(hi));
    } else if (cull) {                                  // short lists (M < 64): one wave
        __syncthreads();                                // s_rmax set
        hook();
        if (t < 64) {                                   // the whole wave of t in [0, 64)
            const mppi_obstacle o = obs[t < M ? t : 0];  // one load per lane, kept
            const float key = t < M ? o.c[0] - phx : INFINITY;
            int rank = 0;
            for (int j = 0; j < M; ++j) {               // key j broadcast from lane j
                const float kj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(key), j));
                rank += (kj < key || (kj == key && j < t)) ? 1 : 0;
            }
            if (t < M) place(o, rank);
            float lo, hi;                               // R_max over the wave, no atomics
            wave_range(t < M ? fmaxf(o.r + margin, 0.0f) : 0.0f, lo, hi);
            if (t == 0) s_rmax = __float_as_uint(hi);
        }
    } else {                                            // order kept, culling off
        __syncthreads();                                // s_rmax set
        hook();
        for (int i = t; i < M; i += blockDim.x) put(i, i);
    }
    for (int i = t; i < kObsPad; i += blockDim.x) {
        const int m = (M > 0 ? M : 0) + i;
        o_lds[2 * m] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        o_lds[2 * m + 1] = make_float4(-INFINITY, -INFINITY, 0.0f, 0.0f);
    }
    __syncthreads();
    float x0 = 0.0f, w = 1.0f;
    if (cull) {
        x0 = o_lds[0].x;
        w = fmaxf((o_lds[2 * (M - 1)].x - x0) * (1.0f / kObsBins), 1.0e-3f);
        for (int bb = t; bb <= kObsBins; bb += blockDim.x) {
            int idx = M;
            if (bb < kObsBins) {                     // first obstacle with x >= x0 + bb w
                const float edge = x0 + (float)bb * w;
                int lo = 0, hi = M;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (o_lds[2 * mid].x < edge) lo = mid + 1; else hi = mid;
                }
                idx = lo;
            }
            bins[bb] = idx;
        }
    }
    if (t == 0) {
        blk[0] = make_float4(x0, 1.0f / w, __uint_as_float(s_rmax) + kCullSlack, cull ? 1.0f : 0.0f);
        bins[kObsSphereSlot] = (int)s_sph;
    }
}

// Running cost of a state against reference row ref (Eqs. (17), (18), (22)); the row's
// loads are issued before the obstacle tests and used after them.
template <int L, int U>
__device__ __forceinline__ float state_cost(const CostParams& C, const State& x,
                                            const float* __restrict__ ref, float phx, float phy,
                                            float phz, const float4 oh,
                                            const float4* __restrict__ obs_lds, int M, int q,
                                            int& tested)
{
    float r[13];
#pragma unroll
    for (int e = 0; e < 13; ++e) r[e] = ref[e];
    const float co = obstacle_cost<L, U>(C, oh, x.px, x.py, x.pz, obs_lds, M, q, tested);
    return tracking_cost(C, x, r[0] - phx, r[1] - phy, r[2] - phz, r) + co;
}

// Steps whose obstacle terms the one-wave rollouts take together.
constexpr int kRolloutChunk = 4;

// The obstacle terms (Eq. (22)) of C states of this lane's sample, p[s] its positions
// (nv of them valid, the rest copies of the first): the wave's box of all of them, the
// x-window of that box (a sorted block) or the whole list, and among it the obstacles
// near the box, each loaded once and tested at every position (near_tests_chunk; a
// block of vertical cylinders only skips the z terms).  With one lane per sample every
// state's penalty and hit equal those of obstacle_cost, which culls by one state's box:
// the extra candidates lie beyond every reach of the state, and the sum runs in the
// same index order.
template <int L, int U, int C>
__device__ __forceinline__ void obstacle_costs_chunk(const CostParams& Cp, const float4 h,
                                                     const float4* __restrict__ blk, int M, int q,
                                                     const float4 (&p)[C], int nv, float (&co)[C],
                                                     int& tested)
{
    constexpr int R = U < 2 ? 2 : U;
    const int* bins = reinterpret_cast<const int*>(blk + 1);
    const bool zfree = __builtin_amdgcn_readfirstlane(bins[kObsSphereSlot]) == 0;
    const WaveBox bx = zfree ? wave_box_steps<C, false>(p) : wave_box_steps<C, true>(p);
    int i0 = 0, i1 = M;
    if (h.w != 0.0f) {
        int v0, v1;
        obstacle_bins_of(h, blk, bx.xlo, bx.xhi, v0, v1);
        i0 = __builtin_amdgcn_readfirstlane(v0);
        i1 = __builtin_amdgcn_readfirstlane(v1);
    }
    const float4* o = blk + kObsHeaderFloat4;
    const NearLimits lim = near_limits(bx, h.z);
    float hits[C][R], pen[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
        pen[s] = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) hits[s][r] = 0.0f;
    }
    for (int base = i0; base < i1; base += 64) {              // uniform
        const int i = base + __lane_id();
        const NearBlock nb = near_block<L>(o[2 * (i < i1 ? i : M)], base, i1, M, lim);
        tested += nv * nb.cnt;
        if (zfree) near_tests_chunk<L, U, false, C>(o, nb, M, q, p, hits, pen);
        else near_tests_chunk<L, U, true, C>(o, nb, M, q, p, hits, pen);
    }
#pragma unroll
    for (int s = 0; s < C; ++s) co[s] = near_total<L, R>(Cp, hits[s], pen[s]);
}

// Rollout of sample k by lane q of its L lanes.  The L lanes integrate the same
// sample (identical instructions and operands, hence identical trajectories) and
// divide its obstacle tests; lane q = 0 of a valid sample writes delta_u [N][4][ld]
// (unless kStoreDu is false), S [K] and the optional trajectory dump [N+1][17][ld]
// (world-frame positions).  Lanes past the last sample run a copy of sample K-1
// without writing, so that every lane of the wave takes part in the wave-wide
// obstacle culling.  Returns the sample's cost (on all L lanes).
template <int L, int U, bool kLag, bool kDump, bool kStoreDu = true>
__device__ __forceinline__ float rollout_sample(const RolloutParams& a, const float* __restrict__ x_hat,
                                               const float* __restrict__ x_ref,
                                               const float* __restrict__ u_nom,
                                               float* __restrict__ du_out, float* __restrict__ S_out,
                                               float* __restrict__ states,
                                               const float4* __restrict__ obs_lds, int k, int q)
{
    const bool writer = (q == 0) && k < a.K;
    if (k >= a.K) k = a.K - 1;
    const size_t ld = (size_t)a.ld;
    const float phx = x_hat[0], phy = x_hat[1], phz = x_hat[2];

    State x;
    x.px = 0.0f; x.py = 0.0f; x.pz = 0.0f;
    x.qw = x_hat[3]; x.qx = x_hat[4]; x.qy = x_hat[5]; x.qz = x_hat[6];
    x.vx = x_hat[7]; x.vy = x_hat[8]; x.vz = x_hat[9];
    x.wx = x_hat[10]; x.wy = x_hat[11]; x.wz = x_hat[12];
    x.T0 = x_hat[13]; x.T1 = x_hat[14]; x.T2 = x_hat[15]; x.T3 = x_hat[16];

    if (kDump && writer) {
        const float vals[17] = {x.px + phx, x.py + phy, x.pz + phz, x.qw, x.qx, x.qy, x.qz,
                                x.vx, x.vy, x.vz, x.wx, x.wy, x.wz, x.T0, x.T1, x.T2, x.T3};
#pragma unroll
        for (int i = 0; i < 17; ++i) states[(size_t)i * ld + k] = vals[i];
    }

    KahanSum S;
    int tested = 0;
    const float4 oh = obs_lds[0];          // obstacle block header
    // state j = 0 (the estimate itself) is scored like every other state (Eq. (17))
    S.add(state_cost<L, U>(a.cp, x, x_ref, phx, phy, phz, oh, obs_lds, a.M, q, tested));

    float up[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // With L lanes per sample the noise is drawn round-robin: at steps j = 0, L, 2L, ...
    // lane q draws step j + q, and each step's noise is read from its lane of the
    // group -- one draw per L steps in the wave's instruction stream instead of one per
    // step (the values are the same).
    float nz[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const int grp = (__lane_id() & ~(L - 1)) << 2;        // byte address of lane 0 of the group
    // Step j: the perturbed control, its input costs (returned) and the model step.
    auto step = [&](int j) {
        float du[4], u[4];
        if (L == 1) {
            draw_noise(a.np, (uint32_t)k, (uint32_t)j, du);
        } else {
            if (j % L == 0 && j + q < a.N) draw_noise(a.np, (uint32_t)k, (uint32_t)(j + q), nz);
            const int src = grp | ((j % L) << 2);
#pragma unroll
            for (int d = 0; d < 4; ++d)
                du[d] = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(nz[d])));
        }
        if (kStoreDu && writer) {
            float* dst = du_out + (size_t)(4 * j) * ld + k;
#pragma unroll
            for (int d = 0; d < 4; ++d) dst[(size_t)d * ld] = du[d];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) u[d] = u_nom[4 * j + d] + du[d];   // Eq. (2): u = u_nom + du
        // input and input-change terms of Eq. (16)
        float cu = 0.0f;
#pragma unroll
        for (int d = 0; d < 4; ++d) cu = fmaf(a.cp.R[d] * u[d], u[d], cu);
        if (j > 0) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const float e = u[d] - up[d];
                cu = fmaf(a.cp.Rd[d] * e, e, cu);
            }
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) up[d] = u[d];

        float Tc[4];
        rate_controller(a.mp, x.wx, x.wy, x.wz, u, Tc);
        rk4_step<kLag>(a.mp, x, Tc);
        return cu;
    };
    auto dump = [&](int j) {
        if (kDump && writer) {
            const float vals[17] = {x.px + phx, x.py + phy, x.pz + phz, x.qw, x.qx, x.qy, x.qz,
                                    x.vx, x.vy, x.vz, x.wx, x.wy, x.wz, x.T0, x.T1, x.T2, x.T3};
            float* st = states + (size_t)17 * (j + 1) * ld + k;
#pragma unroll
            for (int i = 0; i < 17; ++i) st[(size_t)i * ld] = vals[i];
        }
    };
    if (a.M >= kCullMin) {
        // Culled lists: the obstacle terms of kRolloutChunk steps at a time, by the box
        // of the wave's positions over those steps (obstacle_costs_chunk); the running
        // cost is added step by step as below, cu + (tracking + obstacle).
        for (int j0 = 0; j0 < a.N; j0 += kRolloutChunk) {
            const int nv = a.N - j0 < kRolloutChunk ? a.N - j0 : kRolloutChunk;   // uniform
            float4 pc[kRolloutChunk];      // position and tracking cost of each state
            float cus[kRolloutChunk];
#pragma unroll
            for (int s = 0; s < kRolloutChunk; ++s) {
                if (s < nv) {
                    const int j = j0 + s;
                    cus[s] = step(j);
                    const float* rf = x_ref + (size_t)13 * (j + 1);
                    const float tr = tracking_cost(a.cp, x, rf[0] - phx, rf[1] - phy, rf[2] - phz, rf);
                    pc[s] = make_float4(x.px, x.py, x.pz, tr);
                    dump(j);
                } else {
                    pc[s] = pc[0];         // past the horizon: a copy of the first (unused)
                    cus[s] = 0.0f;
                }
            }
            float co[kRolloutChunk];
            obstacle_costs_chunk<L, U>(a.cp, oh, obs_lds, a.M, q, pc, nv, co, tested);
#pragma unroll
            for (int s = 0; s < kRolloutChunk; ++s)
                if (s < nv) S.add(cus[s] + (pc[s].w + co[s]));
        }
    } else {
        for (int j = 0; j < a.N; ++j) {
            const float cu = step(j);
            const float cx = state_cost<L, U>(a.cp, x, x_ref + (size_t)13 * (j + 1), phx, phy, phz,
                                              oh, obs_lds, a.M, q, tested);
            S.add(cu + cx);
            dump(j);
        }
    }
    if (writer) S_out[k] = S.s;
    if (a.obs_tests) {                     // one atomic per wave: valid samples x tests
        const unsigned long long samples = __popcll(__ballot(writer));
        if (__lane_id() == 0) atomicAdd(a.obs_tests, samples * (unsigned long long)tested);
    }
    return S.s;
}

// ---------------------------------------------------------------------------
// Wave-specialised rollouts: one workgroup per 64 samples, 4 + L waves.  The chains
// of a step depend on one another in one direction only: the body rates and rotor
// thrusts (rk4_rates) on u alone, the attitude (rk4_attitude) on the stage rates and
// thrusts, p and v (rk4_translational) on the stage accelerations, and the obstacle
// term on p.  So the step is split across waves that run on different SIMDs: wave 0
// draws the noise and forms u and the input costs, wave 1 runs the controller and the
// rates, wave 2 the attitude and the stage accelerations, wave 3 integrates p and v
// and scores the tracking cost, and waves 4 .. 4 + L - 1 score the obstacles and sum
// the running cost (L lanes per sample dividing the obstacle tests, as in
// rollout_sample).  The roles hand over chunks of C steps (kPipeChunk, or 2 for
// horizons up to kPipeShortN steps: a shorter fill) through
// double-buffered LDS, one workgroup barrier per chunk, each role one chunk behind the
// previous.  The arithmetic is rollout_sample's, operation for operation (the values
// handed between chains pass through opaque() in both).
// ---------------------------------------------------------------------------

constexpr int kPipeChunk = 4;        // steps per chunk (2 for short horizons)
constexpr int kPipeShortN = 24;      // horizons up to this many steps use chunks of 2

template <int C>
struct PipeLdsT {
    float4 u[2][C][64];         // u_j per sample
    float cu[2][C][64];         // input and input-change cost of step j
    float4 w[2][C][5][64];      // stage rates x, y, z, stage thrust F, (omega, cost)
    float4 r[2][C][5][64];      // stage accelerations x, y, z, q, (omega, cost)
    float4 p[2][C][64];         // p_{j+1} relative to p_hat, tracking cost
    int2 win[2][C][8];          // culling window of p_{j+1} per obstacle wave
    float cu_fwd[2][C][64];     // input cost, forwarded to the obstacle role
    float4 xr[4][C][4];         // reference rows j + 1 of chunk c in slot c % 4 (13 floats)
};

template <int C = kPipeChunk>
__host__ __device__ constexpr size_t pipe_lds_bytes(int M)
{
    return obstacle_lds_bytes(M) + sizeof(PipeLdsT<C>);
}

// Noise role: chunk c of sample k (kk: k clamped to K - 1).  It also copies the chunk's
// reference rows j + 1 into the ring P.xr, one float per lane, for the translation role
// three phases later: those reads then wait for LDS alone, not for scalar loads from
// global memory (which return out of order and so make every wait a full one).
template <bool kStoreDu, int C>
__device__ __forceinline__ void pipe_noise_chunk(const RolloutParams& a, const float* __restrict__ u_nom,
                                                 const float* __restrict__ x_ref,
                                                 float* __restrict__ du_out, bool writer, int kk,
                                                 int c, float (&up)[4], PipeLdsT<C>& P, int lane)
{
    const size_t ld = (size_t)a.ld;
    const int rs = lane >> 4, re = lane & 15;         // step and element of the ring entry
    float xr = 0.0f;
    if (rs < C && re < 13) {
        const int row = c * C + rs + 1 < a.N ? c * C + rs + 1 : a.N;
        xr = x_ref[(size_t)13 * row + re];
    }
    float un[C][4];                                   // the chunk's u_nom rows, loaded
#pragma unroll                                                 // together (the last clamped)
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s < a.N ? c * C + s : a.N - 1;
#pragma unroll
        for (int d = 0; d < 4; ++d) un[s][d] = u_nom[4 * j + d];
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s;
        if (j >= a.N) break;                                   // uniform
        float du[4], u[4];
        draw_noise(a.np, (uint32_t)kk, (uint32_t)j, du);
        if (kStoreDu && writer) {
            float* dst = du_out + (size_t)(4 * j) * ld + kk;
#pragma unroll
            for (int d = 0; d < 4; ++d) dst[(size_t)d * ld] = du[d];
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) u[d] = un[s][d] + du[d];
        float cu = 0.0f;
#pragma unroll
        for (int d = 0; d < 4; ++d) cu = fmaf(a.cp.R[d] * u[d], u[d], cu);
        if (j > 0) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const float e = u[d] - up[d];
                cu = fmaf(a.cp.Rd[d] * e, e, cu);
            }
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) up[d] = u[d];
        P.u[c & 1][s][lane] = make_float4(u[0], u[1], u[2], u[3]);
        P.cu[c & 1][s][lane] = cu;
    }
    if (rs < C) reinterpret_cast<float*>(P.xr[c & 3][rs])[re] = xr;
}

// Rates role: chunk c (x holds omega and the rotor thrusts): the controller, then
// the body rates and thrusts at the stage points.
template <bool kLag, int C>
__device__ __forceinline__ void pipe_rates_chunk(const RolloutParams& a, State& x, int c, PipeLdsT<C>& P,
                                                 int lane)
{
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s;
        if (j >= a.N) break;
        const float4 uv = P.u[c & 1][s][lane];
        const float u[4] = {uv.x, uv.y, uv.z, uv.w};
        float Tc[4];
        rate_controller(a.mp, x.wx, x.wy, x.wz, u, Tc);
        RateStages R;
        rk4_rates<kLag>(a.mp, x, Tc, R);
        P.w[c & 1][s][0][lane] = make_float4(R.wx[0], R.wx[1], R.wx[2], R.wx[3]);
        P.w[c & 1][s][1][lane] = make_float4(R.wy[0], R.wy[1], R.wy[2], R.wy[3]);
        P.w[c & 1][s][2][lane] = make_float4(R.wz[0], R.wz[1], R.wz[2], R.wz[3]);
        P.w[c & 1][s][3][lane] = make_float4(R.F[0], R.F[1], R.F[2], R.F[3]);
        P.w[c & 1][s][4][lane] = make_float4(x.wx, x.wy, x.wz, P.cu[c & 1][s][lane]);
    }
}

// Attitude role: chunk c (x holds q): q over the step from the stage rates and
// thrusts, and the stage accelerations.
template <int C>
__device__ __forceinline__ void pipe_attitude_chunk(const RolloutParams& a, State& x, int c, PipeLdsT<C>& P,
                                                    int lane)
{
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s;
        if (j >= a.N) break;
        const float4 wx = P.w[c & 1][s][0][lane], wy = P.w[c & 1][s][1][lane];
        const float4 wz = P.w[c & 1][s][2][lane], F = P.w[c & 1][s][3][lane];
        const RateStages R{{wx.x, wx.y, wx.z, wx.w}, {wy.x, wy.y, wy.z, wy.w},
                           {wz.x, wz.y, wz.z, wz.w}, {F.x, F.y, F.z, F.w}};
        StageAccel A;
        rk4_attitude(a.mp, x, R, A);
        P.r[c & 1][s][0][lane] = make_float4(A.x[0], A.x[1], A.x[2], A.x[3]);
        P.r[c & 1][s][1][lane] = make_float4(A.y[0], A.y[1], A.y[2], A.y[3]);
        P.r[c & 1][s][2][lane] = make_float4(A.z[0], A.z[1], A.z[2], A.z[3]);
        P.r[c & 1][s][3][lane] = make_float4(x.qw, x.qx, x.qy, x.qz);
        P.r[c & 1][s][4][lane] = P.w[c & 1][s][4][lane];
    }
}

// Translation role: chunk c of sample `lane` (x holds p relative to p_hat, and v):
// integrates p and v with the hand-over of the attitude role, scores the tracking cost
// and takes the culling window of each obstacle wave's 64 / L samples (lanes of one
// group of 64 / L here): the window that wave would take itself; hands p, that cost,
// the input cost and the windows on to the obstacle role.
template <int L, int C>
__device__ __forceinline__ void pipe_translation_chunk(const RolloutParams& a, const float4 oh,
                                                       const float4* __restrict__ obs_lds,
                                                       float phx, float phy, float phz, State& x,
                                                       int c, int lane, PipeLdsT<C>& P, bool win)
{
    float4 h[5], g[4];                     // step s's hand-over and reference row, loaded
#pragma unroll                             // during step s - 1
    for (int e = 0; e < 5; ++e) h[e] = P.r[c & 1][0][e][lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) g[e] = P.xr[c & 3][0][e];
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s;
        if (j >= a.N) break;
        const float4 ax = h[0], ay = h[1], az = h[2], qv = h[3], wv = h[4];
        const float rf[13] = {g[0].x, g[0].y, g[0].z, g[0].w, g[1].x, g[1].y, g[1].z,
                              g[1].w, g[2].x, g[2].y, g[2].z, g[2].w, g[3].x};
        if (s + 1 < C) {
#pragma unroll
            for (int e = 0; e < 5; ++e) h[e] = P.r[c & 1][s + 1][e][lane];
#pragma unroll
            for (int e = 0; e < 4; ++e) g[e] = P.xr[c & 3][s + 1][e];
        }
        const StageAccel A{{ax.x, ax.y, ax.z, ax.w}, {ay.x, ay.y, ay.z, ay.w}, {az.x, az.y, az.z, az.w}};
        rk4_translational(a.mp, x, A);
        x.qw = qv.x; x.qx = qv.y; x.qy = qv.z; x.qz = qv.w;
        x.wx = wv.x; x.wy = wv.y; x.wz = wv.z;
        constexpr int G = 64 / L;
        int v0 = 0, v1 = a.M;              // bin reads in flight during the tracking cost
        if (win && oh.w != 0.0f) {         // (uniform; no window when the obstacle role culls)
            float lo, hi;
            group_range<G>(x.px, lo, hi);
            obstacle_bins_of(oh, obs_lds, lo, hi, v0, v1);
        }
        const float tr = tracking_cost(a.cp, x, rf[0] - phx, rf[1] - phy, rf[2] - phz, rf);
        P.p[c & 1][s][lane] = make_float4(x.px, x.py, x.pz, tr);
        P.cu_fwd[c & 1][s][lane] = wv.w;
        if (lane % G == 0) P.win[c & 1][s][lane / G] = make_int2(v0, v1);
    }
}

// Obstacle role (obstacle wave ow): chunk c for the sample at position sb of the
// workgroup, lane q of its L lanes: the obstacle term at the handed-over position, and
// the running cost in the order of rollout_sample, cu + (tracking + obstacle).
template <int L, int U, bool kZ, int C>
__device__ __forceinline__ void pipe_obstacle_chunk(const RolloutParams& a,
                                                    const float4* __restrict__ obs_lds,
                                                    KahanSum& S, int& tested, int c, int sb, int q,
                                                    int ow, const PipeLdsT<C>& P)
{
    // the chunk's hand-over read together (one wait for all of it; obstacle_tests waits
    // for every outstanding LDS read before its own)
    float4 pts[C];
    float cus[C];
    int2 wins[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
        pts[s] = P.p[c & 1][s][sb];
        cus[s] = P.cu_fwd[c & 1][s][sb];
        wins[s] = P.win[c & 1][s][ow];
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
        const int j = c * C + s;
        if (j >= a.N) break;
        const float co = obstacle_tests<L, U, kZ>(a.cp, pts[s].x, pts[s].y, pts[s].z, obs_lds,
                                              __builtin_amdgcn_readfirstlane(wins[s].x),
                                              __builtin_amdgcn_readfirstlane(wins[s].y), q, tested);
        S.add(cus[s] + (pts[s].w + co));
    }
}

// Obstacle role with chunk culling (4 or 8 lanes per sample, at least kCullMin
// obstacles): the wave takes the box of its samples' positions over the chunk's steps
// and tests only the obstacles of that box's x-window near the box (the exact culling of
// obstacle_tests_near), at all the chunk's positions at once, each candidate's operands
// loaded once; then adds each step's running cost as pipe_obstacle_chunk does.
template <int L, int U, bool kZ, int C>
__device__ __forceinline__ void pipe_obstacle_chunk_box(const RolloutParams& a, const float4 oh,
                                                        const float4* __restrict__ obs_lds,
                                                        KahanSum& S, int& tested, int c, int sb,
                                                        int q, const PipeLdsT<C>& P)
{
    constexpr int R = U < 2 ? 2 : U;
    const int nv = a.N - c * C < C ? a.N - c * C : C;       // the chunk's steps (>= 1)
    float4 pts[C];
    float cus[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
        const int ss = s < nv ? s : 0;     // past the horizon: a copy of step 0 (unused)
        pts[s] = P.p[c & 1][ss][sb];
        cus[s] = P.cu_fwd[c & 1][ss][sb];
    }
    const WaveBox bx = wave_box_steps<C, kZ>(pts);
    int i0 = 0, i1 = a.M;
    if (oh.w != 0.0f) {
        int v0, v1;
        obstacle_bins_of(oh, obs_lds, bx.xlo, bx.xhi, v0, v1);
        i0 = __builtin_amdgcn_readfirstlane(v0);
        i1 = __builtin_amdgcn_readfirstlane(v1);
    }
    const float4* o = obs_lds + kObsHeaderFloat4;
    const NearLimits lim = near_limits(bx, oh.z);
    float hits[C][R], pen[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
        pen[s] = 0.0f;
#pragma unroll
        for (int r = 0; r < R; ++r) hits[s][r] = 0.0f;
    }
    for (int base = i0; base < i1; base += 64) {              // uniform
        const int i = base + __lane_id();
        const NearBlock nb = near_block<L>(o[2 * (i < i1 ? i : a.M)], base, i1, a.M, lim);
        tested += nv * nb.cnt;
        near_tests_chunk<L, U, kZ, C>(o, nb, a.M, q, pts, hits, pen);
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
        if (s >= nv) break;
        const float co = near_total<L, R>(a.cp, hits[s], pen[s]);
        S.add(cus[s] + (pts[s].w + co));
    }
}

// ---------------------------------------------------------------------------
// Block reductions (wave64 shuffles, then LDS across waves)
// ---------------------------------------------------------------------------

// Lexicographic (value, index) minimum; NaN never wins.
__device__ __forceinline__ void argmin_merge(float& v, int& i, float v2, int i2)
{
    if (v2 < v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// Error-free sum of two compensated pairs (Knuth two-sum).
__device__ __forceinline__ void twosum_merge(float& s, float& c, float s2, float c2)
{
    const float t = s + s2;
    const float bp = t - s;
    const float e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = c + c2 + e;
}

// Deterministic reductions over the 64 lanes of a wave (all lanes active), read from
// lane 63: a butterfly within each row of 16 lanes by DPP moves (quad permutations xor
// 1 and xor 2, half-row mirror, row mirror), then the row broadcasts 15 and 31 fold the
// rows into lane 63.  Lanes a step does not write receive the operation's identity.
// No LDS traffic: each step is one VALU move.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i(int x, int identity)
{
    return __builtin_amdgcn_update_dpp(identity, x, kCtrl, kRowMask, 0xF, false);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_f(float x, float identity)
{
    return __int_as_float(dpp_i<kCtrl, kRowMask>(__float_as_int(x), __float_as_int(identity)));
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_d(double x)      // identity 0.0
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<kCtrl, kRowMask>((int)(unsigned)(b & 0xffffffffll), 0);
    const int hi = dpp_i<kCtrl, kRowMask>((int)(b >> 32), 0);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane63(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ __forceinline__ double lane63(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

#define MPPI_WAVE_STEPS(STEP) STEP(0xB1, 0xF) STEP(0x4E, 0xF) STEP(0x141, 0xF) STEP(0x140, 0xF) \
                              STEP(0x142, 0xA) STEP(0x143, 0xC)

__device__ __forceinline__ float wave_sum(float v)
{
#define MPPI_STEP(C, R) v += dpp_f<C, R>(v, 0.0f);
    MPPI_WAVE_STEPS(MPPI_STEP)
#undef MPPI_STEP
    return lane63(v);
}

__device__ __forceinline__ double wave_sum(double v)
{
#define MPPI_STEP(C, R) v += dpp_d<C, R>(v);
    MPPI_WAVE_STEPS(MPPI_STEP)
#undef MPPI_STEP
    return lane63(v);
}

// (value, index) minimum with argmin_merge and the sum of n over the wave.
__device__ __forceinline__ void wave_argmin_count(float& v, int& i, int& n)
{
#define MPPI_STEP(C, R)                                                          \
    {                                                                            \
        const float v2 = dpp_f<C, R>(v, INFINITY);                               \
        const int i2 = dpp_i<C, R>(i, INT_MAX);                                  \
        argmin_merge(v, i, v2, i2);                                              \
        n += dpp_i<C, R>(n, 0);                                                  \
    }
    MPPI_WAVE_STEPS(MPPI_STEP)
#undef MPPI_STEP
    v = lane63(v); i = lane63(i); n = lane63(n);
}

// Compensated (two-sum) total of (s, c) pairs and the plain sum q over the wave.
__device__ __forceinline__ void wave_twosum(float& s, float& c, float& q)
{
#define MPPI_STEP(C, R)                                                          \
    {                                                                            \
        const float s2 = dpp_f<C, R>(s, 0.0f), c2 = dpp_f<C, R>(c, 0.0f);        \
        twosum_merge(s, c, s2, c2);                                              \
        q += dpp_f<C, R>(q, 0.0f);                                               \
    }
    MPPI_WAVE_STEPS(MPPI_STEP)
#undef MPPI_STEP
    s = lane63(s); c = lane63(c); q = lane63(q);
}

// ---------------------------------------------------------------------------
// G2: softmin weights
// ---------------------------------------------------------------------------

// One workgroup of kWeightsThreads threads computes the weights of one instance.
__device__ __forceinline__ void weights_block(const float* __restrict__ S, int K, float lambda,
                                              float* __restrict__ w, mppi_diag* __restrict__ diag,
                                              int lanes)
{
    __shared__ float sh_v[kWeightsThreads / 64];
    __shared__ int sh_i[kWeightsThreads / 64], sh_n[kWeightsThreads / 64];
    __shared__ float sh_s[kWeightsThreads / 64], sh_c[kWeightsThreads / 64], sh_q[kWeightsThreads / 64];
    __shared__ float bc_rho;
    __shared__ int bc_n;
    __shared__ float bc_eta;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;

    // rho = min over finite costs, its first index, and the finite count
    float mv = INFINITY;
    int mi = INT_MAX, nf = 0;
    for (int k = tid; k < K; k += blockDim.x) {
        const float s = S[k];
        if (isfinite(s)) {
            ++nf;
            if (s < mv) { mv = s; mi = k; }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_xor(mv, off);
        const int i2 = __shfl_xor(mi, off);
        argmin_merge(mv, mi, v2, i2);
        nf += __shfl_xor(nf, off);
    }
    if (lane == 0) { sh_v[wv] = mv; sh_i[wv] = mi; sh_n[wv] = nf; }
    __syncthreads();
    if (tid == 0) {
        float v = sh_v[0];
        int i = sh_i[0], n = sh_n[0];
        for (int q = 1; q < nw; ++q) { argmin_merge(v, i, sh_v[q], sh_i[q]); n += sh_n[q]; }
        bc_rho = v; bc_n = n;
        diag->rho = v; diag->argmin = n > 0 ? i : -1; diag->n_finite = n; diag->lanes = lanes;
    }
    __syncthreads();
    const float rho = bc_rho;
    if (bc_n == 0) {
        for (int k = tid; k < K; k += blockDim.x) w[k] = 0.0f;
        if (tid == 0) {
            diag->eta = 0.0f; diag->ess = 0.0f; diag->status = MPPI_E_ALL_NONFINITE;
        }
        return;
    }

    // e_k = exp(-(S_k - rho) / lambda) = 2^((rho - S_k) log2(e) / lambda); eta = sum_k e_k
    const float scale = 1.44269504089f / lambda;
    float es = 0.0f, ec = 0.0f, q2 = 0.0f;
    for (int k = tid; k < K; k += blockDim.x) {
        const float s = S[k];
        const float e = isfinite(s) ? __builtin_amdgcn_exp2f((rho - s) * scale) : 0.0f;
        w[k] = e;
        const float y = e - ec, t = es + y;          // Kahan
        ec = (t - es) - y;
        es = t;
        q2 = fmaf(e, e, q2);
    }
    ec = -ec;   // pair (es, ec) with es + ec the compensated value
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float s2 = __shfl_xor(es, off), c2 = __shfl_xor(ec, off);
        twosum_merge(es, ec, s2, c2);
        q2 += __shfl_xor(q2, off);
    }
    if (lane == 0) { sh_s[wv] = es; sh_c[wv] = ec; sh_q[wv] = q2; }
    __syncthreads();
    if (tid == 0) {
        float s = sh_s[0], c = sh_c[0], q = sh_q[0];
        for (int i = 1; i < nw; ++i) { twosum_merge(s, c, sh_s[i], sh_c[i]); q += sh_q[i]; }
        const float eta = s + c;
        bc_eta = eta;
        diag->eta = eta;
        diag->ess = eta * eta / q;
        diag->status = MPPI_OK;
    }
    __syncthreads();
    const float inv_eta = 1.0f / bc_eta;
    for (int k = tid; k < K; k += blockDim.x) w[k] *= inv_eta;
}

// ---------------------------------------------------------------------------
// G3: weighted sum of the perturbations, one workgroup per (j, d) row
// ---------------------------------------------------------------------------

// One workgroup of kSumThreads threads reduces row `row` = 4 j + d of delta_u.
__device__ __forceinline__ void weighted_sum_row(const float* __restrict__ w,
                                                 const float* __restrict__ du, int K, int ld,
                                                 const float* __restrict__ u_in,
                                                 float* __restrict__ u_out,
                                                 const mppi_diag* __restrict__ diag, int row)
{
    __shared__ float sh[kSumThreads / 64];
    const int tid = threadIdx.x;
    const float* src = du + (size_t)row * ld;
    float acc = 0.0f;
    if ((ld & 3) == 0) {
        const int K4 = K >> 2;
        const float4* s4 = reinterpret_cast<const float4*>(src);
        const float4* w4 = reinterpret_cast<const float4*>(w);
        for (int i = tid; i < K4; i += blockDim.x) {
            const float4 a = s4[i], b = w4[i];
            acc = fmaf(a.x, b.x, acc);
            acc = fmaf(a.y, b.y, acc);
            acc = fmaf(a.z, b.z, acc);
            acc = fmaf(a.w, b.w, acc);
        }
        for (int k = 4 * K4 + tid; k < K; k += blockDim.x) acc = fmaf(src[k], w[k], acc);
    } else {
        for (int k = tid; k < K; k += blockDim.x) acc = fmaf(src[k], w[k], acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        float t = 0.0f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        const bool ok = diag == nullptr || diag->status == MPPI_OK;
        u_out[row] = ok ? u_in[row] + t : u_in[row];
    }
    __syncthreads();   // sh is reused by the caller's next row
}

// ---------------------------------------------------------------------------
// G4: apply and shift
// ---------------------------------------------------------------------------

__device__ __forceinline__ void feasible_input(const ModelParams& P, const float* x, const float* u, float* out)
{
    // Eqs. (12)-(15): clipped thrusts -> [F_clip; tau_clip] -> omega_clip
    float Tc[4];
    const float uu[4] = {u[0], u[1], u[2], u[3]};
    rate_controller(P, x[10], x[11], x[12], uu, Tc);
    const float s01 = Tc[0] + Tc[1], s23 = Tc[2] + Tc[3], d10 = Tc[1] - Tc[0], d23 = Tc[2] - Tc[3];
    const float F = s01 + s23;
    const float tau[3] = {P.s * (d10 + d23), P.s * (d10 - d23), P.c * (s23 - s01)};
    const float gyr[3] = {P.G[0] * x[11] * x[12], P.G[1] * x[12] * x[10], P.G[2] * x[10] * x[11]};
    const float lim[3] = {P.w_xy_max, P.w_xy_max, P.w_z_max};
    out[0] = F;
    for (int i = 0; i < 3; ++i) {
        float wc = fmaf((tau[i] - gyr[i]) * P.J_inv[i], P.dt, x[10 + i]);
        if (lim[i] > 0.0f) wc = clampf(wc, -lim[i], lim[i]);
        out[1 + i] = wc;
    }
}

// ---------------------------------------------------------------------------
// The update in two launches.  The rollout launch ends with per-wave statistics of
// the weights (Eq. (4) relative to each wave's minimum), which its last workgroup
// reduces into the update's rho, eta and diagnostics; the second launch forms the
// weighted sum (Eq. (5)) and applies and advances the warm start.  The weighted sum
// reads either the stored delta_u (a GEMV, one workgroup per step, which also writes
// that step's knot) or, in the single pass, per-wave partial sums that the rollout
// waves formed from regenerated noise, so that delta_u never goes to memory (its last
// workgroup applies).
// ---------------------------------------------------------------------------

// Eq. (4) over one wave, relative to its own minimum.
struct WaveSums {
    float rho;      // minimum finite cost of the wave's valid samples (+inf if none)
    int argmin;     // first sample attaining it (INT_MAX if none)
    int n;          // finite costs, each sample counted once
    float es, ec;   // compensated sum of e_k = exp(-(S_k - rho) / lambda)
    float q2;       // sum of e_k^2
    float e;        // this lane's e_k (0 for an invalid lane or a non-finite cost)
};

// S: the lane's sample cost; k its sample, q its lane within the sample, valid = k < K.
// Every lane of the wave calls it and gets the wave's sums.
__device__ __forceinline__ WaveSums wave_sums(float S, int k, int q, bool valid, float lambda)
{
    WaveSums w;
    const bool fin = valid && isfinite(S);
    float mv = fin ? S : INFINITY;
    int mi = fin ? k : INT_MAX;
    int nf = (fin && q == 0) ? 1 : 0;
    wave_argmin_count(mv, mi, nf);
    w.rho = mv; w.argmin = mi; w.n = nf;
    const float scale = 1.44269504089f / lambda;
    w.e = fin ? __builtin_amdgcn_exp2f((mv - S) * scale) : 0.0f;
    float es = q == 0 ? w.e : 0.0f, ec = 0.0f, q2 = es * es;
    wave_twosum(es, ec, q2);
    w.es = es; w.ec = ec; w.q2 = q2;
    return w;
}

__device__ __forceinline__ void write_wave_stat(WaveStat* __restrict__ stat, const WaveSums& w,
                                                bool skipped)
{
    if (__lane_id() == 0) {
        WaveStat s;
        s.rho = w.rho; s.eta_s = w.es; s.eta_c = w.ec; s.q = w.q2;
        s.argmin = w.n > 0 ? w.argmin : -1; s.n = w.n; s.skipped = skipped ? 1 : 0; s.pad = 0;
        *stat = s;
    }
}

// Sum of v[0..15] over the lanes of the wave that share lane % L (the samples of the
// wave, one lane per sample for each of the L lane positions), by a butterfly that
// halves the values each lane carries at every exchange.  Afterwards a lane holds
// R = 16 >> ST sums: v[m] is the total of value (m << ST) | ((lane >> log2 L) & (2^ST - 1)),
// ST = min(4, 6 - log2 L); lanes whose bits above log2 L + ST are zero hold distinct
// totals.
template <int L>
__device__ __forceinline__ void wave_sum16(float (&v)[16], int lane)
{
    constexpr int LB = L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : 3;
    constexpr int BITS = 6 - LB;
    constexpr int ST = BITS < 4 ? BITS : 4;
#pragma unroll
    for (int s = 0; s < ST; ++s) {
        const int mask = 1 << (LB + s);
        const bool hi = (lane & mask) != 0;
#pragma unroll
        for (int m = 0; m < (16 >> (s + 1)); ++m) {
            const float keep = hi ? v[2 * m + 1] : v[2 * m];
            const float send = hi ? v[2 * m] : v[2 * m + 1];
            v[m] = keep + __shfl_xor(send, mask);
        }
    }
#pragma unroll
    for (int s = ST; s < BITS; ++s) v[0] += __shfl_xor(v[0], 1 << (LB + s));
}

// Single pass, per wave: P_w[4 j + d] = sum_k e_k delta_u_{k,j,d} (Eq. (5) before the
// normalisation) with delta_u regenerated from the counter-based noise; lane q of a
// sample regenerates the chunks of four steps c = r L + q, so the L lanes of a sample
// share the regeneration.
//
// rho_run holds the bits of the smallest wave minimum published so far (costs are sums
// of non-negative terms, so the bits order like the values).  A wave whose minimum lies
// more than kSkipLog2 / (log2(e) / lambda) above it has every weight below
// 2^-kSkipLog2 relative to the final minimum -- exactly zero in binary32, as in the
// stored form -- and skips the regeneration (stat->skipped = 1).
template <int L>
__device__ __forceinline__ void fused_wave_partials(const RolloutParams& a, float lambda,
                                                    const WaveSums& ws, int k, int q,
                                                    WaveStat* __restrict__ stat,
                                                    float* __restrict__ part,
                                                    unsigned int* __restrict__ rho_run)
{
    const int lane = __lane_id();
    const float scale = 1.44269504089f / lambda;
    unsigned int seen = 0x7f800000u;            // +inf
    if (lane == 0 && ws.n > 0) seen = atomicMin(rho_run, __float_as_uint(ws.rho + 0.0f));
    const float best = fminf(ws.rho, __uint_as_float(__builtin_amdgcn_readfirstlane(seen)));
    const bool skip = ws.n == 0 || (ws.rho - best) * scale > kSkipLog2;
    write_wave_stat(stat, ws, skip);
    if (skip) return;                           // wave-uniform

    constexpr int LB = L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : 3;
    constexpr int ST = 6 - LB < 4 ? 6 - LB : 4;
    const int nchunks = (a.N + 3) >> 2, n4 = 4 * a.N;
    const int idx_bits = (lane >> LB) & ((1 << ST) - 1);
    const bool store = (lane >> (LB + ST)) == 0;
    const float e = ws.e;
    for (int r = 0; r * L < nchunks; ++r) {
        const int c = r * L + q;
        float v[16];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = 4 * c + s;
            float du[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (e != 0.0f && j < a.N) draw_noise(a.np, (uint32_t)k, (uint32_t)j, du);
#pragma unroll
            for (int d = 0; d < 4; ++d) v[4 * s + d] = e * du[d];
        }
        wave_sum16<L>(v, lane);
        if (store) {
#pragma unroll
            for (int m = 0; m < (16 >> ST); ++m) {
                const int elem = 16 * c + ((m << ST) | idx_bits);
                if (elem < n4) part[elem] = v[m];
            }
        }
    }
}

// Arrival counter: every thread of a workgroup calls it after the workgroup's writes;
// true (on all its threads) for the workgroup that brings the count to `total`, which
// then sees the writes of every workgroup counted before it.  With reset, that
// workgroup also sets the counter back to 0.
__device__ __forceinline__ bool last_of(unsigned int* counter, unsigned int total, bool reset)
{
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                                    // release this workgroup's writes
        const bool last = atomicAdd(counter, 1u) == total - 1;
        if (last && reset) atomicExch(counter, 0u);
        s_last = last ? 1 : 0;
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) __threadfence();                              // acquire the others' writes
    return last;
}

// The workgroup of a launch that arrives last (the counter returns to 0 for the next).
__device__ __forceinline__ bool last_to_arrive(unsigned int* counter)
{
    return last_of(counter, gridDim.x * gridDim.y * gridDim.z, true);
}

// Records of wave statistics are split into kStatParts fixed parts: part p holds records
// 64 (p + kStatParts i) + l for lane l, i = 0, 1, ...  A lane sums its records in i order,
// a part's lanes are combined by one fixed shuffle tree and the parts in p order, so the
// binary64 sums depend on W alone: not on how many waves of the calling workgroup share
// the parts (wave v takes parts v, v + waves, ...) nor on how many records a lane has in
// flight (kB).
constexpr int kStatParts = 8;
constexpr int kStatStride = 64 * kStatParts;   // records between a lane's consecutive ones

template <int kB>
__device__ __forceinline__ void load_stat_batch(const WaveStat* __restrict__ stat, int W, int w0,
                                                WaveStat (&r)[kB])
{
#pragma unroll
    for (int u = 0; u < kB; ++u)             // unconditional loads: one wait for the batch
        r[u] = stat[w0 + kStatStride * u < W ? w0 + kStatStride * u : W - 1];
#pragma unroll
    for (int u = 0; u < kB; ++u)
        if (w0 + kStatStride * u >= W) r[u].n = 0;
}

struct StatSums {
    float rho;          // minimum finite cost (+inf if none)
    int argmin, nf;     // its first sample, finite costs
    double eta, q2;     // sum_w s_w eta_w, sum_w s_w^2 q_w
};

// The per-wave statistics stat[0..W) of one update reduced, returned to every thread of
// the calling workgroup (which it synchronises): rho = min rho_w with its first sample,
// n_finite, and with s_w = exp(-(rho_w - rho) / lambda), eta = sum_w s_w eta_w and
// sum_w s_w^2 q_w (binary64, in the fixed part order above; Eq. (4)).  When every part
// is one batch held by a wave of its own, the records stay in registers between the
// minimum pass and the sum pass: one memory round trip in all.
// With pre, the caller has already loaded each wave's batch into r (load_stat_batch at
// w0 = 64 wave + lane, waves below kStatParts), which requires stat_parts_fit(W): the
// records can then be loaded before other loads and waited for alone.
template <int kB>
__host__ __device__ constexpr bool stat_parts_fit(int W)
{
    return W <= kStatStride * kB;
}

template <int kB>
__device__ __forceinline__ StatSums reduce_stat_parts(const WaveStat* __restrict__ stat, int W,
                                                      float lambda, WaveStat (&r)[kB], bool pre)
{
    __shared__ float sh_v[kStatParts];
    __shared__ int sh_i[kStatParts], sh_n[kStatParts];
    __shared__ double sh_eta[kStatParts], sh_q[kStatParts];
    const int nw = (int)(blockDim.x >> 6);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const float scale = 1.44269504089f / lambda;
    const int used = (W + 63) / 64 < kStatParts ? (W + 63) / 64 : kStatParts;   // parts with records
    const bool keep = stat_parts_fit<kB>(W) && used <= nw;
    pre = pre && keep;
    if (!pre)
#pragma unroll
        for (int u = 0; u < kB; ++u) r[u] = WaveStat{INFINITY, 0.0f, 0.0f, 0.0f, -1, 0, 0, 0};

    for (int p = wv; p < kStatParts; p += nw) {
        float mv = INFINITY;
        int mi = INT_MAX, nf = 0;
        for (int w0 = 64 * p + lane; w0 < W; w0 += kStatStride * kB) {
            if (!pre) load_stat_batch<kB>(stat, W, w0, r);
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                nf += r[u].n;
                if (r[u].n > 0) argmin_merge(mv, mi, r[u].rho, r[u].argmin);
            }
        }
        wave_argmin_count(mv, mi, nf);
        if (lane == 0) { sh_v[p] = mv; sh_i[p] = mi; sh_n[p] = nf; }
    }
    __syncthreads();
    StatSums t;
    t.rho = sh_v[0]; t.argmin = sh_i[0]; t.nf = sh_n[0];
#pragma unroll
    for (int p = 1; p < kStatParts; ++p) { argmin_merge(t.rho, t.argmin, sh_v[p], sh_i[p]); t.nf += sh_n[p]; }
    t.eta = 0.0; t.q2 = 0.0;
    if (t.nf == 0) return t;                   // uniform: every thread read the same parts

    for (int p = wv; p < kStatParts; p += nw) {
        double eta = 0.0, q2 = 0.0;
        for (int w0 = 64 * p + lane; w0 < W; w0 += kStatStride * kB) {
            if (!keep) load_stat_batch<kB>(stat, W, w0, r);
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                if (r[u].n > 0) {
                    const double f = (double)__builtin_amdgcn_exp2f((t.rho - r[u].rho) * scale);
                    eta += f * ((double)r[u].eta_s + (double)r[u].eta_c);
                    q2 += f * f * (double)r[u].q;
                }
            }
        }
        eta = wave_sum(eta);
        q2 = wave_sum(q2);
        if (lane == 0) { sh_eta[p] = eta; sh_q[p] = q2; }
    }
    __syncthreads();
    t.eta = sh_eta[0]; t.q2 = sh_q[0];
#pragma unroll
    for (int p = 1; p < kStatParts; ++p) { t.eta += sh_eta[p]; t.q2 += sh_q[p]; }
    return t;
}

template <int kB>
__device__ __forceinline__ StatSums reduce_stat_parts(const WaveStat* __restrict__ stat, int W,
                                                      float lambda)
{
    WaveStat r[kB];
    return reduce_stat_parts<kB>(stat, W, lambda, r, false);
}

// diag from the reduced statistics (ess = 1 / sum w_k^2 = eta^2 / sum_w s_w^2 q_w).
__device__ __forceinline__ void write_stat_diag(const StatSums& t, int lanes, mppi_diag* __restrict__ diag)
{
    diag->rho = t.rho; diag->argmin = t.nf > 0 ? t.argmin : -1; diag->n_finite = t.nf; diag->lanes = lanes;
    if (t.nf == 0) {
        diag->eta = 0.0f; diag->ess = 0.0f; diag->status = MPPI_E_ALL_NONFINITE;
    } else {
        diag->eta = (float)t.eta; diag->ess = (float)(t.eta * t.eta / t.q2); diag->status = MPPI_OK;
    }
}

// Single pass: reduce the per-wave statistics stat[0..W) into diag as reduce_stat_parts
// does, with the list of the waves with s_w > 0 that formed partial sums, in index
// order, with their s_w.  Done by the first wave of the calling workgroup (lane l takes
// records l, l + 64, ...), eight records in flight per lane, so one wave builds the
// list in order without a scan across waves.
__device__ inline void reduce_wave_stats(const WaveStat* __restrict__ stat, int W, float lambda,
                                         int lanes, mppi_diag* __restrict__ diag,
                                         int* __restrict__ list_idx, float* __restrict__ list_s,
                                         int* __restrict__ list_n)
{
    if (threadIdx.x >= 64) return;
    constexpr int kBatch = 8;
    const int lane = threadIdx.x;
    const float scale = 1.44269504089f / lambda;

    float mv = INFINITY;
    int mi = INT_MAX, nf = 0;
    for (int w0 = lane; w0 < W; w0 += 64 * kBatch) {
        WaveStat r[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int w = w0 + 64 * u;
            if (w < W) r[u] = stat[w]; else r[u].n = 0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            nf += r[u].n;
            if (r[u].n > 0) argmin_merge(mv, mi, r[u].rho, r[u].argmin);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float v2 = __shfl_xor(mv, off);
        const int i2 = __shfl_xor(mi, off);
        argmin_merge(mv, mi, v2, i2);
        nf += __shfl_xor(nf, off);
    }
    const float rho = mv;
    if (lane == 0) {
        diag->rho = rho; diag->argmin = nf > 0 ? mi : -1; diag->n_finite = nf; diag->lanes = lanes;
        if (nf == 0) {
            diag->eta = 0.0f; diag->ess = 0.0f; diag->status = MPPI_E_ALL_NONFINITE;
            if (list_n) *list_n = 0;
        }
    }
    if (nf == 0) return;

    double eta = 0.0, q2 = 0.0;
    int base = 0;
    for (int c0 = 0; c0 < W; c0 += 64 * kBatch) {
        WaveStat r[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int w = c0 + 64 * u + lane;
            if (w < W) r[u] = stat[w]; else r[u].n = 0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const float f = r[u].n > 0 ? __builtin_amdgcn_exp2f((rho - r[u].rho) * scale) : 0.0f;
            if (r[u].n > 0) {
                eta += (double)f * ((double)r[u].eta_s + (double)r[u].eta_c);
                q2 += (double)f * (double)f * (double)r[u].q;
            }
            if (list_idx) {                    // contributing waves, in index order
                const bool in = f != 0.0f && !r[u].skipped;
                const unsigned long long m = __ballot(in);
                const int at = base + __popcll(m & ((1ull << lane) - 1ull));
                if (in) { list_idx[at] = c0 + 64 * u + lane; list_s[at] = f; }
                base += __popcll(m);
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        eta += __shfl_xor(eta, off);
        q2 += __shfl_xor(q2, off);
    }
    if (lane == 0) {
        diag->eta = (float)eta; diag->ess = (float)(eta * eta / q2); diag->status = MPPI_OK;
        if (list_n) *list_n = base;
    }
}

// Stored form, one workgroup of kSumThreads per row 4 j + d of delta_u [N][4][ld]:
// u_out[row] = u_in[row] + sum_k e_k delta_u[row][k] / eta with e_k = exp(-(S_k - rho)
// / lambda) (0 for non-finite costs), rho and eta from diag; u_out = u_in when every
// cost is non-finite.
__device__ __forceinline__ void update_sum_row(const float* __restrict__ S, const float* __restrict__ du,
                                               int K, int ld, float lambda,
                                               const float* __restrict__ u_in, float* __restrict__ u_out,
                                               const mppi_diag* __restrict__ diag, int row)
{
    __shared__ float sh[kSumThreads / 64];
    const int tid = threadIdx.x;
    const float rho = diag->rho, eta = diag->eta;
    const bool ok = diag->status == MPPI_OK;
    if (!ok) {
        if (tid == 0) u_out[row] = u_in[row];
        return;
    }
    const float scale = 1.44269504089f / lambda;
    const float* src = du + (size_t)row * ld;
    float acc = 0.0f;
    auto wt = [&](float s) { return isfinite(s) ? __builtin_amdgcn_exp2f((rho - s) * scale) : 0.0f; };
    if ((ld & 3) == 0) {
        const int K4 = K >> 2;
        const float4* s4 = reinterpret_cast<const float4*>(src);
        const float4* c4 = reinterpret_cast<const float4*>(S);
        const int stride = blockDim.x;
        for (int i = tid; i < K4; i += 4 * stride) {     // four float4 pairs in flight
            float4 a[4], c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int idx = i + u * stride;
                a[u] = idx < K4 ? s4[idx] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                c[u] = idx < K4 ? c4[idx] : make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc = fmaf(a[u].x, wt(c[u].x), acc);
                acc = fmaf(a[u].y, wt(c[u].y), acc);
                acc = fmaf(a[u].z, wt(c[u].z), acc);
                acc = fmaf(a[u].w, wt(c[u].w), acc);
            }
        }
        for (int k = 4 * K4 + tid; k < K; k += blockDim.x) acc = fmaf(src[k], wt(S[k]), acc);
    } else {
        for (int k = tid; k < K; k += blockDim.x) acc = fmaf(src[k], wt(S[k]), acc);
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        float t = 0.0f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
        u_out[row] = u_in[row] + t / eta;
    }
}

// The four rows of step j (controls d = 0..3) by one workgroup of kSumThreads threads:
// every thread sums the same samples of each row as update_sum_row's thread of the same
// index, in the same order, and each row is reduced by the same tree, so the results
// equal update_sum_row's bit for bit; the weight of each sample is formed once for the
// four rows and all four rows' loads are in flight together.
__device__ __forceinline__ void update_sum_step4(const float* __restrict__ S,
                                                 const float* __restrict__ du, int K, int ld,
                                                 float lambda, const float* __restrict__ u_in,
                                                 float* __restrict__ u_out,
                                                 const mppi_diag* __restrict__ diag, int j)
{
    __shared__ float sh[4][kSumThreads / 64];
    const int tid = threadIdx.x;
    const float rho = diag->rho, eta = diag->eta;
    const bool ok = diag->status == MPPI_OK;
    if (!ok) {
        if (tid < 4) u_out[4 * j + tid] = u_in[4 * j + tid];
        return;
    }
    const float scale = 1.44269504089f / lambda;
    const float* src = du + (size_t)(4 * j) * ld;
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto wt = [&](float s) { return isfinite(s) ? __builtin_amdgcn_exp2f((rho - s) * scale) : 0.0f; };
    constexpr int stride = kSumThreads;
    if ((ld & 3) == 0) {
        const int K4 = K >> 2;
        const float4* c4 = reinterpret_cast<const float4*>(S);
        auto clamp4 = [&](int idx) { return idx < K4 ? idx : K4 - 1; };
        for (int i = tid; i < K4; i += 4 * stride) {     // four float4 per row in flight
            float4 c[4], a[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ic = clamp4(i + u * stride);
                c[u] = c4[ic];
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    a[d][u] = reinterpret_cast<const float4*>(src + (size_t)d * ld)[ic];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool in = i + u * stride < K4;
                const float4 cc = in ? c[u] : make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
                const float4 w = make_float4(wt(cc.x), wt(cc.y), wt(cc.z), wt(cc.w));
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const float4 av = in ? a[d][u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    acc[d] = fmaf(av.x, w.x, acc[d]);
                    acc[d] = fmaf(av.y, w.y, acc[d]);
                    acc[d] = fmaf(av.z, w.z, acc[d]);
                    acc[d] = fmaf(av.w, w.w, acc[d]);
                }
            }
        }
        for (int k = 4 * K4 + tid; k < K; k += stride) {
            const float w = wt(S[k]);
#pragma unroll
            for (int d = 0; d < 4; ++d) acc[d] = fmaf(src[(size_t)d * ld + k], w, acc[d]);
        }
    } else {
        for (int k = tid; k < K; k += stride) {
            const float w = wt(S[k]);
#pragma unroll
            for (int d = 0; d < 4; ++d) acc[d] = fmaf(src[(size_t)d * ld + k], w, acc[d]);
        }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        acc[d] = wave_sum(acc[d]);
        if ((tid & 63) == 0) sh[d][tid >> 6] = acc[d];
    }
    __syncthreads();
    if (tid < 4) {
        float t = 0.0f;
        for (int i = 0; i < kSumThreads / 64; ++i) t += sh[tid][i];
        u_out[4 * j + tid] = u_in[4 * j + tid] + t / eta;
    }
}

// Weighted sums of step j's rows (Eq. (5)), then the apply and advance (Algorithm 1;
// Sec. IV-B), one workgroup of kSumStepThreads per step j.  With the plain shift
// (alpha = 1) workgroup j writes knot j - 1 (= step j's update) and the last also the
// refilled knot N - 1; with interpolation it also sums step j + 1's rows and writes knot
// j, so no workgroup reads another's result.  u_src is a copy of the warm start the
// update started from (the rollout launch makes it), since u_nom is written here.  Every workgroup first reduces the rollout waves'
// statistics stat[0..W) itself (the same result in each; workgroup 0 writes diag), with
// its first costs and delta_u loads already in flight.  Group d of kSumThreads threads
// sums control d of steps j and j + 1, each row in update_sum_row's order (the same
// samples per thread, the same reduction tree), so the results equal those of the
// separate statistics, sum and apply launches bit for bit.
constexpr int kSumStepThreads = 4 * kSumThreads;

__device__ __forceinline__ void update_sum_shift_step(const float* __restrict__ S,
                                                      const float* __restrict__ du, int K, int ld,
                                                      float lambda, const float* __restrict__ u_src,
                                                      const ModelParams& P,
                                                      const float* __restrict__ x_hat,
                                                      float* __restrict__ u_nom,
                                                      float* __restrict__ u_apply, int N,
                                                      float4 u_init, float alpha,
                                                      const WaveStat* __restrict__ stat, int W,
                                                      int lanes, mppi_diag* __restrict__ diag, int j)
{
    constexpr int nw = kSumThreads / 64;              // waves per group
    __shared__ float sh[8][nw];
    const int tid = threadIdx.x, d = tid / kSumThreads, gt = tid % kSumThreads;
    const bool shift = alpha == 1.0f;
    const int nr = !shift && j + 1 < N ? 2 : 1;       // control d of step j (and j + 1)
    const float* src = du + (size_t)(4 * j + d) * ld;  // row of step j; + 4 ld: step j + 1
    const bool vec = (ld & 3) == 0;
    const int K4 = vec ? K >> 2 : 0;
    const float4* c4 = reinterpret_cast<const float4*>(S);
    // Loads at clamped indices, masked where they are used: no load sits in a branch,
    // so a batch of them is in flight together.
    auto clamp4 = [&](int idx) { return idx < K4 ? idx : K4 - 1; };
    // the statistics records first (vector loads complete in order: they can be waited
    // for while the delta_u loads below are still in flight)
    WaveStat rec[4];
    const bool pre = stat_parts_fit<4>(W);
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (pre && wv < kStatParts) load_stat_batch<4>(stat, W, 64 * wv + (tid & 63), rec);
    float4 c0[4], a0[2][4];                           // the first iteration's operands
    if (K4 > 0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int ic = clamp4(gt + u * kSumThreads);
            c0[u] = c4[ic];
#pragma unroll
            for (int r = 0; r < 2; ++r)               // step j + 1 only if it exists
                a0[r][u] = reinterpret_cast<const float4*>(src + (size_t)(4 * (r < nr ? r : 0)) * ld)[ic];
        }
    }
    float us[8];                                      // u_src of steps j and j + 1, for thread 0
    if (tid == 0)
#pragma unroll
        for (int r = 0; r < 8; ++r) us[r] = u_src[4 * j + (r < 4 * nr ? r : 0)];
    const StatSums st = reduce_stat_parts<4>(stat, W, lambda, rec, pre);
    if (j == 0 && tid == 0) write_stat_diag(st, lanes, diag);
    const bool ok = st.nf > 0;
    float acc[2] = {0.0f, 0.0f};
    float eta = 1.0f;
    if (ok) {
        const float rho = st.rho;
        eta = (float)st.eta;
        const float scale = 1.44269504089f / lambda;
        auto wt = [&](float s) { return isfinite(s) ? __builtin_amdgcn_exp2f((rho - s) * scale) : 0.0f; };
        if (vec) {
            for (int i = gt; i < K4; i += 4 * kSumThreads) {   // four float4 pairs in flight
                const bool first = i == gt;
                float4 w[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int idx = i + u * kSumThreads;
                    const float4 cl = first ? c0[u] : c4[clamp4(idx)];
                    const float4 c = idx < K4 ? cl : make_float4(INFINITY, INFINITY, INFINITY, INFINITY);
                    w[u] = make_float4(wt(c.x), wt(c.y), wt(c.z), wt(c.w));
                }
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    if (r >= nr) break;
                    const float4* s4 = reinterpret_cast<const float4*>(src + (size_t)(4 * r) * ld);
                    float4 a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int idx = i + u * kSumThreads;
                        const float4 al = first ? a0[r][u] : s4[clamp4(idx)];
                        a[u] = idx < K4 ? al : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        acc[r] = fmaf(a[u].x, w[u].x, acc[r]);
                        acc[r] = fmaf(a[u].y, w[u].y, acc[r]);
                        acc[r] = fmaf(a[u].z, w[u].z, acc[r]);
                        acc[r] = fmaf(a[u].w, w[u].w, acc[r]);
                    }
                }
            }
            for (int k = 4 * K4 + gt; k < K; k += kSumThreads) {
                const float w = wt(S[k]);
                for (int r = 0; r < nr; ++r) acc[r] = fmaf(src[(size_t)(4 * r) * ld + k], w, acc[r]);
            }
        } else {
            for (int k = gt; k < K; k += kSumThreads) {
                const float w = wt(S[k]);
                for (int r = 0; r < nr; ++r) acc[r] = fmaf(src[(size_t)(4 * r) * ld + k], w, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            acc[r] = wave_sum(acc[r]);
            if ((gt & 63) == 0) sh[4 * r + d][gt >> 6] = acc[r];
        }
        __syncthreads();
    }
    if (tid != 0) return;
    const float init[4] = {u_init.x, u_init.y, u_init.z, u_init.w};
    float up[8];                                      // u_upd of steps j (0..3) and j + 1 (4..7)
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if (r >= 4 * nr) {
            up[r] = init[r - 4];
            continue;
        }
        float t = 0.0f;
        if (ok)
            for (int i = 0; i < nw; ++i) t += sh[r][i];
        up[r] = ok ? us[r] + t / eta : us[r];
    }
    if (j == 0) {
        for (int c = 0; c < 4; ++c) u_apply[c] = up[c];
        feasible_input(P, x_hat, up, u_apply + 4);
    }
    if (!ok) return;   // all costs non-finite: keep the warm start as it was
    if (shift) {       // the plain shift, copied exactly: knot j - 1 <- step j
        if (j > 0)
            for (int c = 0; c < 4; ++c) u_nom[4 * (j - 1) + c] = up[c];
        if (j == N - 1)
            for (int c = 0; c < 4; ++c) u_nom[4 * j + c] = init[c];
        return;
    }
    // knot j moves to the value at j + alpha of the interpolant (Sec. IV-B)
    const float keep = 1.0f - alpha;
    for (int c = 0; c < 4; ++c) u_nom[4 * j + c] = fmaf(alpha, up[4 + c], keep * up[c]);
}

// Single pass, one workgroup of kMergeThreads = 64 columns x 4 waves: u_out[col] =
// u_in[col] + sum over the listed waves of s_w P_w[col] / eta (binary64), the waves
// of the list divided among the workgroup's waves.
__device__ __forceinline__ void merge_sum_cols(const float* __restrict__ part, int N,
                                               const int* __restrict__ list_idx,
                                               const float* __restrict__ list_s,
                                               const int* __restrict__ list_n,
                                               const float* __restrict__ u_in, float* __restrict__ u_out,
                                               const mppi_diag* __restrict__ diag, int col0)
{
    __shared__ double sh[kMergeThreads];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
    const int col = col0 + lane;
    const int n4 = 4 * N;
    const bool ok = diag->status == MPPI_OK;
    double acc = 0.0;
    if (ok && col < n4) {
        const int n = *list_n;
        const size_t ldp = (size_t)n4;
        int t = wv;
        for (; t + 3 * nw < n; t += 4 * nw) {              // four independent loads in flight
            const float p0 = part[(size_t)list_idx[t] * ldp + col];
            const float p1 = part[(size_t)list_idx[t + nw] * ldp + col];
            const float p2 = part[(size_t)list_idx[t + 2 * nw] * ldp + col];
            const float p3 = part[(size_t)list_idx[t + 3 * nw] * ldp + col];
            acc += (double)list_s[t] * p0;
            acc += (double)list_s[t + nw] * p1;
            acc += (double)list_s[t + 2 * nw] * p2;
            acc += (double)list_s[t + 3 * nw] * p3;
        }
        for (; t < n; t += nw) acc += (double)list_s[t] * part[(size_t)list_idx[t] * ldp + col];
    }
    sh[tid] = acc;
    __syncthreads();
    if (wv == 0 && col < n4) {
        double tot = 0.0;
        for (int w = 0; w < nw; ++w) tot += sh[w * 64 + lane];
        u_out[col] = ok ? u_in[col] + (float)(tot / (double)diag->eta) : u_in[col];
    }
}

// `steps` noise-free model steps of one command held (the closed-loop plant, and the
// delay prediction of Sec. IV-E), by one thread; x_out may alias x_in.
__device__ inline void model_steps(const ModelParams& P, const float* x_in,
                                   const float* __restrict__ u_in, float* x_out, int steps)
{
    State x;
    x.px = x_in[0]; x.py = x_in[1]; x.pz = x_in[2];
    x.qw = x_in[3]; x.qx = x_in[4]; x.qy = x_in[5]; x.qz = x_in[6];
    x.vx = x_in[7]; x.vy = x_in[8]; x.vz = x_in[9];
    x.wx = x_in[10]; x.wy = x_in[11]; x.wz = x_in[12];
    x.T0 = x_in[13]; x.T1 = x_in[14]; x.T2 = x_in[15]; x.T3 = x_in[16];
    const float u[4] = {u_in[0], u_in[1], u_in[2], u_in[3]};
    for (int s = 0; s < steps; ++s) {
        float Tc[4];
        rate_controller(P, x.wx, x.wy, x.wz, u, Tc);
        if (P.lag)
            rk4_step<true>(P, x, Tc);
        else
            rk4_step<false>(P, x, Tc);
    }
    const float out[17] = {x.px, x.py, x.pz, x.qw, x.qx, x.qy, x.qz, x.vx, x.vy, x.vz,
                           x.wx, x.wy, x.wz, x.T0, x.T1, x.T2, x.T3};
    for (int i = 0; i < 17; ++i) x_out[i] = out[i];
}

// One workgroup writes u_apply and the shifted warm start of one instance.
__device__ __forceinline__ void apply_shift_block(const ModelParams& P, const float* __restrict__ x_hat,
                                                  const float* __restrict__ u_upd,
                                                  float* __restrict__ u_nom,
                                                  float* __restrict__ u_apply, int N, float4 u_init,
                                                  float alpha, const mppi_diag* __restrict__ diag)
{
    const bool ok = diag == nullptr || diag->status == MPPI_OK;
    if (threadIdx.x == 0) {
        for (int d = 0; d < 4; ++d) u_apply[d] = u_upd[d];
        feasible_input(P, x_hat, u_upd, u_apply + 4);
    }
    if (!ok) return;   // all costs non-finite: keep the warm start as it was
    const float init[4] = {u_init.x, u_init.y, u_init.z, u_init.w};
    // Knot j moves to the value at j + alpha of the linear interpolant through
    // u_upd[0..N-1] and u_init (Sec. IV-B); alpha = 1 is the plain shift, copied exactly.
    const bool shift = alpha == 1.0f;
    const float keep = 1.0f - alpha;
    for (int i = threadIdx.x; i < 4 * N; i += blockDim.x) {
        const float next = i < 4 * (N - 1) ? u_upd[i + 4] : init[i & 3];
        u_nom[i] = shift ? next : fmaf(alpha, next, keep * u_upd[i]);
    }
}

}  // namespace mppi
