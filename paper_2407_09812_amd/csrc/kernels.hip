// One-instance MPPI kernels for gfx950 (wave64, CDNA4).
//
//   rollout_kernel      one sample per L lanes: in-register Philox noise, rate
//                       controller, RK4 of the 17-value state, tracking and
//                       obstacle cost (obstacles staged in LDS)        Eqs. (2)-(3)
//   rollout_pipe_kernel the same rollouts wave-specialised: noise, body rates,
//                       attitude, translation and obstacle waves per 64 samples,
//                       handing chunks of steps over through LDS        Sec. III
//   weights_kernel      one workgroup: wave-shuffle min, compensated
//                       sum of exp(-(S - rho)/lambda), normalisation   Eq. (4)
//   weighted_sum_kernel one workgroup per (j, d) row of delta_u [N][4][ld]:
//                       coalesced float4 GEMV against the weights       Eq. (5)
//   update_sum_kernel   the full update's weighted sum, one workgroup per step: it
//                       reduces the rollout waves' weight statistics, forms the
//                       weights on the fly from the costs, applies and advances
//   rollout_fused_kernel, merge_sum_kernel   the single pass: per-wave partial sums
//                       with regenerated noise instead of stored delta_u, then their
//                       rescaled sum (and apply)
//   apply_shift_kernel  u_apply and the advanced warm start   Algorithm 1, Sec. IV-B
//   plant_kernel        noise-free model steps (plant, delay prediction)  Sec. IV-E
//   noise_kernel, philox_kernel   the rollout's noise on its own (checks)
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "stages.h"

namespace mppi {

// Rollouts; with stat (a full update), each wave also writes its weight statistics
// (the sum launch reduces them).
template <int L, int U, bool kLag, bool kDump>
__global__ __launch_bounds__(256) void rollout_kernel(
    RolloutParams a, const float* __restrict__ x_hat, const float* __restrict__ x_ref,
    const mppi_obstacle* __restrict__ obs, const float* __restrict__ u_nom,
    float* __restrict__ du_out, float* __restrict__ S_out, float* __restrict__ states,
    UpdateTail tail)
{
    extern __shared__ float4 obs_lds[];   // obstacle_lds_bytes(M)
    if (tail.u_copy && blockIdx.x == 0)   // the warm start, for the sum launch that rewrites it
        for (int i = threadIdx.x; i < 4 * a.N; i += blockDim.x) tail.u_copy[i] = u_nom[i];
    stage_obstacles(obs_lds, obs, a.M, x_hat[0], x_hat[1], x_hat[2], a.cp.margin);
    __syncthreads();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = g / L, q = g % L;
    const float S = rollout_sample<L, U, kLag, kDump>(a, x_hat, x_ref, u_nom, du_out, S_out, states,
                                                      obs_lds, k, q);
    if (tail.stat == nullptr) return;                       // launch-uniform
    write_wave_stat(tail.stat + (g >> 6), wave_sums(S, k, q, k < a.K, tail.lambda), false);
}

// Single pass: rollouts, per-wave statistics and partial sums; the last workgroup
// reduces the statistics into diag and the list of contributing waves.
template <int L, int U, bool kLag>
__global__ __launch_bounds__(256) void rollout_fused_kernel(
    RolloutParams a, const float* __restrict__ x_hat, const float* __restrict__ x_ref,
    const mppi_obstacle* __restrict__ obs, const float* __restrict__ u_nom,
    float* __restrict__ S_out, UpdateTail tail)
{
    extern __shared__ float4 obs_lds[];   // obstacle_lds_bytes(M)
    stage_obstacles(obs_lds, obs, a.M, x_hat[0], x_hat[1], x_hat[2], a.cp.margin);
    __syncthreads();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = g / L, q = g % L;
    const float S = rollout_sample<L, U, kLag, false, false>(a, x_hat, x_ref, u_nom, nullptr, S_out,
                                                             nullptr, obs_lds, k, q);
    const int w = g >> 6;
    fused_wave_partials<L>(a, tail.lambda, wave_sums(S, k, q, k < a.K, tail.lambda), k, q,
                           tail.stat + w, tail.part + (size_t)w * 4 * a.N, tail.rho_run);
    if (last_to_arrive(tail.counter)) {
        reduce_wave_stats(tail.stat, (int)(gridDim.x * blockDim.x >> 6), tail.lambda, L, tail.diag,
                          tail.list_idx, tail.list_s, tail.list_n);
        if (threadIdx.x == 0) *tail.rho_run = 0x7f800000u;   // every wave has published
    }
}

// Wave-specialised rollouts of 64 samples per workgroup (roles in stages.h): wave 0
// noise, wave 1 body rates, wave 2 attitude, wave 3 translation and tracking cost,
// waves 4 .. 4 + L - 1 obstacles and the running cost.  Obstacles and hand-over buffers live in LDS; with
// tail.stat the obstacle waves write the weight statistics, which the sum launch
// reduces (single pass, kFused: and their partial sums, delta_u not stored, and the
// last workgroup reduces the statistics with the list of contributing waves).
static_assert(pipe_lds_bytes(kPipeMaxM) <= 160 * 1024, "the pipe's LDS must fit one gfx950 CU");

template <int L, int U, bool kLag, bool kFused, int C>
__global__ __launch_bounds__(64 * (4 + 8)) void rollout_pipe_kernel(
    RolloutParams a, const float* __restrict__ x_hat, const float* __restrict__ x_ref,
    const mppi_obstacle* __restrict__ obs, const float* __restrict__ u_nom,
    float* __restrict__ du_out, float* __restrict__ S_out, UpdateTail tail)
{
    extern __shared__ float4 lds[];       // obstacles, then PipeLds
    float4* obs_lds = lds;
    PipeLdsT<C>& P = *reinterpret_cast<PipeLdsT<C>*>(lds + obstacle_lds_float4(a.M));
    if (tail.u_copy && blockIdx.x == 0)   // the warm start, for the sum launch that rewrites it
        for (int i = threadIdx.x; i < 4 * a.N; i += blockDim.x) tail.u_copy[i] = u_nom[i];
    const float phx = x_hat[0], phy = x_hat[1], phz = x_hat[2];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int nch = (a.N + C - 1) / C;
    constexpr int kO = 4;                 // first obstacle wave
    int sb = lane, q = 0;
    if (wv >= kO) {                       // 64 / L samples per obstacle wave
        sb = (wv - kO) * (64 / L) + lane / L;
        q = lane % L;
    }
    const int k = blockIdx.x * 64 + sb;
    const bool valid = k < a.K;
    const int kk = valid ? k : a.K - 1;
    const bool writer = valid && q == 0;
    float up[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // The noise role runs one chunk ahead of the rates role: its first chunk is drawn
    // while the other waves stage the obstacles (the staging work is shifted off wave 0).
    stage_obstacles(obs_lds, obs, a.M, phx, phy, phz, a.cp.margin, (int)blockDim.x - 64, [&]() {
        if (wv == 0) pipe_noise_chunk<!kFused>(a, u_nom, x_ref, du_out, writer, kk, 0, up, P, lane);
    });
    __syncthreads();

    State x;
    x.px = 0.0f; x.py = 0.0f; x.pz = 0.0f;
    x.qw = x_hat[3]; x.qx = x_hat[4]; x.qy = x_hat[5]; x.qz = x_hat[6];
    x.vx = x_hat[7]; x.vy = x_hat[8]; x.vz = x_hat[9];
    x.wx = x_hat[10]; x.wy = x_hat[11]; x.wz = x_hat[12];
    x.T0 = x_hat[13]; x.T1 = x_hat[14]; x.T2 = x_hat[15]; x.T3 = x_hat[16];
    KahanSum S;
    int tested = 0;
    const float4 oh = obs_lds[0];          // obstacle block header
    if (wv >= kO)                          // state j = 0 is scored too (Eq. (17))
        S.add(state_cost<L, U>(a.cp, x, x_ref, phx, phy, phz, oh, obs_lds, a.M, q, tested));

    // Each role runs its own loop over the nch + kO - 1 phases (chunk c: noise in phase
    // c - 1, its first chunk during the staging; rates in phase c, attitude c + 1,
    // translation c + 2, obstacles c + 3), with one workgroup barrier per phase in every
    // loop (the barrier counts waves, not code locations), so that only the role's own
    // parameters are live in its loop.
    const int nph = nch + kO - 1;
    // with 4 or 8 lanes per sample and a list worth culling, the obstacle waves cull by
    // the box of each chunk's positions and the translation role takes no windows
    const bool boxed = L >= 4 && a.M >= kCullMin;
    if (wv == 0) {
        for (int ph = 0; ph < nph; ++ph) {
            if (ph + 1 < nch) pipe_noise_chunk<!kFused>(a, u_nom, x_ref, du_out, writer, kk, ph + 1, up, P, lane);
            __syncthreads();
        }
    } else if (wv == 1) {
        for (int ph = 0; ph < nph; ++ph) {
            if (ph < nch) pipe_rates_chunk<kLag>(a, x, ph, P, lane);
            __syncthreads();
        }
    } else if (wv == 2) {
        for (int ph = 0; ph < nph; ++ph) {
            if (ph >= 1 && ph < nch + 1) pipe_attitude_chunk(a, x, ph - 1, P, lane);
            __syncthreads();
        }
    } else if (wv == 3) {
        for (int ph = 0; ph < nph; ++ph) {
            if (ph >= 2 && ph < nch + 2)
                pipe_translation_chunk<L>(a, oh, obs_lds, phx, phy, phz, x, ph - 2, lane, P, !boxed);
            __syncthreads();
        }
    } else {
        // The obstacle waves share their SIMDs with the role waves (wave w + 4 with wave
        // w) and are the ones whose chunk takes longest; by default the older role wave
        // is issued first, so the obstacle waves raise their issue priority.
        __builtin_amdgcn_s_setprio(1);
        // a block of vertical cylinders only skips the z terms of the tests
        const int* bins = reinterpret_cast<const int*>(obs_lds + 1);
        const bool zfree = __builtin_amdgcn_readfirstlane(bins[kObsSphereSlot]) == 0;
        auto phases = [&](auto chunk) {
            for (int ph = 0; ph < nph; ++ph) {
                if (ph >= kO - 1) chunk(ph - (kO - 1));
                __syncthreads();
            }
        };
        if constexpr (L >= 4) {
            if (boxed) {
                if (zfree)
                    phases([&](int cc) { pipe_obstacle_chunk_box<L, U, false>(a, oh, obs_lds, S, tested, cc, sb, q, P); });
                else
                    phases([&](int cc) { pipe_obstacle_chunk_box<L, U, true>(a, oh, obs_lds, S, tested, cc, sb, q, P); });
            }
        }
        if (!boxed) {
            if (zfree)
                phases([&](int cc) { pipe_obstacle_chunk<L, U, false>(a, obs_lds, S, tested, cc, sb, q, wv - kO, P); });
            else
                phases([&](int cc) { pipe_obstacle_chunk<L, U, true>(a, obs_lds, S, tested, cc, sb, q, wv - kO, P); });
        }
    }
    if (wv >= kO) {
        if (writer) S_out[k] = S.s;
        if (a.obs_tests) {
            const unsigned long long samples = __popcll(__ballot(writer));
            if (lane == 0) atomicAdd(a.obs_tests, samples * (unsigned long long)tested);
        }
        const int w = blockIdx.x * L + (wv - kO);
        if (kFused)
            fused_wave_partials<L>(a, tail.lambda, wave_sums(S.s, k, q, valid, tail.lambda), kk, q,
                                   tail.stat + w, tail.part + (size_t)w * 4 * a.N, tail.rho_run);
        else if (tail.stat)
            write_wave_stat(tail.stat + w, wave_sums(S.s, k, q, valid, tail.lambda), false);
    }
    if (kFused && last_to_arrive(tail.counter)) {
        reduce_wave_stats(tail.stat, (int)gridDim.x * L, tail.lambda, L, tail.diag, tail.list_idx,
                          tail.list_s, tail.list_n);
        if (threadIdx.x == 0) *tail.rho_run = 0x7f800000u;   // every wave has published
    }
}

// Weighted sum of the stored delta_u with the apply and advance, one workgroup per
// step j (Eq. (5); Algorithm 1): it sums the rows of steps j and j + 1 and writes knot
// j (and, for j = 0, u_apply), so no workgroup waits for another's result.
__global__ __launch_bounds__(kSumStepThreads) void update_sum_kernel(
    const float* __restrict__ S, const float* __restrict__ du, int K, int ld, float lambda,
    const float* __restrict__ u_src, const WaveStat* __restrict__ stat, int W, int lanes,
    mppi_diag* __restrict__ diag, ApplyArgs ap)
{
    update_sum_shift_step(S, du, K, ld, lambda, u_src, ap.P, ap.x_hat, ap.u_nom, ap.u_apply, ap.N,
                          ap.u_init, ap.alpha, stat, W, lanes, diag, blockIdx.x);
}

// Single pass: the listed waves' partial sums, 64 columns per workgroup; the last
// workgroup applies and advances.
__global__ __launch_bounds__(kMergeThreads) void merge_sum_kernel(
    const float* __restrict__ part, int N, const int* __restrict__ list_idx,
    const float* __restrict__ list_s, const int* __restrict__ list_n, const float* __restrict__ u_in,
    float* __restrict__ u_upd, const mppi_diag* __restrict__ diag, ApplyArgs ap,
    unsigned int* __restrict__ counter)
{
    merge_sum_cols(part, N, list_idx, list_s, list_n, u_in, u_upd, diag, blockIdx.x * 64);
    if (last_to_arrive(counter))
        apply_shift_block(ap.P, ap.x_hat, u_upd, ap.u_nom, ap.u_apply, ap.N, ap.u_init, ap.alpha,
                          diag);
}

__global__ __launch_bounds__(kWeightsThreads) void weights_kernel(const float* __restrict__ S, int K,
                                                                 float lambda, float* __restrict__ w,
                                                                 mppi_diag* __restrict__ diag, int lanes)
{
    weights_block(S, K, lambda, w, diag, lanes);
}

__global__ __launch_bounds__(kSumThreads) void weighted_sum_kernel(
    const float* __restrict__ w, const float* __restrict__ du, int K, int ld,
    const float* __restrict__ u_in, float* __restrict__ u_out, const mppi_diag* __restrict__ diag)
{
    const int row = blockIdx.x;
    weighted_sum_row(w, du, K, ld, u_in, u_out, diag, row);
}

__global__ void apply_shift_kernel(ModelParams P, const float* __restrict__ x_hat,
                                   const float* __restrict__ u_upd, float* __restrict__ u_nom,
                                   float* __restrict__ u_apply, int N, float4 u_init,
                                   float alpha, const mppi_diag* __restrict__ diag)
{
    apply_shift_block(P, x_hat, u_upd, u_nom, u_apply, N, u_init, alpha, diag);
}

// ---------------------------------------------------------------------------
// Plant, noise and Philox kernels
// ---------------------------------------------------------------------------

__global__ void plant_kernel(ModelParams P, const float* x_in, const float* __restrict__ u_in,
                             float* x_out, int steps)
{
    if (threadIdx.x == 0) model_steps(P, x_in, u_in, x_out, steps);
}

__global__ void noise_kernel(NoiseParams np, int K, int N, float* __restrict__ du, int ld)
{
    const size_t total = (size_t)K * N;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i % K), j = (int)(i / K);
        float v[4];
        draw_noise(np, (uint32_t)k, (uint32_t)j, v);
        for (int d = 0; d < 4; ++d) du[(size_t)(4 * j + d) * ld + k] = v[d];
    }
}

__global__ void philox_kernel(int n, const uint4* __restrict__ ctr, const uint2* __restrict__ key,
                              uint4* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = philox4x32_10(ctr[i], key[i].x, key[i].y);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------

bool valid_config(const LaunchConfig& c)
{
    return (c.block == 64 || c.block == 128 || c.block == 256) &&
           (c.lanes == 1 || c.lanes == 2 || c.lanes == 4 || c.lanes == 8) &&
           (c.unroll == 1 || c.unroll == 4) && (c.fused == 0 || c.fused == 1) &&
           (c.pipe == 0 || c.pipe == 1);
}

int rollout_waves(int K, const LaunchConfig& c)
{
    const size_t threads = (size_t)K * c.lanes;
    const size_t grid = (threads + c.block - 1) / c.block;
    return (int)(grid * c.block / 64);
}

template <int L, int U>
static hipError_t launch_rollout_lu(const RolloutArgs& a, int block, const UpdateTail& tail,
                                    bool fused, hipStream_t stream)
{
    const size_t threads = (size_t)a.K * L;
    const int grid = (int)((threads + block - 1) / block);
    const size_t lds = obstacle_lds_bytes(a.M);
    const RolloutParams p{a.mp, a.cp, a.np, a.M, a.K, a.N, a.ld, a.obs_tests};
    if (fused) {
        auto kernel = a.mp.lag ? rollout_fused_kernel<L, U, true> : rollout_fused_kernel<L, U, false>;
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, p, a.x_hat, a.x_ref, a.obs,
                           a.u_nom, a.S, tail);
    } else {
        auto kernel = a.mp.lag ? (a.states ? rollout_kernel<L, U, true, true> : rollout_kernel<L, U, true, false>)
                               : (a.states ? rollout_kernel<L, U, false, true> : rollout_kernel<L, U, false, false>);
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), lds, stream, p, a.x_hat, a.x_ref, a.obs,
                           a.u_nom, a.du, a.S, a.states, tail);
    }
    return hipGetLastError();
}

template <int L>
static hipError_t launch_rollout_l(const RolloutArgs& a, const LaunchConfig& c, const UpdateTail& tail,
                                   bool fused, hipStream_t stream)
{
    return c.unroll == 4 ? launch_rollout_lu<L, 4>(a, c.block, tail, fused, stream)
                         : launch_rollout_lu<L, 1>(a, c.block, tail, fused, stream);
}

static hipError_t launch_rollout_any(const RolloutArgs& a, const LaunchConfig& c,
                                     const UpdateTail& tail, bool fused, hipStream_t stream)
{
    if (!valid_config(c)) return hipErrorInvalidValue;
    switch (c.lanes) {
    case 1: return launch_rollout_l<1>(a, c, tail, fused, stream);
    case 2: return launch_rollout_l<2>(a, c, tail, fused, stream);
    case 4: return launch_rollout_l<4>(a, c, tail, fused, stream);
    default: return launch_rollout_l<8>(a, c, tail, fused, stream);
    }
}

hipError_t launch_rollout(const RolloutArgs& a, const LaunchConfig& c, hipStream_t stream,
                          const UpdateTail* tail)
{
    UpdateTail none{};
    return launch_rollout_any(a, c, tail ? *tail : none, false, stream);
}

hipError_t launch_rollout_fused(const RolloutArgs& a, const LaunchConfig& c, const UpdateTail& tail,
                                hipStream_t stream)
{
    if (!tail.stat || !tail.part || !tail.rho_run || !tail.list_idx) return hipErrorInvalidValue;
    return launch_rollout_any(a, c, tail, true, stream);
}

template <int L, int U, int C>
static hipError_t launch_pipe_luc(const RolloutArgs& a, const UpdateTail& tail, bool fused,
                                  hipStream_t stream)
{
    const int grid = (a.K + 63) / 64;
    const RolloutParams p{a.mp, a.cp, a.np, a.M, a.K, a.N, a.ld, a.obs_tests};
    auto kernel = fused ? (a.mp.lag ? rollout_pipe_kernel<L, U, true, true, C> : rollout_pipe_kernel<L, U, false, true, C>)
                        : (a.mp.lag ? rollout_pipe_kernel<L, U, true, false, C> : rollout_pipe_kernel<L, U, false, false, C>);
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(64 * (4 + L)), pipe_lds_bytes<C>(a.M), stream, p, a.x_hat,
                       a.x_ref, a.obs, a.u_nom, a.du, a.S, tail);
    return hipGetLastError();
}

// Chunks of 2 steps for short horizons: the pipeline's fill (3 phases) is a smaller
// share of the few chunks there are.
template <int L, int U>
static hipError_t launch_pipe_lu(const RolloutArgs& a, const UpdateTail& tail, bool fused,
                                 hipStream_t stream)
{
    return a.N <= kPipeShortN ? launch_pipe_luc<L, U, 2>(a, tail, fused, stream)
                              : launch_pipe_luc<L, U, kPipeChunk>(a, tail, fused, stream);
}

template <int L>
static hipError_t launch_pipe_l(const RolloutArgs& a, const LaunchConfig& c, const UpdateTail& tail,
                                hipStream_t stream)
{
    const bool fused = c.fused != 0;
    return c.unroll == 4 ? launch_pipe_lu<L, 4>(a, tail, fused, stream)
                         : launch_pipe_lu<L, 1>(a, tail, fused, stream);
}

hipError_t launch_rollout_pipe(const RolloutArgs& a, const LaunchConfig& c, hipStream_t stream,
                               const UpdateTail* tail)
{
    if (!valid_config(c) || !c.pipe || a.M > kPipeMaxM) return hipErrorInvalidValue;
    if (c.fused && (!tail || !tail->stat || !tail->part || !tail->rho_run || !tail->list_idx))
        return hipErrorInvalidValue;
    UpdateTail none{};
    const UpdateTail& t = tail ? *tail : none;
    switch (c.lanes) {
    case 1: return launch_pipe_l<1>(a, c, t, stream);
    case 2: return launch_pipe_l<2>(a, c, t, stream);
    case 4: return launch_pipe_l<4>(a, c, t, stream);
    default: return launch_pipe_l<8>(a, c, t, stream);
    }
}

hipError_t launch_update_sum(const float* S, const float* du, int K, int N, int ld, float lambda,
                             const float* u_src, const WaveStat* stat, int W, int lanes,
                             mppi_diag* diag, const ApplyArgs& ap, hipStream_t stream)
{
    hipLaunchKernelGGL(update_sum_kernel, dim3(N), dim3(kSumStepThreads), 0, stream, S, du, K, ld,
                       lambda, u_src, stat, W, lanes, diag, ap);
    return hipGetLastError();
}

hipError_t launch_merge_sum(const float* part, int N, const int* list_idx, const float* list_s,
                            const int* list_n, const float* u_in, float* u_upd,
                            const mppi_diag* diag, const ApplyArgs& ap, unsigned int* counter,
                            hipStream_t stream)
{
    const int grid = (4 * N + 63) / 64;
    hipLaunchKernelGGL(merge_sum_kernel, dim3(grid), dim3(kMergeThreads), 0, stream, part, N,
                       list_idx, list_s, list_n, u_in, u_upd, diag, ap, counter);
    return hipGetLastError();
}

hipError_t launch_weights(const float* S, int K, float lambda, float* w, mppi_diag* diag, int lanes,
                          hipStream_t stream)
{
    hipLaunchKernelGGL(weights_kernel, dim3(1), dim3(kWeightsThreads), 0, stream, S, K, lambda, w,
                       diag, lanes);
    return hipGetLastError();
}

hipError_t launch_weighted_sum(const float* w, const float* du, int K, int N, int ld,
                               const float* u_in, float* u_out, const mppi_diag* diag,
                               hipStream_t stream)
{
    hipLaunchKernelGGL(weighted_sum_kernel, dim3(4 * N), dim3(kSumThreads), 0, stream, w, du, K,
                       ld, u_in, u_out, diag);
    return hipGetLastError();
}

hipError_t launch_apply_shift(const ModelParams& P, const float* x_hat, const float* u_upd,
                              float* u_nom, float* u_apply, int N, const float u_init[4],
                              float alpha, const mppi_diag* diag, hipStream_t stream)
{
    const float4 ui = make_float4(u_init[0], u_init[1], u_init[2], u_init[3]);
    hipLaunchKernelGGL(apply_shift_kernel, dim3(1), dim3(256), 0, stream, P, x_hat, u_upd, u_nom,
                       u_apply, N, ui, alpha, diag);
    return hipGetLastError();
}

hipError_t launch_plant(const ModelParams& P, const float* x, const float* u, float* x_out,
                        int steps, hipStream_t stream)
{
    hipLaunchKernelGGL(plant_kernel, dim3(1), dim3(64), 0, stream, P, x, u, x_out, steps);
    return hipGetLastError();
}

hipError_t launch_noise(const NoiseParams& np, int K, int N, float* du, int ld, hipStream_t stream)
{
    const size_t total = (size_t)K * N;
    const int block = 256;
    const int grid = (int)((total + block - 1) / block < 65536 ? (total + block - 1) / block : 65536);
    hipLaunchKernelGGL(noise_kernel, dim3(grid), dim3(block), 0, stream, np, K, N, du, ld);
    return hipGetLastError();
}

hipError_t launch_philox(int n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                         hipStream_t stream)
{
    const int block = 256;
    hipLaunchKernelGGL(philox_kernel, dim3((n + block - 1) / block), dim3(block), 0, stream, n,
                       reinterpret_cast<const uint4*>(ctr), reinterpret_cast<const uint2*>(key),
                       reinterpret_cast<uint4*>(out));
    return hipGetLastError();
}

}  // namespace mppi
