// Internal interface between the C ABI (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mppi.h"
#include "model.h"

namespace mppi {

// Arguments of one rollout launch (host side).  The kernel receives the scalar part
// by value and the read-only inputs as separate __restrict__ arguments, so that their
// wave-uniform rows are fetched with scalar loads.
struct RolloutArgs {
    ModelParams mp;
    CostParams cp;
    NoiseParams np;
    const float* x_hat;          // 17
    const float* x_ref;          // (N+1) x 13
    const mppi_obstacle* obs;    // M
    int M;
    const float* u_nom;          // N x 4
    int K, N;
    float* du;                   // [N][4][ld]
    int ld;
    float* S;                    // K
    float* states;               // [N+1][17][ld] or nullptr
    unsigned long long* obs_tests;   // obstacle-test counter or nullptr
};


// Rollout launch shape: `lanes` consecutive lanes per sample (the obstacle tests are
// divided among them), `block` threads per workgroup, obstacle loop unrolled `unroll`.
struct LaunchConfig {
    int block;      // 64, 128, 256
    int lanes;      // 1, 2, 4, 8
    int unroll;     // 1, 4
    int fused = 0;  // 1: single pass (per-wave partial sums), 0: stored delta_u
    int pipe = 0;   // 1: wave-specialised rollouts (block is 64 (4 + lanes))
};

bool valid_config(const LaunchConfig& c);
// What the rollout launch of a full update does after the rollouts: per-wave weight
// statistics, reduced into diag by the last workgroup (and, in the single pass, the
// per-wave partial sums and the list of contributing waves).
struct UpdateTail {
    float lambda = 1.0f;
    WaveStat* stat = nullptr;          // [W]; nullptr: rollouts only (stage call)
    unsigned int* counter = nullptr;   // arrival counter, 0 between launches
    mppi_diag* diag = nullptr;
    float* part = nullptr;             // single pass: [W][4 N]
    unsigned int* rho_run = nullptr;   // single pass: running minimum, +inf between launches
    int* list_idx = nullptr;           // single pass: contributing waves [W]
    float* list_s = nullptr;           //   and their factors exp(-(rho_w - rho) / lambda)
    int* list_n = nullptr;
    float* u_copy = nullptr;           // stored form: the first workgroup copies u_nom [4 N] here
};

// Apply and advance, done by the last workgroup of the weighted-sum launch.
struct ApplyArgs {
    ModelParams P;
    const float* x_hat;
    float* u_nom;
    float* u_apply;
    int N;
    float4 u_init;
    float alpha;
};

// Rollouts (with tail: and the full update's weight statistics).
hipError_t launch_rollout(const RolloutArgs& a, const LaunchConfig& cfg, hipStream_t stream,
                          const UpdateTail* tail = nullptr);
// Wave-specialised rollouts for M <= kPipeMaxM: the LDS of a workgroup (160 KB on
// gfx950) holds the obstacles (32 B each, plus padding) and about 100 KB of hand-over
// buffers (pipe_lds_bytes).
constexpr int kPipeMaxM = 1536;
hipError_t launch_rollout_pipe(const RolloutArgs& a, const LaunchConfig& cfg, hipStream_t stream,
                               const UpdateTail* tail = nullptr);
// Waves of a rollout launch of this shape (one statistics record each).
int rollout_waves(int K, const LaunchConfig& c);   // not for pipe shapes
hipError_t launch_rollout_fused(const RolloutArgs& a, const LaunchConfig& c, const UpdateTail& tail,
                                hipStream_t stream);
// The stored form's weighted sum with the apply and advance, one launch; u_src is the
// copy of the warm start the rollout launch made (UpdateTail::u_copy).
hipError_t launch_update_sum(const float* S, const float* du, int K, int N, int ld, float lambda,
                             const float* u_src, const WaveStat* stat, int W, int lanes,
                             mppi_diag* diag, const ApplyArgs& ap, hipStream_t stream);
hipError_t launch_merge_sum(const float* part, int N, const int* list_idx, const float* list_s,
                            const int* list_n, const float* u_in, float* u_upd,
                            const mppi_diag* diag, const ApplyArgs& ap, unsigned int* counter,
                            hipStream_t stream);
hipError_t launch_weights(const float* S, int K, float lambda, float* w, mppi_diag* diag, int lanes,
                          hipStream_t stream);
hipError_t launch_weighted_sum(const float* w, const float* du, int K, int N, int ld,
                               const float* u_in, float* u_out, const mppi_diag* diag,
                               hipStream_t stream);
hipError_t launch_apply_shift(const ModelParams& P, const float* x_hat, const float* u_upd,
                              float* u_nom, float* u_apply, int N, const float u_init[4],
                              float alpha, const mppi_diag* diag, hipStream_t stream);
hipError_t launch_plant(const ModelParams& P, const float* x, const float* u, float* x_out,
                        int steps, hipStream_t stream);
hipError_t launch_noise(const NoiseParams& np, int K, int N, float* du, int ld, hipStream_t stream);
hipError_t launch_philox(int n, const uint32_t* ctr, const uint32_t* key, uint32_t* out,
                         hipStream_t stream);

}  // namespace mppi
