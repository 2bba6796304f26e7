// The library context (opaque mppi_ctx of the C ABI) and host helpers shared by the
// one-instance API (api.hip) and the batch API (batch_api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mppi.h"
#include "batch.h"
#include "kernels.h"

namespace mppi {

// Device arena and host staging of the batched path.
struct BatchState {
    int n_cap = 0, M_cap = 0;
    size_t du_cap = 0, k_cap = 0, u_cap = 0, items_cap = 0;   // floats / items
    size_t plan_bytes = 0;
    void* plan_dev = nullptr;        // BatchHeader | InstanceDesc[n_cap] | WorkItem[items_cap]
    void* plan_host = nullptr;       // pinned staging of the same layout
    mppi_diag* diags = nullptr;      // [n_cap], used when a request passes no diag
    float* du = nullptr;
    float* S = nullptr;
    WaveStat* stat = nullptr;        // [stat_cap] weight statistics of the rollout waves
    size_t stat_cap = 0;
    float* u_upd = nullptr;
    hipEvent_t staged = nullptr;     // the last H2D copy out of plan_host has completed
    bool staged_pending = false;
    BatchLaunch cfg{256, 0, 1, 8};   // lanes by occupancy, plain obstacle loop, 8 per CU
    bool use_graph = true;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::tuple<int, int, int, int, int, int> graph_key{};   // cfg + lds + n_cap
};

}  // namespace mppi

struct mppi_ctx {
    int device = 0;
    int cu_count = 0;
    int K_cap = 0, N_cap = 0, M_cap = 0, ld = 0;
    float* du = nullptr;        // [N_cap][4][ld]
    float* S = nullptr;         // [ld]
    float* w = nullptr;         // [ld]
    float* u_upd = nullptr;     // [N_cap][4]
    mppi_diag* diag = nullptr;  // 1
    // weight statistics per rollout wave; single pass: partial sums [W_cap][4 N]
    int W_cap = 0;
    mppi::WaveStat* wstat = nullptr;
    float* part = nullptr;
    unsigned int* rho_run = nullptr;   // running minimum of the waves (+inf between updates)
    int* list_idx = nullptr;           // waves contributing partial sums [W_cap]
    float* list_s = nullptr;           //   and their factors
    int* list_n = nullptr;
    // arrival counters of the rollout and weighted-sum launches (0 between launches)
    unsigned int* counters = nullptr;
    float* u_tmp = nullptr;            // autotuning's advanced sequence and applied control
    std::map<std::tuple<int, int, int>, mppi::LaunchConfig> tuned;   // size class -> shape
    std::string last_error;
    // profiling: 5 events per update bracket rollout, weights, sum, apply
    bool profiling = false;
    std::vector<hipEvent_t> pool, pending, batch_pending;   // 5 per update, 3 per batch
    mppi_profile acc{};
    unsigned long long* obs_tests = nullptr;   // device counter while profiling
    mppi::BatchState batch;
    // device address of mppi_update_static's static scratch on this context's device
    // (taken by mppi_create), or nullptr with the reason
    void* static_scratch = nullptr;
    std::string static_scratch_error;
};

namespace mppi {

mppi_status fail(mppi_ctx* ctx, mppi_status s, const std::string& msg);
mppi_status hip_fail(mppi_ctx* ctx, hipError_t e, const char* where);
mppi_status check_vehicle(const mppi_vehicle* v);
mppi_status check_cost(const mppi_cost* c);
mppi_status check_solve(const mppi_solve* s);
ModelParams model_params(const mppi_vehicle& v, float dt);
CostParams cost_params(const mppi_cost& c);
// Fraction of a prediction step the warm start advances per update (Sec. IV-B).
float advance_fraction(const mppi_solve& s);
// Delay prediction (Sec. IV-E): number of equal steps of at most dt covering delay
// (-1 if invalid or above kPredictMaxSteps), and the model parameters of those steps.
constexpr int kPredictMaxSteps = 4096;
int predict_steps(float dt, float delay);
ModelParams predict_params(const mppi_vehicle& v, float dt, float delay, int steps);
NoiseParams noise_params(const mppi_solve& s);
void free_batch(mppi_ctx* ctx);
mppi_status batch_reserve_raw(mppi_ctx* ctx, int n, size_t du, size_t k, size_t u, size_t items,
                              int M);
hipEvent_t take_event(mppi_ctx* ctx);

}  // namespace mppi

#define HIP_TRY(ctx, expr)                                             \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return mppi::hip_fail(ctx, e_, #expr);   \
    } while (0)
