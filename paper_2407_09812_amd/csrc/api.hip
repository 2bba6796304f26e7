// C ABI of libmppi (declared in include/mppi.h): argument validation, device
// scratch, launch sequencing of one MPPI update, profiling and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "context.h"
#include "kernels.h"

using namespace mppi;

namespace mppi {

mppi_status fail(mppi_ctx* ctx, mppi_status s, const std::string& msg)
{
    if (ctx) ctx->last_error = msg;
    return s;
}

mppi_status hip_fail(mppi_ctx* ctx, hipError_t e, const char* where)
{
    return fail(ctx, MPPI_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool finite_all(const float* v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

mppi_status check_vehicle(const mppi_vehicle* v)
{
    if (!v) return MPPI_E_INVALID_ARG;
    const float vals[13] = {v->mass, v->J[0], v->J[1], v->J[2], v->arm_l, v->c_tf, v->g,
                            v->T_min, v->T_max, v->tau_m, v->k_rate, v->w_xy_max, v->w_z_max};
    if (!finite_all(vals, 13)) return MPPI_E_NONFINITE_INPUT;
    if (!(v->mass > 0) || !(v->J[0] > 0) || !(v->J[1] > 0) || !(v->J[2] > 0)) return MPPI_E_INVALID_ARG;
    if (!(v->arm_l > 0) || !(v->c_tf > 0) || v->T_min > v->T_max) return MPPI_E_INVALID_ARG;
    if (v->tau_m < 0 || v->k_rate < 0 || v->w_xy_max < 0 || v->w_z_max < 0) return MPPI_E_INVALID_ARG;
    return MPPI_OK;
}

mppi_status check_cost(const mppi_cost* c)
{
    if (!c) return MPPI_E_INVALID_ARG;
    const float vals[15] = {c->c_p, c->c_v, c->c_q, c->c_w, c->R[0], c->R[1], c->R[2], c->R[3],
                            c->R_d[0], c->R_d[1], c->R_d[2], c->R_d[3], c->obs_margin, c->obs_w,
                            c->obs_collision};
    if (!finite_all(vals, 15)) return MPPI_E_NONFINITE_INPUT;
    for (float x : vals)
        if (x < 0) return MPPI_E_INVALID_ARG;
    return MPPI_OK;
}

mppi_status check_solve(const mppi_solve* s)
{
    if (!s) return MPPI_E_INVALID_ARG;
    if (s->K < 1 || s->N < 1 || s->N > MPPI_N_MAX) return MPPI_E_INVALID_ARG;
    const float vals[10] = {s->dt, s->lambda, s->sigma[0], s->sigma[1], s->sigma[2], s->sigma[3],
                            s->u_init[0], s->u_init[1], s->u_init[2], s->u_init[3]};
    if (!finite_all(vals, 10)) return MPPI_E_NONFINITE_INPUT;
    if (!std::isfinite(s->dt_ctrl)) return MPPI_E_NONFINITE_INPUT;
    if (!(s->dt > 0) || !(s->lambda > 0)) return MPPI_E_INVALID_ARG;
    if (s->dt_ctrl < 0 || s->dt_ctrl > s->dt) return MPPI_E_INVALID_ARG;
    for (int d = 0; d < 4; ++d)
        if (s->sigma[d] < 0) return MPPI_E_INVALID_ARG;
    return MPPI_OK;
}

float advance_fraction(const mppi_solve& s)
{
    return s.dt_ctrl > 0 ? (float)((double)s.dt_ctrl / (double)s.dt) : 1.0f;
}

ModelParams model_params(const mppi_vehicle& v, float dt)
{
    ModelParams P{};
    const double s = (double)v.arm_l / std::sqrt(2.0);
    P.m_inv = (float)(1.0 / v.mass);
    P.g = v.g;
    for (int i = 0; i < 3; ++i) {
        P.J[i] = v.J[i];
        P.J_inv[i] = (float)(1.0 / v.J[i]);
    }
    P.G[0] = v.J[2] - v.J[1];
    P.G[1] = v.J[0] - v.J[2];
    P.G[2] = v.J[1] - v.J[0];
    P.s = (float)s;
    P.c = v.c_tf;
    P.inv_4s = (float)(1.0 / (4.0 * s));
    P.inv_4c = (float)(1.0 / (4.0 * v.c_tf));
    P.T_min = v.T_min;
    P.T_max = v.T_max;
    P.lag = v.tau_m > 0.0f ? 1 : 0;
    P.tau_inv = P.lag ? (float)(1.0 / v.tau_m) : 0.0f;
    if (P.lag) {
        const double z = (double)dt / (double)v.tau_m;
        const double c1 = 0.5 * z, c2 = c1 * (1.0 - c1), c3 = z * (1.0 - c2);
        const double c4 = z * (6.0 - 2.0 * c1 - 2.0 * c2 - c3) / 6.0;
        P.lag_c[0] = (float)c1; P.lag_c[1] = (float)c2; P.lag_c[2] = (float)c3; P.lag_c[3] = (float)c4;
    }
    P.k_w = v.k_rate > 0.0f ? v.k_rate : (float)(1.0 / dt);
    P.dt = dt;
    P.w_xy_max = v.w_xy_max;
    P.w_z_max = v.w_z_max;
    return P;
}

int predict_steps(float dt, float delay)
{
    if (!(dt > 0) || !(delay >= 0)) return -1;
    const double n = std::ceil((double)delay / (double)dt);
    return n <= kPredictMaxSteps ? (int)n : -1;
}

ModelParams predict_params(const mppi_vehicle& v, float dt, float delay, int steps)
{
    // Steps of h = delay / steps; the rate controller's gain stays that of the
    // prediction step dt (Eq. (8)).
    ModelParams P = model_params(v, steps > 0 ? (float)((double)delay / steps) : dt);
    P.k_w = v.k_rate > 0.0f ? v.k_rate : (float)(1.0 / dt);
    return P;
}

CostParams cost_params(const mppi_cost& c)
{
    CostParams C{};
    C.c_p = c.c_p; C.c_v = c.c_v; C.c_q = c.c_q; C.c_w = c.c_w;
    for (int d = 0; d < 4; ++d) { C.R[d] = c.R[d]; C.Rd[d] = c.R_d[d]; }
    C.margin = c.obs_margin; C.w_obs = c.obs_w; C.c_col = c.obs_collision;
    return C;
}

NoiseParams noise_params(const mppi_solve& s)
{
    NoiseParams np{};
    for (int d = 0; d < 4; ++d) np.sigma[d] = s.sigma[d];
    np.key0 = (uint32_t)(s.seed & 0xFFFFFFFFull);
    np.key1 = s.vehicle_id;
    np.t = s.t;
    np.seed_hi = (uint32_t)(s.seed >> 32);
    return np;
}

RolloutArgs rollout_args(const mppi_vehicle& v, const mppi_cost& c, const mppi_solve& s)
{
    RolloutArgs a{};
    a.mp = model_params(v, s.dt);
    a.cp = cost_params(c);
    a.np = noise_params(s);
    a.K = s.K;
    a.N = s.N;
    return a;
}

}  // namespace mppi

namespace {

// Device scratch of one update: the context's reserved buffers, or carved out of the
// static array of mppi_update_static (stored form only: no single-pass buffers).
struct Scratch {
    float* du;               // [N][4][ld]
    int ld;
    float* S;                // [ld]
    WaveStat* wstat;         // one record per rollout wave
    float* u_upd;            // [4 N]
    unsigned int* counters;  // single pass: two arrival counters, 0 between launches
    float* part;             // single pass: [W][4 N]
    unsigned int* rho_run;   // single pass: +inf between launches
    int* list_idx;
    float* list_s;
    int* list_n;
};

// Scratch of mppi_update_static: one array on every GPU the library runs on, held until
// the process ends.  Host code never uses the name `scratch` as an address (on the host
// it is only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device by mppi_create with that device current.
static __device__ __align__(256) unsigned char scratch[MPPI_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device

// With `device` current: the device address of its static scratch (taken on first use).
hipError_t static_scratch_address(int device, void** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The stored form's scratch carved out of the static array for (K, N) with `waves`
// rollout waves; the bytes it needs (for the capacity check) in *bytes.
Scratch carve_static(unsigned char* base, int K, int N, int waves, mppi_diag** diag, size_t* bytes)
{
    Scratch sc{};
    const int ld = (K + 63) & ~63;
    size_t off = 0;
    auto take = [&](size_t b) { unsigned char* p = base + off; off += align256(b); return p; };
    sc.ld = ld;
    sc.du = reinterpret_cast<float*>(take(sizeof(float) * 4 * (size_t)N * ld));
    sc.S = reinterpret_cast<float*>(take(sizeof(float) * (size_t)ld));
    sc.wstat = reinterpret_cast<WaveStat*>(take(sizeof(WaveStat) * (size_t)waves));
    sc.u_upd = reinterpret_cast<float*>(take(sizeof(float) * 4 * (size_t)N));
    *diag = reinterpret_cast<mppi_diag*>(take(sizeof(mppi_diag)));
    *bytes = off;
    return sc;
}

constexpr int kEventsPerUpdate = 3;   // before, between and after the two launches

void free_scratch(mppi_ctx* ctx)
{
    (void)hipFree(ctx->du); (void)hipFree(ctx->S); (void)hipFree(ctx->w);
    (void)hipFree(ctx->u_upd); (void)hipFree(ctx->diag);
    (void)hipFree(ctx->wstat); (void)hipFree(ctx->part); (void)hipFree(ctx->rho_run);
    (void)hipFree(ctx->counters); (void)hipFree(ctx->list_idx); (void)hipFree(ctx->list_s);
    (void)hipFree(ctx->list_n); (void)hipFree(ctx->u_tmp);
    ctx->rho_run = ctx->counters = nullptr;
    ctx->list_idx = ctx->list_n = nullptr;
    ctx->list_s = ctx->u_tmp = nullptr;
    ctx->du = ctx->S = ctx->w = ctx->u_upd = ctx->part = nullptr;
    ctx->diag = nullptr;
    ctx->wstat = nullptr;
    ctx->W_cap = 0;
    ctx->K_cap = ctx->N_cap = ctx->M_cap = ctx->ld = 0;
}

constexpr unsigned int kInfBits = 0x7f800000u;

int ceil_log2(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

std::tuple<int, int, int> size_class(int K, int N, int M)
{
    return {ceil_log2(K), ceil_log2(N), M == 0 ? -1 : ceil_log2(M)};
}

// One wave per SIMD (1024 on the chip) is the target for a lone instance; lanes
// beyond one per sample only pay off when there are obstacles to divide.
// Without a tuned entry: the wave-specialised rollouts (the fastest form for every
// single instance measured, see the autotuner's choices), with more obstacle lanes for
// longer obstacle lists; past their obstacle limit the one-wave kernel, aiming at one
// wave per SIMD.
LaunchConfig heuristic_config(int K, int M)
{
    LaunchConfig c;
    if (M <= kPipeMaxM) {
        c.block = 64;
        c.lanes = M < 16 ? 1 : M < 64 ? 2 : 4;     // 4: the obstacle waves cull by chunk
        c.unroll = 1;
        c.pipe = 1;
        return c;
    }
    const int waves = (K + 63) / 64;
    int lanes = 1;
    while (lanes < 8 && waves * lanes * 2 <= 1024 && M >= 8 * lanes) lanes *= 2;
    c.lanes = lanes;
    c.block = (waves * lanes >= 1024) ? 256 : 64;
    c.unroll = M >= 16 ? 4 : 1;
    return c;
}

LaunchConfig config_for(const mppi_ctx* ctx, int K, int N, int M)
{
    auto it = ctx->tuned.find(size_class(K, N, M));
    if (it == ctx->tuned.end()) return heuristic_config(K, M);
    LaunchConfig c = it->second;
    // A size class spans M up to the next power of two, which for 1025..2048 crosses
    // the pipe's obstacle limit: a pipe shape stored at M <= kPipeMaxM runs past it as
    // the one-wave kernel with the same lanes, unroll and variant.
    if (c.pipe && M > kPipeMaxM) {
        c.pipe = 0;
        c.block = heuristic_config(K, M).block;
    }
    return c;
}

}  // namespace

hipEvent_t mppi::take_event(mppi_ctx* ctx)
{
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

namespace {

Scratch ctx_scratch(mppi_ctx* ctx)
{
    return Scratch{ctx->du, ctx->ld, ctx->S, ctx->wstat, ctx->u_upd, ctx->counters, ctx->part,
                   ctx->rho_run, ctx->list_idx, ctx->list_s, ctx->list_n};
}

// Waves of the rollout launch of this shape: one weight-statistics record each.
int update_waves(int K, const LaunchConfig& cfg)
{
    return cfg.pipe ? (K + 63) / 64 * cfg.lanes : rollout_waves(K, cfg);
}

// The full update in two launches on stream s: the rollouts with the weight
// statistics (reduced by their last workgroup into dg), then the weighted sum, which
// applies and advances as `ap` says: over the stored delta_u, one workgroup per step
// (the rollout launch copies the warm start into sc.u_upd for it), or, with
// cfg.fused, over the per-wave partial sums into sc.u_upd, whose last workgroup
// applies.  mark(1) is called between the two launches.
template <typename Mark>
hipError_t update_core(const Scratch& sc, RolloutArgs a, const LaunchConfig& cfg, float lambda,
                       const float* u_in, const ApplyArgs& ap, mppi_diag* dg, hipStream_t s,
                       Mark mark)
{
    a.du = sc.du;
    a.ld = sc.ld;
    a.S = sc.S;
    UpdateTail tail;
    tail.lambda = lambda;
    tail.stat = sc.wstat;
    tail.counter = sc.counters;
    tail.diag = dg;
    hipError_t e;
    if (cfg.fused) {
        tail.part = sc.part;
        tail.rho_run = sc.rho_run;
        tail.list_idx = sc.list_idx;
        tail.list_s = sc.list_s;
        tail.list_n = sc.list_n;
        e = cfg.pipe ? launch_rollout_pipe(a, cfg, s, &tail) : launch_rollout_fused(a, cfg, tail, s);
        if (e == hipSuccess) e = mark(1);
        if (e == hipSuccess)
            e = launch_merge_sum(sc.part, a.N, sc.list_idx, sc.list_s, sc.list_n, u_in, sc.u_upd, dg,
                                 ap, sc.counters + 1, s);
    } else {
        tail.u_copy = sc.u_upd;
        e = cfg.pipe ? launch_rollout_pipe(a, cfg, s, &tail) : launch_rollout(a, cfg, s, &tail);
        if (e == hipSuccess) e = mark(1);
        if (e == hipSuccess)
            e = launch_update_sum(sc.S, sc.du, a.K, a.N, sc.ld, lambda, sc.u_upd, sc.wstat,
                                  update_waves(a.K, cfg), cfg.lanes, dg, ap, s);
    }
    return e;
}

ApplyArgs apply_args(const ModelParams& P, const float* x_hat, float* u_nom, float* u_apply, int N,
                     const mppi_solve& solve)
{
    ApplyArgs ap;
    ap.P = P;
    ap.x_hat = x_hat;
    ap.u_nom = u_nom;
    ap.u_apply = u_apply;
    ap.N = N;
    ap.u_init = make_float4(solve.u_init[0], solve.u_init[1], solve.u_init[2], solve.u_init[3]);
    ap.alpha = advance_fraction(solve);
    return ap;
}

}  // namespace

extern "C" {

const char* mppi_status_str(mppi_status s)
{
    switch (s) {
    case MPPI_OK: return "MPPI_OK";
    case MPPI_E_INVALID_ARG: return "MPPI_E_INVALID_ARG";
    case MPPI_E_NONFINITE_INPUT: return "MPPI_E_NONFINITE_INPUT";
    case MPPI_E_ALL_NONFINITE: return "MPPI_E_ALL_NONFINITE";
    case MPPI_E_BUDGET: return "MPPI_E_BUDGET";
    case MPPI_E_OOM: return "MPPI_E_OOM";
    case MPPI_E_HIP: return "MPPI_E_HIP";
    case MPPI_E_PENDING: return "MPPI_E_PENDING";
    case MPPI_E_CAPACITY: return "MPPI_E_CAPACITY";
    default: return "MPPI_E_UNKNOWN";
    }
}

const char* mppi_last_error(const mppi_ctx* ctx)
{
    return ctx ? ctx->last_error.c_str() : "null context";
}

mppi_status mppi_validate(const mppi_vehicle* veh, const mppi_cost* cost, const mppi_solve* solve,
                          int32_t M)
{
    mppi_status s;
    if ((s = check_vehicle(veh)) != MPPI_OK) return s;
    if ((s = check_cost(cost)) != MPPI_OK) return s;
    if ((s = check_solve(solve)) != MPPI_OK) return s;
    if (M < 0 || M > MPPI_M_MAX) return MPPI_E_INVALID_ARG;
    return MPPI_OK;
}

mppi_status mppi_create(int device, mppi_ctx** out)
{
    if (!out) return MPPI_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MPPI_E_INVALID_ARG;
    mppi_ctx* ctx = new (std::nothrow) mppi_ctx();
    if (!ctx) return MPPI_E_OOM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess) {
        delete ctx;
        return MPPI_E_HIP;
    }
    // the static scratch of mppi_update_static on this device (once per device); a
    // failure is kept for that entry point to report
    void* p = nullptr;
    const hipError_t e = static_scratch_address(device, &p);
    ctx->static_scratch = e == hipSuccess ? p : nullptr;
    if (e != hipSuccess) {
        ctx->static_scratch_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        (void)hipGetLastError();
    }
    *out = ctx;
    return MPPI_OK;
}

mppi_status mppi_destroy(mppi_ctx* ctx)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_scratch(ctx);
    free_batch(ctx);
    (void)hipFree(ctx->obs_tests);
    for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->pending) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->batch_pending) (void)hipEventDestroy(e);
    delete ctx;
    return MPPI_OK;
}

mppi_status mppi_reserve(mppi_ctx* ctx, int32_t K, int32_t N, int32_t M)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    if (K < 1 || N < 1 || N > MPPI_N_MAX || M < 0 || M > MPPI_M_MAX)
        return fail(ctx, MPPI_E_INVALID_ARG, "reserve: size out of range");
    if (K <= ctx->K_cap && N <= ctx->N_cap) {
        if (M > ctx->M_cap) ctx->M_cap = M;
        return MPPI_OK;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    const int Kc = K > ctx->K_cap ? K : ctx->K_cap;
    const int Nc = N > ctx->N_cap ? N : ctx->N_cap;
    const int Mc = M > ctx->M_cap ? M : ctx->M_cap;
    free_scratch(ctx);
    const int ld = (Kc + 63) & ~63;   // rows start on 256-byte boundaries
    const size_t du_bytes = sizeof(float) * (size_t)Nc * 4 * ld;
    // the most waves a rollout launch has: 8 lanes per sample, whole workgroups of 256
    const int W = (int)(((size_t)ld * 8 + 255) / 256 * 4);
    if (hipMalloc(&ctx->du, du_bytes) != hipSuccess || hipMalloc(&ctx->S, sizeof(float) * ld) != hipSuccess ||
        hipMalloc(&ctx->w, sizeof(float) * ld) != hipSuccess ||
        hipMalloc(&ctx->u_upd, sizeof(float) * 4 * (size_t)Nc) != hipSuccess ||
        hipMalloc(&ctx->diag, sizeof(mppi_diag)) != hipSuccess ||
        hipMalloc(&ctx->wstat, sizeof(WaveStat) * (size_t)W) != hipSuccess ||
        hipMalloc(&ctx->part, sizeof(float) * 4 * (size_t)Nc * W) != hipSuccess ||
        hipMalloc(&ctx->rho_run, sizeof(unsigned int)) != hipSuccess ||
        hipMemcpy(ctx->rho_run, &kInfBits, sizeof(unsigned int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&ctx->counters, 2 * sizeof(unsigned int)) != hipSuccess ||
        hipMemset(ctx->counters, 0, 2 * sizeof(unsigned int)) != hipSuccess ||
        hipMalloc(&ctx->list_idx, sizeof(int) * (size_t)W) != hipSuccess ||
        hipMalloc(&ctx->list_s, sizeof(float) * (size_t)W) != hipSuccess ||
        hipMalloc(&ctx->list_n, sizeof(int)) != hipSuccess ||
        hipMalloc(&ctx->u_tmp, sizeof(float) * (4 * (size_t)Nc + 8)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_scratch(ctx);
        (void)hipGetLastError();
        return fail(ctx, MPPI_E_OOM, "reserve: device allocation failed");
    }
    ctx->K_cap = Kc; ctx->N_cap = Nc; ctx->M_cap = Mc; ctx->ld = ld; ctx->W_cap = W;
    return MPPI_OK;
}

mppi_status mppi_update(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh, const mppi_cost* cost,
                        const mppi_solve* solve, const float* x_hat, const float* x_ref,
                        const mppi_obstacle* obs, int32_t M, float* u_nom, float* u_apply,
                        mppi_diag* diag)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = mppi_validate(veh, cost, solve, M);
    if (st != MPPI_OK) return fail(ctx, st, "update: invalid parameters");
    if (!x_hat || !x_ref || !u_nom || !u_apply || (M > 0 && !obs))
        return fail(ctx, MPPI_E_INVALID_ARG, "update: null device pointer");
    if (solve->K > ctx->K_cap || solve->N > ctx->N_cap || M > ctx->M_cap)
        return fail(ctx, MPPI_E_CAPACITY, "update: request exceeds reserved scratch");
    hipStream_t s = (hipStream_t)stream;
    mppi_diag* dg = diag ? diag : ctx->diag;

    RolloutArgs a = rollout_args(*veh, *cost, *solve);
    a.x_hat = x_hat; a.x_ref = x_ref; a.obs = obs; a.M = M; a.u_nom = u_nom;
    a.du = ctx->du; a.ld = ctx->ld; a.S = ctx->S; a.states = nullptr;
    a.obs_tests = ctx->profiling ? ctx->obs_tests : nullptr;

    hipEvent_t ev[kEventsPerUpdate] = {};
    if (ctx->profiling)
        for (int i = 0; i < kEventsPerUpdate; ++i)
            if (!(ev[i] = take_event(ctx))) return fail(ctx, MPPI_E_HIP, "update: event creation");
    auto mark = [&](int i) -> hipError_t {
        return ctx->profiling ? hipEventRecord(ev[i], s) : hipSuccess;
    };

    const LaunchConfig cfg = config_for(ctx, solve->K, solve->N, M);
    const ApplyArgs ap = apply_args(a.mp, x_hat, u_nom, u_apply, solve->N, *solve);
    HIP_TRY(ctx, mark(0));
    HIP_TRY(ctx, update_core(ctx_scratch(ctx), a, cfg, solve->lambda, u_nom, ap, dg, s, mark));
    HIP_TRY(ctx, mark(2));
    if (ctx->profiling)
        for (int i = 0; i < kEventsPerUpdate; ++i) ctx->pending.push_back(ev[i]);
    return MPPI_OK;
}

mppi_status mppi_update_static(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh,
                               const mppi_cost* cost, const mppi_solve* solve, const float* x_hat,
                               const float* x_ref, const mppi_obstacle* obs, int32_t M,
                               float* u_nom, float* u_apply, mppi_diag* diag)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = mppi_validate(veh, cost, solve, M);
    if (st != MPPI_OK) return fail(ctx, st, "update_static: invalid parameters");
    if (!x_hat || !x_ref || !u_nom || !u_apply || (M > 0 && !obs))
        return fail(ctx, MPPI_E_INVALID_ARG, "update_static: null device pointer");
    if (!ctx->static_scratch)
        return fail(ctx, MPPI_E_HIP, "update_static: " + ctx->static_scratch_error);
    LaunchConfig cfg = config_for(ctx, solve->K, solve->N, M);
    cfg.fused = 0;                                    // the stored form only
    mppi_diag* own_diag = nullptr;
    size_t need = 0;
    const Scratch sc = carve_static(static_cast<unsigned char*>(ctx->static_scratch), solve->K,
                                    solve->N, update_waves(solve->K, cfg), &own_diag, &need);
    if (need > (size_t)MPPI_STATIC_SCRATCH_BYTES)
        return fail(ctx, MPPI_E_CAPACITY, "update_static: " + std::to_string(need) +
                                              " bytes of scratch needed, the static array holds " +
                                              std::to_string((size_t)MPPI_STATIC_SCRATCH_BYTES));
    RolloutArgs a = rollout_args(*veh, *cost, *solve);
    a.x_hat = x_hat; a.x_ref = x_ref; a.obs = obs; a.M = M; a.u_nom = u_nom;
    a.states = nullptr;
    a.obs_tests = nullptr;
    const ApplyArgs ap = apply_args(a.mp, x_hat, u_nom, u_apply, solve->N, *solve);
    HIP_TRY(ctx, update_core(sc, a, cfg, solve->lambda, u_nom, ap, diag ? diag : own_diag,
                             (hipStream_t)stream, [](int) { return hipSuccess; }));
    return MPPI_OK;
}

mppi_status mppi_rollout(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh, const mppi_cost* cost,
                         const mppi_solve* solve, const float* x_hat, const float* x_ref,
                         const mppi_obstacle* obs, int32_t M, const float* u_nom, float* du,
                         int32_t ld, float* S, float* states)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = mppi_validate(veh, cost, solve, M);
    if (st != MPPI_OK) return fail(ctx, st, "rollout: invalid parameters");
    if (!x_hat || !x_ref || !u_nom || !du || !S || (M > 0 && !obs) || ld < solve->K)
        return fail(ctx, MPPI_E_INVALID_ARG, "rollout: null pointer or ld < K");
    RolloutArgs a = rollout_args(*veh, *cost, *solve);
    a.x_hat = x_hat; a.x_ref = x_ref; a.obs = obs; a.M = M; a.u_nom = u_nom;
    a.du = du; a.ld = ld; a.S = S; a.states = states;
    const LaunchConfig cfg = config_for(ctx, solve->K, solve->N, M);
    if (cfg.pipe && !states && M <= kPipeMaxM)
        HIP_TRY(ctx, launch_rollout_pipe(a, LaunchConfig{cfg.block, cfg.lanes, cfg.unroll, 0, 1},
                                         (hipStream_t)stream));
    else
        HIP_TRY(ctx, launch_rollout(a, LaunchConfig{cfg.block, cfg.lanes, cfg.unroll, 0, 0},
                                    (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_get_config(const mppi_ctx* ctx, int32_t K, int32_t N, int32_t M,
                            mppi_launch_config* out)
{
    if (!ctx || !out || K < 1 || N < 1 || M < 0) return MPPI_E_INVALID_ARG;
    const LaunchConfig c = config_for(ctx, K, N, M);
    out->block = c.block; out->lanes = c.lanes; out->unroll = c.unroll; out->fused = c.fused;
    out->pipe = c.pipe;
    return MPPI_OK;
}

mppi_status mppi_set_config(mppi_ctx* ctx, int32_t K, int32_t N, int32_t M,
                            const mppi_launch_config* cfg)
{
    if (!ctx || !cfg || K < 1 || N < 1 || M < 0) return MPPI_E_INVALID_ARG;
    const LaunchConfig c{cfg->block, cfg->lanes, cfg->unroll, cfg->fused, cfg->pipe};
    if (!valid_config(c) || (c.pipe && M > kPipeMaxM))
        return fail(ctx, MPPI_E_INVALID_ARG, "set_config: invalid shape");
    ctx->tuned[size_class(K, N, M)] = c;
    return MPPI_OK;
}

mppi_status mppi_autotune(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh, const mppi_cost* cost,
                          const mppi_solve* solve, const float* x_hat, const float* x_ref,
                          const mppi_obstacle* obs, int32_t M, const float* u_nom, int32_t reps,
                          mppi_launch_config* best)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = mppi_validate(veh, cost, solve, M);
    if (st != MPPI_OK) return fail(ctx, st, "autotune: invalid parameters");
    if (!x_hat || !x_ref || !u_nom || (M > 0 && !obs) || reps < 1)
        return fail(ctx, MPPI_E_INVALID_ARG, "autotune: bad argument");
    if (solve->K > ctx->K_cap || solve->N > ctx->N_cap)
        return fail(ctx, MPPI_E_CAPACITY, "autotune: request exceeds reserved scratch");
    hipStream_t s = (hipStream_t)stream;
    RolloutArgs a = rollout_args(*veh, *cost, *solve);
    a.x_hat = x_hat; a.x_ref = x_ref; a.obs = obs; a.M = M; a.u_nom = u_nom;
    a.du = ctx->du; a.ld = ctx->ld; a.S = ctx->S; a.states = nullptr;
    hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx);
    if (!e0 || !e1) return fail(ctx, MPPI_E_HIP, "autotune: event creation");
    // what is timed: the whole update, both variants, writing its outputs to scratch
    const ApplyArgs ap = apply_args(a.mp, x_hat, ctx->u_tmp, ctx->u_tmp + 4 * (size_t)solve->N,
                                    solve->N, *solve);
    auto core = [&](const LaunchConfig& c) -> hipError_t {
        return update_core(ctx_scratch(ctx), a, c, solve->lambda, u_nom, ap, ctx->diag, s,
                           [](int) { return hipSuccess; });
    };
    std::vector<LaunchConfig> cands;
    for (int variant : {0, 1, 2, 3})   // one-wave stored / single pass, wave-specialised ditto
        for (int lanes : {1, 2, 4, 8}) {
            const bool pipe = variant >= 2, fused = variant & 1;
            if (lanes > 1 && M < 2 * lanes) continue;        // nothing to divide
            if (pipe && M > kPipeMaxM) continue;
            for (int block : {64, 128, 256})
                for (int unroll : {1, 4}) {
                    if (unroll > 1 && M < 8) continue;
                    if (pipe && block != 64) continue;   // its workgroup is 64 (4 + lanes)
                    cands.push_back(LaunchConfig{block, lanes, unroll, fused ? 1 : 0, pipe ? 1 : 0});
                }
        }
    LaunchConfig best_c{};
    float best_ms = 1e30f;
    mppi_status result = MPPI_OK;
    for (const LaunchConfig& c : cands) {
        hipError_t e = core(c);                           // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = core(c);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { result = hip_fail(ctx, e, "autotune"); break; }
        if (ms < best_ms) { best_ms = ms; best_c = c; }
    }
    ctx->pool.push_back(e0);
    ctx->pool.push_back(e1);
    if (result != MPPI_OK) return result;
    ctx->tuned[size_class(solve->K, solve->N, M)] = best_c;
    if (best) {
        best->block = best_c.block; best->lanes = best_c.lanes; best->unroll = best_c.unroll;
        best->fused = best_c.fused; best->pipe = best_c.pipe;
    }
    return MPPI_OK;
}

mppi_status mppi_weights(mppi_ctx* ctx, void* stream, int32_t K, const float* S, float lambda,
                         float* w, mppi_diag* diag)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    if (K < 1 || !S || !w || !diag || !std::isfinite(lambda) || !(lambda > 0))
        return fail(ctx, MPPI_E_INVALID_ARG, "weights: bad argument");
    HIP_TRY(ctx, launch_weights(S, K, lambda, w, diag, 0, (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_weighted_sum(mppi_ctx* ctx, void* stream, int32_t K, int32_t N, const float* w,
                              const float* du, int32_t ld, const float* u_in, float* u_out,
                              const mppi_diag* diag)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    if (K < 1 || N < 1 || N > MPPI_N_MAX || ld < K || !w || !du || !u_in || !u_out)
        return fail(ctx, MPPI_E_INVALID_ARG, "weighted_sum: bad argument");
    if ((ld & 3) == 0 && ((reinterpret_cast<uintptr_t>(du) | reinterpret_cast<uintptr_t>(w)) & 15))
        return fail(ctx, MPPI_E_INVALID_ARG, "weighted_sum: du and w must be 16-byte aligned");
    HIP_TRY(ctx, launch_weighted_sum(w, du, K, N, ld, u_in, u_out, diag, (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_apply_shift(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh,
                             const mppi_solve* solve, const float* x_hat, const float* u_upd,
                             float* u_nom, float* u_apply)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st;
    if ((st = check_vehicle(veh)) != MPPI_OK || (st = check_solve(solve)) != MPPI_OK)
        return fail(ctx, st, "apply_shift: invalid parameters");
    if (!x_hat || !u_upd || !u_nom || !u_apply || u_upd == u_nom)
        return fail(ctx, MPPI_E_INVALID_ARG, "apply_shift: null or aliased pointer");
    HIP_TRY(ctx, launch_apply_shift(model_params(*veh, solve->dt), x_hat, u_upd, u_nom, u_apply,
                                    solve->N, solve->u_init, advance_fraction(*solve), nullptr,
                                    (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_noise(mppi_ctx* ctx, void* stream, const mppi_solve* solve, float* du, int32_t ld)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = check_solve(solve);
    if (st != MPPI_OK) return fail(ctx, st, "noise: invalid parameters");
    if (!du || ld < solve->K) return fail(ctx, MPPI_E_INVALID_ARG, "noise: bad argument");
    HIP_TRY(ctx, launch_noise(noise_params(*solve), solve->K, solve->N, du, ld, (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_philox(mppi_ctx* ctx, void* stream, int32_t n, const uint32_t* ctr,
                        const uint32_t* key, uint32_t* out)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    if (n < 0 || (n > 0 && (!ctr || !key || !out)))
        return fail(ctx, MPPI_E_INVALID_ARG, "philox: bad argument");
    if (((reinterpret_cast<uintptr_t>(ctr) | reinterpret_cast<uintptr_t>(out)) & 15) ||
        (reinterpret_cast<uintptr_t>(key) & 7))
        return fail(ctx, MPPI_E_INVALID_ARG, "philox: misaligned buffer");
    if (n == 0) return MPPI_OK;
    HIP_TRY(ctx, launch_philox(n, ctr, key, out, (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_plant_step(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh, float dt,
                            const float* x, const float* u, float* x_out)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = check_vehicle(veh);
    if (st != MPPI_OK) return fail(ctx, st, "plant_step: invalid vehicle");
    if (!std::isfinite(dt) || !(dt > 0) || !x || !u || !x_out)
        return fail(ctx, MPPI_E_INVALID_ARG, "plant_step: bad argument");
    HIP_TRY(ctx, launch_plant(model_params(*veh, dt), x, u, x_out, 1, (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_predict(mppi_ctx* ctx, void* stream, const mppi_vehicle* veh, float dt,
                         float delay, const float* x_hat, const float* u_hold, float* x_out)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    mppi_status st = check_vehicle(veh);
    if (st != MPPI_OK) return fail(ctx, st, "predict: invalid vehicle");
    if (!std::isfinite(dt) || !std::isfinite(delay))
        return fail(ctx, MPPI_E_NONFINITE_INPUT, "predict: non-finite dt or delay");
    const int steps = predict_steps(dt, delay);
    if (!(dt > 0) || steps < 0 || !x_hat || !u_hold || !x_out)
        return fail(ctx, MPPI_E_INVALID_ARG, "predict: bad argument");
    HIP_TRY(ctx, launch_plant(predict_params(*veh, dt, delay, steps), x_hat, u_hold, x_out, steps,
                              (hipStream_t)stream));
    return MPPI_OK;
}

mppi_status mppi_device_address(const void* host_ptr, void** dev_ptr)
{
    if (!host_ptr || !dev_ptr) return MPPI_E_INVALID_ARG;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, const_cast<void*>(host_ptr), 0) != hipSuccess || !d) {
        (void)hipGetLastError();           // leave no error behind for the next call
        return MPPI_E_INVALID_ARG;
    }
    *dev_ptr = d;
    return MPPI_OK;
}

mppi_status mppi_profile_enable(mppi_ctx* ctx, int32_t on)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    if (on && !ctx->obs_tests) {
        HIP_TRY(ctx, hipMalloc(&ctx->obs_tests, sizeof(unsigned long long)));
        HIP_TRY(ctx, hipMemset(ctx->obs_tests, 0, sizeof(unsigned long long)));
        HIP_TRY(ctx, hipDeviceSynchronize());
    }
    ctx->profiling = on != 0;
    return MPPI_OK;
}

mppi_status mppi_profile_read(mppi_ctx* ctx, mppi_profile* out)
{
    if (!ctx || !out) return MPPI_E_INVALID_ARG;
    for (size_t b = 0; b + kEventsPerUpdate <= ctx->pending.size(); b += kEventsPerUpdate) {
        hipEvent_t* e = &ctx->pending[b];
        HIP_TRY(ctx, hipEventSynchronize(e[kEventsPerUpdate - 1]));
        float t[2];
        for (int i = 0; i < 2; ++i) HIP_TRY(ctx, hipEventElapsedTime(&t[i], e[i], e[i + 1]));
        ctx->acc.updates += 1;
        ctx->acc.rollout_ms += t[0];
        ctx->acc.sum_ms += t[1];
    }
    for (hipEvent_t e : ctx->pending) ctx->pool.push_back(e);
    ctx->pending.clear();
    for (size_t b = 0; b + 3 <= ctx->batch_pending.size(); b += 3) {
        hipEvent_t* e = &ctx->batch_pending[b];
        HIP_TRY(ctx, hipEventSynchronize(e[2]));
        float t0 = 0.0f, t1 = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&t0, e[0], e[1]));
        HIP_TRY(ctx, hipEventElapsedTime(&t1, e[1], e[2]));
        ctx->acc.batches += 1;
        ctx->acc.batch_rollout_ms += t0;
        ctx->acc.batch_rest_ms += t1;
    }
    for (hipEvent_t e : ctx->batch_pending) ctx->pool.push_back(e);
    ctx->batch_pending.clear();
    if (ctx->obs_tests) {
        unsigned long long n = 0;
        HIP_TRY(ctx, hipDeviceSynchronize());
        HIP_TRY(ctx, hipMemcpy(&n, ctx->obs_tests, sizeof(n), hipMemcpyDeviceToHost));
        HIP_TRY(ctx, hipMemset(ctx->obs_tests, 0, sizeof(n)));
        HIP_TRY(ctx, hipDeviceSynchronize());
        ctx->acc.obstacle_tests += (int64_t)n;
    }
    *out = ctx->acc;
    ctx->acc = mppi_profile{};
    return MPPI_OK;
}

}  // extern "C"
