// Serving loop for many vehicles: continuous batching of MPPI updates.
//
// submit() copies a request into an arrival-ordered queue.  One worker thread owns
// the device work: whenever a slot (a context with its own stream, batch arena and
// HIP graph) is free it admits queued requests in arrival order -- at most one in
// flight per vehicle, since each update starts from the previous one's warm start --
// while they fit the slot's share of the memory budget, stages their inputs from
// pinned memory and launches them as one batched update; results come back to pinned
// memory behind an event that the worker polls.  Slots run concurrently, so requests
// that arrive while a batch runs are admitted into the next free slot.
//
// Delay compensation (Sec. IV-E): before a batch runs, each request's state estimate
// can be moved forward over its delay (given, or the running median of the served
// latency) with its vehicle's last served command held, by the same model steps as
// mppi_predict; after the batch, each vehicle's served command is recorded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "context.h"
#include "stages.h"

using namespace mppi;

namespace {

using Clock = std::chrono::steady_clock;

size_t pad64(int K) { return (size_t)((K + 63) & ~63); }
size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

struct Pending {
    uint64_t ticket;
    uint32_t vid;
    int K, N, M;
    float dt, lambda, sigma[4], dt_ctrl, delay;
    uint64_t seed;
    std::vector<float> x_hat, x_ref;
    std::vector<mppi_obstacle> obs;
    double submit_s;
};

// Device footprint of one request inside a slot.
struct Footprint {
    size_t du = 0, k = 0, u = 0, items = 0, in_bytes = 0;
    void add(const Footprint& o)
    {
        du += o.du; k += o.k; u += o.u; items += o.items; in_bytes += o.in_bytes;
    }
};

// Per request, on the device: the delay prediction of its state estimate and the
// record of its vehicle's served command.
struct ServeItem {
    ModelParams P;          // steps of the prediction
    float* x;               // the request's state estimate, predicted in place
    float* hold;            // the vehicle's last served command (4 floats)
    const float* u_apply;   // this request's command
    int steps;              // 0: no prediction
};

__global__ void serve_predict_kernel(const ServeItem* __restrict__ items, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && items[i].steps > 0)
        model_steps(items[i].P, items[i].x, items[i].hold, items[i].x, items[i].steps);
}

__global__ void serve_record_kernel(const ServeItem* __restrict__ items, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        for (int d = 0; d < 4; ++d) items[i].hold[d] = items[i].u_apply[d];
}

Footprint footprint(int K, int N, int M)
{
    Footprint f;
    f.du = 4 * (size_t)N * pad64(K);
    f.k = pad64(K);
    f.u = 4 * (size_t)N;
    f.items = (size_t)(K + 7) / 8;
    f.in_bytes = align16(sizeof(float) * 17) + align16(sizeof(float) * 13 * (size_t)(N + 1)) +
                 align16(sizeof(mppi_obstacle) * (size_t)M) + align16(sizeof(ServeItem));
    return f;
}

constexpr int kOutFloats = 16;   // per request: u_apply (8 floats) + mppi_diag (32 bytes)
constexpr size_t kLatencyWindow = 256;

struct Slot {
    mppi_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char* in_dev = nullptr;
    char* in_host = nullptr;
    float* out_dev = nullptr;
    float* out_host = nullptr;
    Footprint cap;
    bool busy = false;
    std::vector<Pending> batch;
    std::vector<uint32_t> ts;
    std::vector<float> delays;
    std::vector<mppi_request> reqs;
    int32_t pipe = 0;          // the batch is one request run by mppi_update's pipe
    double launch_s = 0.0;
};

}  // namespace

struct mppi_server {
    mppi_server_cfg cfg{};
    Clock::time_point t0;
    float* u_warm = nullptr;                   // device [n_vehicles][N_max][4], then
    float* u_hold = nullptr;                   //   [n_vehicles][4] last served commands
    std::vector<uint32_t> t_next;
    std::vector<double> latency;               // submit-to-result seconds, ring
    size_t latency_next = 0;
    std::vector<char> in_flight, seen;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, mppi_server_result> results;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::vector<Slot> slots;
    mppi_server_stats stats{};
    int busy_slots = 0;
    double busy_since = 0.0;
    int64_t in_flight_reqs = 0;
    mppi_batch_config bcfg{256, 0, 4, 8, 1};   // lanes chosen per instance
    bool bcfg_dirty = false;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    size_t warm_floats() const { return (size_t)cfg.n_vehicles * (cfg.N_max * 4 + 4); }
};

namespace {

bool fits(const Footprint& used, const Footprint& f, const Footprint& cap, size_t n, int max_batch)
{
    return (int)n < max_batch && used.du + f.du <= cap.du && used.k + f.k <= cap.k &&
           used.u + f.u <= cap.u && used.items + f.items <= cap.items &&
           used.in_bytes + f.in_bytes <= cap.in_bytes;
}

// Complete every request of a batch that could not run, with `status` in its diag.
void fail_batch(mppi_server* s, Slot& sl, int32_t status)
{
    const double now = s->now();
    for (size_t i = 0; i < sl.batch.size(); ++i) {
        const Pending& p = sl.batch[i];
        mppi_server_result r{};
        r.ticket = p.ticket; r.vehicle_id = p.vid; r.t = sl.ts.empty() ? 0 : sl.ts[i];
        for (float& v : r.u_apply) v = NAN;
        r.diag.status = status;
        r.submit_s = p.submit_s; r.launch_s = sl.launch_s; r.done_s = now; r.K = p.K; r.N = p.N;
        r.delay = i < sl.delays.size() ? sl.delays[i] : 0.0f;
        s->results[p.ticket] = r;
        s->in_flight[p.vid] = 0;
        s->stats.completed += 1;
    }
    s->in_flight_reqs -= (int64_t)sl.batch.size();
    sl.batch.clear();
    sl.ts.clear();
    s->cv_done.notify_all();
}

void harvest(mppi_server* s, Slot& sl)
{
    const double now = s->now();
    for (size_t i = 0; i < sl.batch.size(); ++i) {
        const Pending& p = sl.batch[i];
        mppi_server_result r{};
        r.ticket = p.ticket;
        r.vehicle_id = p.vid;
        r.t = sl.ts[i];
        std::memcpy(r.u_apply, sl.out_host + kOutFloats * i, sizeof(r.u_apply));
        std::memcpy(&r.diag, sl.out_host + kOutFloats * i + 8, sizeof(mppi_diag));
        r.submit_s = p.submit_s;
        r.launch_s = sl.launch_s;
        r.done_s = now;
        r.K = p.K;
        r.N = p.N;
        r.delay = sl.delays[i];
        r.pipe = sl.pipe;
        s->results[p.ticket] = r;
        if (s->latency.size() < kLatencyWindow) {
            s->latency.push_back(now - p.submit_s);
        } else {
            s->latency[s->latency_next] = now - p.submit_s;
            s->latency_next = (s->latency_next + 1) % kLatencyWindow;
        }
        s->in_flight[p.vid] = 0;
        s->stats.completed += 1;
        s->stats.rollout_steps += (int64_t)p.K * p.N;
    }
    s->in_flight_reqs -= (int64_t)sl.batch.size();
    sl.batch.clear();
    sl.ts.clear();
    sl.busy = false;
    if (--s->busy_slots == 0) s->stats.busy_s += now - s->busy_since;
    s->cv_done.notify_all();
}

// Median submit-to-result latency of the last completed requests (0 before any).
double latency_estimate(mppi_server* s)
{
    if (s->latency.empty()) return 0.0;
    std::vector<double> v(s->latency);
    std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
    return v[v.size() / 2];
}

// Admit queued requests into a free slot and launch them.  Called with the lock held.
bool dispatch(mppi_server* s, Slot& sl)
{
    std::fill(s->seen.begin(), s->seen.end(), 0);
    std::vector<size_t> pick;
    Footprint used;
    for (size_t i = 0; i < s->queue.size() && (int)pick.size() < s->cfg.max_batch; ++i) {
        const Pending& p = s->queue[i];
        if (s->in_flight[p.vid] || s->seen[p.vid]) {   // keep each vehicle's order
            s->seen[p.vid] = 1;
            continue;
        }
        s->seen[p.vid] = 1;
        const Footprint f = footprint(p.K, p.N, p.M);
        if (!fits(used, f, sl.cap, pick.size(), s->cfg.max_batch)) continue;
        pick.push_back(i);
        used.add(f);
    }
    if (pick.empty()) return false;

    sl.batch.clear();
    for (size_t i : pick) sl.batch.push_back(std::move(s->queue[i]));
    for (auto it = pick.rbegin(); it != pick.rend(); ++it) s->queue.erase(s->queue.begin() + *it);

    const int n = (int)sl.batch.size();
    sl.reqs.assign(n, mppi_request{});
    sl.ts.assign(n, 0);
    sl.delays.assign(n, 0.0f);
    std::vector<size_t> o_x(n);
    bool predict = false;
    double auto_delay = -1.0;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const Pending& p = sl.batch[i];
        float* xh = reinterpret_cast<float*>(sl.in_host + off);
        std::memcpy(xh, p.x_hat.data(), sizeof(float) * 17);
        const size_t o_xh = o_x[i] = off;
        off += align16(sizeof(float) * 17);
        std::memcpy(sl.in_host + off, p.x_ref.data(), sizeof(float) * p.x_ref.size());
        const size_t o_xr = off;
        off += align16(sizeof(float) * p.x_ref.size());
        if (p.M > 0) std::memcpy(sl.in_host + off, p.obs.data(), sizeof(mppi_obstacle) * p.M);
        const size_t o_ob = off;
        off += align16(sizeof(mppi_obstacle) * (size_t)p.M);

        mppi_request& r = sl.reqs[i];
        r.veh = s->cfg.veh;
        r.cost = s->cfg.cost;
        r.solve.K = p.K; r.solve.N = p.N; r.solve.dt = p.dt; r.solve.lambda = p.lambda;
        for (int d = 0; d < 4; ++d) { r.solve.sigma[d] = p.sigma[d]; r.solve.u_init[d] = s->cfg.u_init[d]; }
        r.solve.seed = p.seed;
        r.solve.dt_ctrl = p.dt_ctrl;
        r.solve.vehicle_id = p.vid;
        r.solve.t = sl.ts[i] = s->t_next[p.vid]++;
        r.x_hat = reinterpret_cast<const float*>(sl.in_dev + o_xh);
        r.x_ref = reinterpret_cast<const float*>(sl.in_dev + o_xr);
        r.obs = p.M > 0 ? reinterpret_cast<const mppi_obstacle*>(sl.in_dev + o_ob) : nullptr;
        r.M = p.M;
        r.u_nom = s->u_warm + (size_t)p.vid * s->cfg.N_max * 4;
        r.u_apply = sl.out_dev + kOutFloats * i;
        r.diag = reinterpret_cast<mppi_diag*>(sl.out_dev + kOutFloats * i + 8);
        s->in_flight[p.vid] = 1;
        float delay = p.delay;
        if (delay < 0) {
            if (auto_delay < 0) auto_delay = latency_estimate(s);
            delay = (float)std::min(auto_delay, (double)kPredictMaxSteps * p.dt);
        }
        sl.delays[i] = delay;
        predict = predict || delay > 0;
    }
    // the per-request items follow the inputs
    const size_t o_items = off;
    ServeItem* items = reinterpret_cast<ServeItem*>(sl.in_host + o_items);
    for (int i = 0; i < n; ++i) {
        const Pending& p = sl.batch[i];
        ServeItem& it = items[i];
        it.steps = std::max(predict_steps(p.dt, sl.delays[i]), 0);
        it.P = predict_params(s->cfg.veh, p.dt, sl.delays[i], it.steps);
        it.x = reinterpret_cast<float*>(sl.in_dev + o_x[i]);
        it.hold = s->u_hold + 4 * (size_t)p.vid;
        it.u_apply = sl.out_dev + kOutFloats * i;
    }
    off += sizeof(ServeItem) * n;
    const ServeItem* items_dev = reinterpret_cast<const ServeItem*>(sl.in_dev + o_items);
    const int grid = (n + 63) / 64;
    sl.launch_s = s->now();
    s->in_flight_reqs += n;
    s->stats.max_in_flight = std::max(s->stats.max_in_flight, s->in_flight_reqs);
    hipError_t e = hipMemcpyAsync(sl.in_dev, sl.in_host, off, hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess && predict) {
        hipLaunchKernelGGL(serve_predict_kernel, dim3(grid), dim3(64), 0, sl.stream, items_dev, n);
        e = hipGetLastError();
    }
    // A lone request runs as a single-instance update (wave-specialised rollouts under
    // the default shape), a batch as one batched launch sequence.
    mppi_status st = MPPI_E_HIP;
    sl.pipe = 0;
    if (e == hipSuccess && n == 1) {
        const mppi_request& r = sl.reqs[0];
        mppi_launch_config cfg{};
        st = mppi_get_config(sl.ctx, r.solve.K, r.solve.N, r.M, &cfg);
        if (st == MPPI_OK)
            st = mppi_update(sl.ctx, sl.stream, &r.veh, &r.cost, &r.solve, r.x_hat, r.x_ref, r.obs, r.M,
                             r.u_nom, r.u_apply, r.diag);
        sl.pipe = cfg.pipe != 0 && r.M <= kPipeMaxM ? 1 : 0;
    } else if (e == hipSuccess) {
        st = mppi_batch_update(sl.ctx, sl.stream, sl.reqs.data(), n);
    }
    if (st == MPPI_OK) {
        hipLaunchKernelGGL(serve_record_kernel, dim3(grid), dim3(64), 0, sl.stream, items_dev, n);
        e = hipGetLastError();
    }
    if (st == MPPI_OK && e == hipSuccess)
        e = hipMemcpyAsync(sl.out_host, sl.out_dev, sizeof(float) * kOutFloats * n,
                           hipMemcpyDeviceToHost, sl.stream);
    if (st == MPPI_OK && e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (st != MPPI_OK || e != hipSuccess) {
        (void)hipStreamSynchronize(sl.stream);
        fail_batch(s, sl, st != MPPI_OK ? st : MPPI_E_HIP);
        return true;
    }
    s->stats.batches += 1;
    sl.busy = true;
    if (s->busy_slots++ == 0) s->busy_since = sl.launch_s;
    return true;
}

void worker_main(mppi_server* s)
{
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progressed = false;
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                harvest(s, sl);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                fail_batch(s, sl, MPPI_E_HIP);
                sl.busy = false;
                if (--s->busy_slots == 0) s->stats.busy_s += s->now() - s->busy_since;
                progressed = true;
            }
        }
        if (s->bcfg_dirty && s->busy_slots == 0) {
            for (Slot& sl : s->slots) (void)mppi_batch_set_config(sl.ctx, &s->bcfg);
            s->bcfg_dirty = false;
        }
        if (!s->bcfg_dirty)
            for (Slot& sl : s->slots)
                if (!sl.busy && !s->queue.empty() && dispatch(s, sl)) progressed = true;
        if (s->stop && s->queue.empty() && s->busy_slots == 0) break;
        if (progressed) continue;
        if (s->busy_slots > 0) {             // poll the running batches
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty() || s->bcfg_dirty; });
        }
    }
    s->cv_done.notify_all();
}

void free_slots(mppi_server* s)
{
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.ctx) mppi_destroy(sl.ctx);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        (void)hipFree(sl.in_dev);
        (void)hipFree(sl.out_dev);
        if (sl.in_host) (void)hipHostFree(sl.in_host);
        if (sl.out_host) (void)hipHostFree(sl.out_host);
    }
    s->slots.clear();
}

mppi_status check_cfg(const mppi_server_cfg* c)
{
    if (!c) return MPPI_E_INVALID_ARG;
    if (c->n_vehicles < 1 || c->K_max < 1 || c->N_max < 1 || c->N_max > MPPI_N_MAX || c->M_max < 0 ||
        c->M_max > MPPI_M_MAX || c->n_streams < 1 || c->n_streams > 8 || c->max_batch < 1 ||
        c->budget_bytes <= 0)
        return MPPI_E_INVALID_ARG;
    mppi_solve probe{};
    probe.K = 1; probe.N = 1; probe.dt = 0.01f; probe.lambda = 1.0f;
    for (int d = 0; d < 4; ++d) probe.u_init[d] = c->u_init[d];
    return mppi_validate(&c->veh, &c->cost, &probe, 0);
}

}  // namespace

extern "C" {

mppi_status mppi_server_create(const mppi_server_cfg* cfg, mppi_server** out)
{
    if (!out) return MPPI_E_INVALID_ARG;
    *out = nullptr;
    mppi_status st = check_cfg(cfg);
    if (st != MPPI_OK) return st;
    mppi_server* s = new (std::nothrow) mppi_server();
    if (!s) return MPPI_E_OOM;
    s->cfg = *cfg;
    s->t0 = Clock::now();
    s->t_next.assign(cfg->n_vehicles, 0u);
    s->in_flight.assign(cfg->n_vehicles, 0);
    s->seen.assign(cfg->n_vehicles, 0);
    bool ok = hipSetDevice(cfg->device) == hipSuccess;
    const size_t warm = s->warm_floats();
    if (ok) ok = hipMalloc(&s->u_warm, sizeof(float) * warm) == hipSuccess;
    if (ok) {
        s->u_hold = s->u_warm + (size_t)cfg->n_vehicles * cfg->N_max * 4;
        std::vector<float> init(warm);
        for (size_t i = 0; i < warm; ++i) init[i] = cfg->u_init[i & 3];
        ok = hipMemcpy(s->u_warm, init.data(), sizeof(float) * warm, hipMemcpyHostToDevice) == hipSuccess;
    }
    // each slot gets an equal share of the budget for delta_u; the other arenas are
    // sized for max_batch requests of the largest shape
    const int mb = cfg->max_batch;
    Footprint big = footprint(cfg->K_max, cfg->N_max, cfg->M_max);
    Footprint cap;
    cap.du = (size_t)(cfg->budget_bytes / cfg->n_streams) / sizeof(float);
    cap.k = big.k * mb; cap.u = big.u * mb; cap.items = big.items * mb; cap.in_bytes = big.in_bytes * mb;
    for (int i = 0; ok && i < cfg->n_streams; ++i) {
        s->slots.emplace_back();
        Slot& sl = s->slots.back();
        sl.cap = cap;
        ok = mppi_create(cfg->device, &sl.ctx) == MPPI_OK &&
             batch_reserve_raw(sl.ctx, mb, cap.du, cap.k, cap.u, cap.items, std::max(cfg->M_max, 1)) ==
                 MPPI_OK &&
             mppi_reserve(sl.ctx, cfg->K_max, cfg->N_max, cfg->M_max) == MPPI_OK &&
             hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
             hipMalloc(&sl.in_dev, cap.in_bytes) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&sl.in_host), cap.in_bytes, hipHostMallocDefault) ==
                 hipSuccess &&
             hipMalloc(&sl.out_dev, sizeof(float) * kOutFloats * mb) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&sl.out_host), sizeof(float) * kOutFloats * mb,
                           hipHostMallocDefault) == hipSuccess &&
             mppi_batch_set_config(sl.ctx, &s->bcfg) == MPPI_OK;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_slots(s);
        (void)hipFree(s->u_warm);
        delete s;
        return MPPI_E_OOM;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return MPPI_OK;
}

mppi_status mppi_server_destroy(mppi_server* s)
{
    if (!s) return MPPI_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->cfg.device);
    free_slots(s);
    (void)hipFree(s->u_warm);
    delete s;
    return MPPI_OK;
}

mppi_status mppi_server_set_batch_config(mppi_server* s, const mppi_batch_config* cfg)
{
    if (!s || !cfg) return MPPI_E_INVALID_ARG;
    const BatchLaunch c{cfg->block, cfg->lanes, cfg->unroll, cfg->blocks_per_cu};
    if (!valid_batch_launch(c)) return MPPI_E_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->bcfg = *cfg;
        s->bcfg_dirty = true;
    }
    s->cv_work.notify_all();
    return MPPI_OK;
}

mppi_status mppi_server_submit(mppi_server* s, const mppi_server_request* r, uint64_t* ticket)
{
    if (!s || !r || !ticket) return MPPI_E_INVALID_ARG;
    const mppi_server_cfg& c = s->cfg;
    if (r->vehicle_id >= (uint32_t)c.n_vehicles || r->K < 1 || r->K > c.K_max || r->N < 1 ||
        r->N > c.N_max || r->M < 0 || r->M > c.M_max || !r->x_hat || !r->x_ref ||
        (r->M > 0 && !r->obs))
        return MPPI_E_INVALID_ARG;
    if (!std::isfinite(r->dt) || !(r->dt > 0) || !std::isfinite(r->lambda) || !(r->lambda > 0))
        return MPPI_E_INVALID_ARG;
    if (!std::isfinite(r->dt_ctrl) || r->dt_ctrl < 0 || r->dt_ctrl > r->dt || !std::isfinite(r->delay) ||
        (r->delay >= 0 && predict_steps(r->dt, r->delay) < 0))
        return MPPI_E_INVALID_ARG;
    for (float sg : r->sigma)
        if (!std::isfinite(sg) || sg < 0) return MPPI_E_INVALID_ARG;
    const Footprint f = footprint(r->K, r->N, r->M);
    if (f.du > s->slots.front().cap.du) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stats.rejected += 1;
        return MPPI_E_BUDGET;
    }
    Pending p;
    p.vid = r->vehicle_id; p.K = r->K; p.N = r->N; p.M = r->M; p.dt = r->dt; p.lambda = r->lambda;
    p.dt_ctrl = r->dt_ctrl; p.delay = r->delay;
    for (int d = 0; d < 4; ++d) p.sigma[d] = r->sigma[d];
    p.seed = r->seed;
    p.x_hat.assign(r->x_hat, r->x_hat + 17);
    p.x_ref.assign(r->x_ref, r->x_ref + 13 * (size_t)(r->N + 1));
    if (r->M > 0) p.obs.assign(r->obs, r->obs + r->M);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        p.ticket = s->next_ticket++;
        p.submit_s = s->now();
        *ticket = p.ticket;
        s->queue.push_back(std::move(p));
        s->stats.submitted += 1;
    }
    s->cv_work.notify_one();
    return MPPI_OK;
}

mppi_status mppi_server_poll(mppi_server* s, uint64_t ticket, mppi_server_result* out)
{
    if (!s || !out) return MPPI_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return (ticket > 0 && ticket < s->next_ticket) ? MPPI_E_PENDING : MPPI_E_INVALID_ARG;
    *out = it->second;
    s->results.erase(it);
    return MPPI_OK;
}

mppi_status mppi_server_wait(mppi_server* s, uint64_t ticket, mppi_server_result* out)
{
    if (!s || !out || ticket == 0) return MPPI_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket >= s->next_ticket) return MPPI_E_INVALID_ARG;
    s->cv_done.wait(lk, [&] { return s->results.count(ticket) > 0 || (s->stop && s->queue.empty() && s->busy_slots == 0); });
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return MPPI_E_INVALID_ARG;
    *out = it->second;
    s->results.erase(it);
    return MPPI_OK;
}

mppi_status mppi_server_drain(mppi_server* s)
{
    if (!s) return MPPI_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->queue.empty() && s->busy_slots == 0; });
    return MPPI_OK;
}

mppi_status mppi_server_stats_get(mppi_server* s, mppi_server_stats* out)
{
    if (!s || !out) return MPPI_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    if (s->busy_slots > 0) out->busy_s += s->now() - s->busy_since;
    return MPPI_OK;
}

double mppi_server_clock(const mppi_server* s)
{
    return s ? s->now() : 0.0;
}

mppi_status mppi_server_snapshot(mppi_server* s, void* buf, size_t* size)
{
    if (!s || !size) return MPPI_E_INVALID_ARG;
    const size_t warm = sizeof(float) * s->warm_floats();
    const size_t need = warm + sizeof(uint32_t) * s->cfg.n_vehicles;
    if (!buf) { *size = need; return MPPI_OK; }
    if (*size < need) { *size = need; return MPPI_E_INVALID_ARG; }
    mppi_status st = mppi_server_drain(s);
    if (st != MPPI_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    if (hipMemcpy(buf, s->u_warm, warm, hipMemcpyDeviceToHost) != hipSuccess) return MPPI_E_HIP;
    std::memcpy(static_cast<char*>(buf) + warm, s->t_next.data(), sizeof(uint32_t) * s->cfg.n_vehicles);
    *size = need;
    return MPPI_OK;
}

mppi_status mppi_server_restore(mppi_server* s, const void* buf, size_t size)
{
    if (!s || !buf) return MPPI_E_INVALID_ARG;
    const size_t warm = sizeof(float) * s->warm_floats();
    if (size != warm + sizeof(uint32_t) * s->cfg.n_vehicles) return MPPI_E_INVALID_ARG;
    mppi_status st = mppi_server_drain(s);
    if (st != MPPI_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    if (hipMemcpy(s->u_warm, buf, warm, hipMemcpyHostToDevice) != hipSuccess) return MPPI_E_HIP;
    std::memcpy(s->t_next.data(), static_cast<const char*>(buf) + warm, sizeof(uint32_t) * s->cfg.n_vehicles);
    return MPPI_OK;
}

}  // extern "C"
