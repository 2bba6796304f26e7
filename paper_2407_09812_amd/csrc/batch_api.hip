// C ABI of the batched path: many uneven MPPI instances per launch sequence.
//
// Each call plans the batch on the host (instance descriptors, scratch slices and
// (instance, sample-tile) work items ordered longest first), copies the plan from
// pinned memory to the device on the caller's stream, then either replays a HIP graph
// of the five batch kernels (captured once per launch shape) or launches them.  The
// graph only ever reads the plan from fixed device addresses, so one capture serves
// every batch that fits the reserved capacity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "context.h"

using namespace mppi;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct PlanLayout {
    size_t descs_off, items_off, bytes;
};

PlanLayout plan_layout(int n_cap, size_t items_cap)
{
    PlanLayout p;
    p.descs_off = align_up(sizeof(BatchHeader), kAlign);
    p.items_off = align_up(p.descs_off + sizeof(InstanceDesc) * (size_t)n_cap, kAlign);
    p.bytes = align_up(p.items_off + sizeof(WorkItem) * items_cap, kAlign);
    return p;
}

struct Needs {
    int n = 0, M_max = 0;
    size_t du = 0, k = 0, u = 0, items_min_tile = 0;
};

int pad64(int K) { return (K + 63) & ~63; }

mppi_status check_requests(mppi_ctx* ctx, const mppi_request* reqs, int32_t n, Needs* nd)
{
    if (!reqs || n < 1) return fail(ctx, MPPI_E_INVALID_ARG, "batch: empty request list");
    Needs r;
    r.n = n;
    for (int i = 0; i < n; ++i) {
        const mppi_request& q = reqs[i];
        mppi_status st = mppi_validate(&q.veh, &q.cost, &q.solve, q.M);
        if (st != MPPI_OK)
            return fail(ctx, st, "batch: request " + std::to_string(i) + " has invalid parameters");
        if (!q.x_hat || !q.x_ref || !q.u_nom || !q.u_apply || (q.M > 0 && !q.obs))
            return fail(ctx, MPPI_E_INVALID_ARG, "batch: request " + std::to_string(i) +
                                                     " has a null device pointer");
        const size_t ld = (size_t)pad64(q.solve.K);
        r.du += 4 * (size_t)q.solve.N * ld;
        r.k += ld;
        r.u += 4 * (size_t)q.solve.N;
        r.items_min_tile += (size_t)(q.solve.K + 7) / 8;       // 8 samples: the smallest tile
        r.M_max = std::max(r.M_max, (int)q.M);
    }
    *nd = r;
    return MPPI_OK;
}

void destroy_graph(BatchState& b)
{
    if (b.graph_exec) (void)hipGraphExecDestroy(b.graph_exec);
    b.graph_exec = nullptr;
}

// Fill the pinned plan for `cfg`; returns the number of bytes to upload.  own_diags:
// every instance reports into the arena's diagnostics (autotuning), not the caller's.
size_t fill_plan(mppi_ctx* ctx, const mppi_request* reqs, int n, const BatchLaunch& cfg,
                 bool own_diags)
{
    BatchState& b = ctx->batch;
    const PlanLayout L = plan_layout(b.n_cap, b.items_cap);
    char* host = static_cast<char*>(b.plan_host);
    BatchHeader* hdr = reinterpret_cast<BatchHeader*>(host);
    InstanceDesc* descs = reinterpret_cast<InstanceDesc*>(host + L.descs_off);
    WorkItem* items = reinterpret_cast<WorkItem*>(host + L.items_off);

    // lanes per instance: fixed, or (cfg.lanes == 0) as many as keep the whole batch
    // near one wave per SIMD, capped so that each lane keeps >= 8 obstacles to test
    int auto_lanes = 1;
    if (cfg.lanes == 0) {
        long long waves = 0;
        for (int i = 0; i < n; ++i) waves += (reqs[i].solve.K + 63) / 64;
        while (auto_lanes < 8 && waves * auto_lanes * 2 <= 1024) auto_lanes *= 2;
    }
    size_t du_off = 0, k_off = 0, u_off = 0, st_off = 0;
    int row = 0;
    struct Keyed { long long cost; int inst, k0; };
    std::vector<Keyed> work;
    for (int i = 0; i < n; ++i) {
        const mppi_request& q = reqs[i];
        InstanceDesc& D = descs[i];
        const int K = q.solve.K, N = q.solve.N, ld = pad64(K);
        D.rp.mp = model_params(q.veh, q.solve.dt);
        D.rp.cp = cost_params(q.cost);
        D.rp.np = noise_params(q.solve);
        D.rp.M = q.M; D.rp.K = K; D.rp.N = N; D.rp.ld = ld;
        D.rp.obs_tests = ctx->profiling ? ctx->obs_tests : nullptr;
        D.lambda = q.solve.lambda;
        D.alpha = advance_fraction(q.solve);
        for (int d = 0; d < 4; ++d) D.u_init[d] = q.solve.u_init[d];
        D.row0 = row;
        int lanes = cfg.lanes;
        if (lanes == 0) {
            lanes = 1;
            while (lanes < auto_lanes && q.M >= 8 * 2 * lanes) lanes *= 2;
        }
        D.lanes = lanes;
        const int tile = cfg.block / lanes;
        D.x_hat = q.x_hat; D.x_ref = q.x_ref; D.obs = q.obs;
        D.u_nom = q.u_nom; D.u_apply = q.u_apply;
        D.diag = q.diag && !own_diags ? q.diag : b.diags + i;
        D.du = b.du + du_off; D.S = b.S + k_off; D.u_upd = b.u_upd + u_off;
        D.W = (K + tile - 1) / tile * cfg.block / 64;
        D.stat = b.stat + st_off;
        du_off += 4 * (size_t)N * ld; k_off += ld; u_off += 4 * (size_t)N; row += 4 * N;
        st_off += (size_t)D.W;
        // cost of one tile: N steps of dynamics plus this lane's share of the obstacles
        const long long cost = (long long)N * (650 + 11 * ((q.M + lanes - 1) / lanes));
        for (int k0 = 0; k0 < K; k0 += tile) work.push_back({cost, i, k0});
    }
    std::stable_sort(work.begin(), work.end(),
                     [](const Keyed& a, const Keyed& c) { return a.cost > c.cost; });
    for (size_t t = 0; t < work.size(); ++t) items[t] = WorkItem{work[t].inst, work[t].k0};
    hdr->n_inst = n;
    hdr->n_items = (int)work.size();
    hdr->n_rows = row;
    hdr->next_item = 0u;
    return L.items_off + sizeof(WorkItem) * work.size();
}

// Copy the plan to the device on `s` (waiting first for the previous copy out of the
// pinned buffer, which this call overwrites).
mppi_status stage_plan(mppi_ctx* ctx, const mppi_request* reqs, int n, const BatchLaunch& cfg,
                       hipStream_t s, bool own_diags = false)
{
    BatchState& b = ctx->batch;
    if (b.staged_pending) {
        HIP_TRY(ctx, hipEventSynchronize(b.staged));
        b.staged_pending = false;
    }
    const size_t bytes = fill_plan(ctx, reqs, n, cfg, own_diags);
    HIP_TRY(ctx, hipMemcpyAsync(b.plan_dev, b.plan_host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(b.staged, s));
    b.staged_pending = true;
    return MPPI_OK;
}

BatchHeader* dev_header(const BatchState& b) { return static_cast<BatchHeader*>(b.plan_dev); }
const InstanceDesc* dev_descs(const BatchState& b)
{
    return reinterpret_cast<const InstanceDesc*>(static_cast<char*>(b.plan_dev) +
                                                 plan_layout(b.n_cap, b.items_cap).descs_off);
}
const WorkItem* dev_items(const BatchState& b)
{
    return reinterpret_cast<const WorkItem*>(static_cast<char*>(b.plan_dev) +
                                             plan_layout(b.n_cap, b.items_cap).items_off);
}
int lds_bytes(const BatchState& b) { return (int)obstacle_lds_bytes(std::max(b.M_cap, 1)); }

mppi_status capacity_ok(mppi_ctx* ctx, const Needs& nd)
{
    const BatchState& b = ctx->batch;
    if (nd.n > b.n_cap || nd.du > b.du_cap || nd.k > b.k_cap || nd.u > b.u_cap ||
        nd.items_min_tile > b.items_cap || nd.M_max > b.M_cap)
        return fail(ctx, MPPI_E_CAPACITY, "batch: exceeds reserved capacity (mppi_batch_reserve)");
    return MPPI_OK;
}

}  // namespace

namespace mppi {

void free_batch(mppi_ctx* ctx)
{
    BatchState& b = ctx->batch;
    destroy_graph(b);
    if (b.staged_pending && b.staged) (void)hipEventSynchronize(b.staged);
    (void)hipFree(b.plan_dev); (void)hipFree(b.diags); (void)hipFree(b.du); (void)hipFree(b.S);
    (void)hipFree(b.stat); (void)hipFree(b.u_upd);
    if (b.plan_host) (void)hipHostFree(b.plan_host);
    if (b.staged) (void)hipEventDestroy(b.staged);
    if (b.capture_stream) (void)hipStreamDestroy(b.capture_stream);
    const BatchLaunch cfg = b.cfg;
    const bool g = b.use_graph;
    b = BatchState{};
    b.cfg = cfg;
    b.use_graph = g;
}

}  // namespace mppi

namespace mppi {

// Grow the batch arena to at least these capacities (instances, delta_u floats,
// padded samples, control floats, smallest-tile work items, obstacles).
mppi_status batch_reserve_raw(mppi_ctx* ctx, int n, size_t du, size_t k, size_t u, size_t items,
                              int M)
{
    Needs nd;
    nd.n = n; nd.du = du; nd.k = k; nd.u = u; nd.items_min_tile = items; nd.M_max = M;
    BatchState& b = ctx->batch;
    if (b.plan_dev && capacity_ok(ctx, nd) == MPPI_OK) return MPPI_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    Needs grow;
    grow.n = std::max(nd.n, b.n_cap);
    grow.M_max = std::max(nd.M_max, b.M_cap);
    grow.du = std::max(nd.du, b.du_cap);
    grow.k = std::max(nd.k, b.k_cap);
    grow.u = std::max(nd.u, b.u_cap);
    grow.items_min_tile = std::max(nd.items_min_tile, b.items_cap);
    free_batch(ctx);
    const PlanLayout L = plan_layout(grow.n, grow.items_min_tile);
    bool ok = hipMalloc(&b.plan_dev, L.bytes) == hipSuccess &&
              hipHostMalloc(&b.plan_host, L.bytes, hipHostMallocDefault) == hipSuccess &&
              hipMalloc(&b.diags, sizeof(mppi_diag) * grow.n) == hipSuccess &&
              hipMalloc(&b.du, sizeof(float) * grow.du) == hipSuccess &&
              hipMalloc(&b.S, sizeof(float) * grow.k) == hipSuccess &&
              hipMalloc(&b.stat, sizeof(WaveStat) * (grow.k / 8 + 4 * (size_t)grow.n)) == hipSuccess &&
              hipMalloc(&b.u_upd, sizeof(float) * grow.u) == hipSuccess &&
              hipEventCreateWithFlags(&b.staged, hipEventDisableTiming) == hipSuccess &&
              hipStreamCreateWithFlags(&b.capture_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_batch(ctx);
        return fail(ctx, MPPI_E_OOM, "batch_reserve: allocation failed");
    }
    b.n_cap = grow.n; b.M_cap = grow.M_max; b.du_cap = grow.du; b.k_cap = grow.k; b.u_cap = grow.u;
    b.items_cap = grow.items_min_tile; b.plan_bytes = L.bytes;
    b.stat_cap = grow.k / 8 + 4 * (size_t)grow.n;
    return MPPI_OK;
}

}  // namespace mppi

extern "C" {

mppi_status mppi_batch_reserve(mppi_ctx* ctx, const mppi_request* reqs, int32_t n)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    Needs nd;
    mppi_status st = check_requests(ctx, reqs, n, &nd);
    if (st != MPPI_OK) return st;
    return batch_reserve_raw(ctx, nd.n, nd.du, nd.k, nd.u, nd.items_min_tile, nd.M_max);
}

mppi_status mppi_batch_update(mppi_ctx* ctx, void* stream, const mppi_request* reqs, int32_t n)
{
    if (!ctx) return MPPI_E_INVALID_ARG;
    Needs nd;
    mppi_status st = check_requests(ctx, reqs, n, &nd);
    if (st != MPPI_OK) return st;
    if ((st = capacity_ok(ctx, nd)) != MPPI_OK) return st;
    BatchState& b = ctx->batch;
    hipStream_t s = (hipStream_t)stream;
    if ((st = stage_plan(ctx, reqs, n, b.cfg, s)) != MPPI_OK) return st;
    if (ctx->profiling) {                 // eager launches bracketed by events
        hipEvent_t ev[3];
        for (hipEvent_t& e : ev)
            if (!(e = take_event(ctx))) return fail(ctx, MPPI_E_HIP, "batch: event creation");
        HIP_TRY(ctx, hipEventRecord(ev[0], s));
        HIP_TRY(ctx, launch_batch_rollout(dev_header(b), dev_descs(b), dev_items(b), ctx->cu_count,
                                          lds_bytes(b), b.cfg, s));
        HIP_TRY(ctx, hipEventRecord(ev[1], s));
        HIP_TRY(ctx, launch_batch_tail(dev_header(b), dev_descs(b), b.n_cap, ctx->cu_count, s));
        HIP_TRY(ctx, hipEventRecord(ev[2], s));
        for (hipEvent_t e : ev) ctx->batch_pending.push_back(e);
        return MPPI_OK;
    }
    if (!b.use_graph) {
        HIP_TRY(ctx, launch_batch(dev_header(b), dev_descs(b), dev_items(b), b.n_cap,
                                  ctx->cu_count, lds_bytes(b), b.cfg, s));
        return MPPI_OK;
    }
    const auto key = std::make_tuple(b.cfg.block, b.cfg.lanes, b.cfg.unroll, b.cfg.blocks_per_cu,
                                     lds_bytes(b), b.n_cap);
    if (!b.graph_exec || b.graph_key != key) {
        destroy_graph(b);
        hipGraph_t graph = nullptr;
        HIP_TRY(ctx, hipStreamBeginCapture(b.capture_stream, hipStreamCaptureModeRelaxed));
        hipError_t e = launch_batch(dev_header(b), dev_descs(b), dev_items(b), b.n_cap,
                                    ctx->cu_count, lds_bytes(b), b.cfg, b.capture_stream);
        hipError_t e2 = hipStreamEndCapture(b.capture_stream, &graph);
        if (e != hipSuccess) return hip_fail(ctx, e, "batch: capture");
        if (e2 != hipSuccess) return hip_fail(ctx, e2, "batch: end capture");
        e = hipGraphInstantiate(&b.graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b.graph_exec = nullptr;
            return hip_fail(ctx, e, "batch: graph instantiate");
        }
        b.graph_key = key;
    }
    HIP_TRY(ctx, hipGraphLaunch(b.graph_exec, s));
    return MPPI_OK;
}

mppi_status mppi_batch_get_config(const mppi_ctx* ctx, mppi_batch_config* out)
{
    if (!ctx || !out) return MPPI_E_INVALID_ARG;
    const BatchState& b = ctx->batch;
    out->block = b.cfg.block; out->lanes = b.cfg.lanes; out->unroll = b.cfg.unroll;
    out->blocks_per_cu = b.cfg.blocks_per_cu; out->use_graph = b.use_graph ? 1 : 0;
    return MPPI_OK;
}

mppi_status mppi_batch_set_config(mppi_ctx* ctx, const mppi_batch_config* cfg)
{
    if (!ctx || !cfg) return MPPI_E_INVALID_ARG;
    const BatchLaunch c{cfg->block, cfg->lanes, cfg->unroll, cfg->blocks_per_cu};
    if (!valid_batch_launch(c)) return fail(ctx, MPPI_E_INVALID_ARG, "batch_set_config: invalid shape");
    ctx->batch.cfg = c;
    ctx->batch.use_graph = cfg->use_graph != 0;
    return MPPI_OK;
}

mppi_status mppi_batch_autotune(mppi_ctx* ctx, void* stream, const mppi_request* reqs, int32_t n,
                                int32_t reps, mppi_batch_config* best)
{
    if (!ctx || reps < 1) return MPPI_E_INVALID_ARG;
    Needs nd;
    mppi_status st = check_requests(ctx, reqs, n, &nd);
    if (st != MPPI_OK) return st;
    if ((st = capacity_ok(ctx, nd)) != MPPI_OK) return st;
    BatchState& b = ctx->batch;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    std::vector<BatchLaunch> candidates;
    for (int lanes : {0, 1, 2, 4})
        for (int block : {64, 128, 256})
            for (int unroll : {1, 4})
                for (int bpc : {1, 2, 4, 8}) {
                    if (lanes > 1 && nd.M_max < 4 * lanes) continue;   // nothing to divide
                    if (unroll > 1 && nd.M_max < 8) continue;
                    candidates.push_back(BatchLaunch{block, lanes, unroll, bpc});
                }
    BatchLaunch best_c = b.cfg;
    float best_ms = 1e30f;
    mppi_status result = MPPI_OK;
    for (const BatchLaunch& c : candidates) {
        if ((result = stage_plan(ctx, reqs, n, c, s, true)) != MPPI_OK) break;
        hipError_t e = launch_batch_rollout(dev_header(b), dev_descs(b), dev_items(b),
                                            ctx->cu_count, lds_bytes(b), c, s);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_batch_rollout(dev_header(b), dev_descs(b), dev_items(b), ctx->cu_count,
                                     lds_bytes(b), c, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { result = hip_fail(ctx, e, "batch_autotune"); break; }
        if (ms < best_ms) { best_ms = ms; best_c = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != MPPI_OK) return result;
    b.cfg = best_c;
    if (best) {
        best->block = best_c.block; best->lanes = best_c.lanes; best->unroll = best_c.unroll;
        best->blocks_per_cu = best_c.blocks_per_cu; best->use_graph = b.use_graph ? 1 : 0;
    }
    return MPPI_OK;
}

}  // extern "C"
