// Batched MPPI kernels: many uneven instances (K, N, M differ) in one launch sequence.
//
//   batch_reset_kernel     work-queue head <- 0 (a kernel, so the sequence can be
//                          captured in a HIP graph without memset nodes)
//   batch_rollout_kernel   persistent: each workgroup pulls (instance, sample tile)
//                          items, longest first, from a device queue, stages that
//                          instance's obstacles in LDS, rolls the tile out and writes
//                          its waves' weight statistics
//   batch_stats_kernel     eight waves per instance reduce its weight statistics
//   batch_wsum_kernel      persistent over all instances' steps (four delta_u rows each)
//   batch_apply_kernel     one workgroup per instance applies and advances
// Every stage calls the same device bodies as the one-instance kernels, so an
// instance's results are bit-identical alone and inside a batch (for the same
// lanes-per-sample).  Unlike the one-instance launches, the stages are separate
// kernels rather than last-arrival tails: a batch has too many tiles and rows for a
// device-scope fence on each.
#include <hip/hip_runtime.h>

#include "batch.h"
#include "stages.h"

namespace mppi {

__global__ void batch_reset_kernel(BatchHeader* hdr)
{
    if (threadIdx.x == 0) hdr->next_item = 0u;
}

template <int L, int U>
__device__ __forceinline__ void batch_tile(const InstanceDesc& D, int k0, const float4* obs_lds)
{
    const int k = k0 + (int)threadIdx.x / L, q = (int)threadIdx.x % L;
    const float S = D.rp.mp.lag
        ? rollout_sample<L, U, true, false>(D.rp, D.x_hat, D.x_ref, D.u_nom, D.du, D.S, nullptr,
                                            obs_lds, k, q)
        : rollout_sample<L, U, false, false>(D.rp, D.x_hat, D.x_ref, D.u_nom, D.du, D.S, nullptr,
                                             obs_lds, k, q);
    // the tile starts at sample k0 = (tile index) * blockDim / L: the same waves as
    // a one-instance launch of this workgroup size
    write_wave_stat(D.stat + ((k0 * L + (int)threadIdx.x) >> 6),
                    wave_sums(S, k, q, k < D.rp.K, D.lambda), false);
}

// Four waves per SIMD for the plain obstacle loop (at most 128 VGPRs: a few spill
// slots, 3% more throughput than three waves); the unrolled loop keeps its registers.
template <int U>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(U == 1 ? 4 : 1)))
void batch_rollout_kernel(BatchHeader* hdr, const InstanceDesc* __restrict__ descs,
                          const WorkItem* __restrict__ items)
{
    extern __shared__ float4 obs_lds[];
    __shared__ int s_item;
    const int n_items = __builtin_amdgcn_readfirstlane(hdr->n_items);
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&hdr->next_item, 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();                       // s_item is rewritten next iteration
        if (it >= n_items) return;             // uniform: every wave leaves together
        const int inst = __builtin_amdgcn_readfirstlane(items[it].inst);
        const int k0 = __builtin_amdgcn_readfirstlane(items[it].k0);
        const InstanceDesc& D = descs[inst];
        stage_obstacles(obs_lds, D.obs, D.rp.M, D.x_hat[0], D.x_hat[1], D.x_hat[2],
                        D.rp.cp.margin);
        __syncthreads();
        switch (__builtin_amdgcn_readfirstlane(D.lanes)) {   // uniform per item
        case 1: batch_tile<1, U>(D, k0, obs_lds); break;
        case 2: batch_tile<2, U>(D, k0, obs_lds); break;
        case 4: batch_tile<4, U>(D, k0, obs_lds); break;
        default: batch_tile<8, U>(D, k0, obs_lds); break;
        }
        __syncthreads();                       // LDS is restaged for the next item
    }
}

__global__ __launch_bounds__(64 * kStatParts) void batch_stats_kernel(const BatchHeader* __restrict__ hdr,
                                                        const InstanceDesc* __restrict__ descs)
{
    const int i = blockIdx.x;
    if (i >= hdr->n_inst) return;
    const InstanceDesc& D = descs[i];
    const StatSums t = reduce_stat_parts<8>(D.stat, D.W, D.lambda);
    if (threadIdx.x == 0) write_stat_diag(t, D.lanes, D.diag);
}

// Persistent over every instance's steps (four rows each); the first step of up to
// kWsumLdsInstances instances is staged in LDS once, so that finding a step's instance (a
// binary search) costs LDS reads rather than dependent global loads; larger batches
// search the descriptors themselves.
constexpr int kWsumLdsInstances = 4096;

__global__ __launch_bounds__(kSumThreads) void batch_wsum_kernel(const BatchHeader* __restrict__ hdr,
                                                                 const InstanceDesc* __restrict__ descs)
{
    __shared__ int step0[kWsumLdsInstances];
    const int n_steps = hdr->n_rows >> 2, n_inst = hdr->n_inst;
    const bool staged = n_inst <= kWsumLdsInstances;
    if (staged)
        for (int i = threadIdx.x; i < n_inst; i += blockDim.x) step0[i] = descs[i].row0 >> 2;
    __syncthreads();
    for (int st = blockIdx.x; st < n_steps; st += gridDim.x) {
        int lo = 0, hi = n_inst - 1;           // last instance whose steps start at or before st
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((staged ? step0[mid] : descs[mid].row0 >> 2) <= st) lo = mid; else hi = mid - 1;
        }
        const InstanceDesc& D = descs[lo];
        update_sum_step4(D.S, D.du, D.rp.K, D.rp.ld, D.lambda, D.u_nom, D.u_upd, D.diag,
                         st - (D.row0 >> 2));
        __syncthreads();                       // the step's LDS partials are reused
    }
}

__global__ void batch_apply_kernel(const BatchHeader* __restrict__ hdr,
                                   const InstanceDesc* __restrict__ descs)
{
    const int i = blockIdx.x;
    if (i >= hdr->n_inst) return;
    const InstanceDesc& D = descs[i];
    apply_shift_block(D.rp.mp, D.x_hat, D.u_upd, D.u_nom, D.u_apply, D.rp.N,
                      make_float4(D.u_init[0], D.u_init[1], D.u_init[2], D.u_init[3]), D.alpha,
                      D.diag);
}

// ---------------------------------------------------------------------------

bool valid_batch_launch(const BatchLaunch& c)
{
    return (c.block == 64 || c.block == 128 || c.block == 256) &&
           (c.lanes == 0 || c.lanes == 1 || c.lanes == 2 || c.lanes == 4 || c.lanes == 8) &&
           (c.unroll == 1 || c.unroll == 4) && c.blocks_per_cu >= 1 && c.blocks_per_cu <= 16;
}

hipError_t launch_batch_rollout(BatchHeader* hdr, const InstanceDesc* descs, const WorkItem* items,
                                int cu_count, int lds_bytes, const BatchLaunch& c,
                                hipStream_t stream)
{
    if (!valid_batch_launch(c)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, stream, hdr);
    const dim3 grid(cu_count * c.blocks_per_cu), block(c.block);
#define MPPI_BATCH_ROLLOUT(U) \
    hipLaunchKernelGGL((batch_rollout_kernel<U>), grid, block, lds_bytes, stream, hdr, descs, items)
    if (c.unroll == 4)
        MPPI_BATCH_ROLLOUT(4);
    else
        MPPI_BATCH_ROLLOUT(1);
#undef MPPI_BATCH_ROLLOUT
    return hipGetLastError();
}

hipError_t launch_batch(BatchHeader* hdr, const InstanceDesc* descs, const WorkItem* items,
                        int n_cap, int cu_count, int lds_bytes, const BatchLaunch& c,
                        hipStream_t stream)
{
    hipError_t e = launch_batch_rollout(hdr, descs, items, cu_count, lds_bytes, c, stream);
    if (e != hipSuccess) return e;
    return launch_batch_tail(hdr, descs, n_cap, cu_count, stream);
}

hipError_t launch_batch_tail(BatchHeader* hdr, const InstanceDesc* descs, int n_cap, int cu_count,
                             hipStream_t stream)
{
    hipLaunchKernelGGL(batch_stats_kernel, dim3(n_cap), dim3(64 * kStatParts), 0, stream, hdr,
                       descs);
    hipLaunchKernelGGL(batch_wsum_kernel, dim3(cu_count * 4), dim3(kSumThreads), 0, stream, hdr,
                       descs);
    hipLaunchKernelGGL(batch_apply_kernel, dim3(n_cap), dim3(256), 0, stream, hdr, descs);
    return hipGetLastError();
}

}  // namespace mppi
