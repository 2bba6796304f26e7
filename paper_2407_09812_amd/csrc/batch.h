// Device-side descriptors of a batch of uneven MPPI instances and the launchers of
// the batched kernels (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mppi.h"
#include "model.h"

namespace mppi {

// One instance of a batch, in device memory.  Scratch slices (du, S, w, u_upd, diag)
// point into the batch arena; the other pointers are the caller's.
struct InstanceDesc {
    RolloutParams rp;            // model, cost, noise, M, K, N, ld
    float lambda;
    float alpha;                 // warm-start advance per update, (0, 1]
    float u_init[4];
    int row0;                    // first weighted-sum row of this instance (4 N rows)
    int lanes;                   // lanes per sample (1, 2, 4, 8)
    const float* x_hat;
    const float* x_ref;
    const mppi_obstacle* obs;
    float* u_nom;
    float* u_apply;
    mppi_diag* diag;
    float* du;                   // [N][4][ld]
    float* S;                    // [ld]
    float* u_upd;                // [N][4]
    WaveStat* stat;              // [W] weight statistics of the rollout waves
    int W;                       // waves of its tiles: (sample tiles) * block / 64
};

// A tile of consecutive samples of one instance: the unit the persistent rollout
// kernel takes from the shared queue.
struct WorkItem {
    int inst;
    int k0;
};

struct BatchHeader {
    int n_inst;
    int n_items;
    int n_rows;
    unsigned int next_item;      // work-queue head, reset by batch_reset_kernel
};

// Launch shape of the batched rollout: `block` threads per workgroup, `lanes` per
// sample (0: chosen per instance at planning), obstacle loop `unroll`,
// `blocks_per_cu` persistent workgroups per CU.
struct BatchLaunch {
    int block, lanes, unroll, blocks_per_cu;
};

bool valid_batch_launch(const BatchLaunch& c);

// All five stages on `stream`: queue reset, persistent rollouts (with the waves'
// weight statistics), per-instance statistics reduction, persistent weighted sum,
// per-instance apply and advance.  Grid sizes depend only on (cu_count, n_cap, cfg),
// so the sequence can be captured once and replayed.
hipError_t launch_batch(BatchHeader* hdr, const InstanceDesc* descs, const WorkItem* items,
                        int n_cap, int cu_count, int lds_bytes, const BatchLaunch& cfg,
                        hipStream_t stream);
// The statistics, weighted-sum and apply stages.
hipError_t launch_batch_tail(BatchHeader* hdr, const InstanceDesc* descs, int n_cap, int cu_count,
                             hipStream_t stream);
// Only the reset and the rollout stage (autotuning).
hipError_t launch_batch_rollout(BatchHeader* hdr, const InstanceDesc* descs, const WorkItem* items,
                                int cu_count, int lds_bytes, const BatchLaunch& cfg,
                                hipStream_t stream);

}  // namespace mppi
