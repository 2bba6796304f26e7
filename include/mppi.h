/*
 * mppi.h -- C ABI of libmppi, an MI355X (gfx950) implementation of one Model
 * Predictive Path Integral (MPPI) update for a quadrotor, after arXiv 2407.09812
 * ("MPPI control for agile UAVs", Algorithm 1 and Sec. III).
 *
 * One update (Algorithm 1, loop body) takes the state estimate x_hat, the warm-start
 * nominal sequence u_nom (N x 4), a reference trajectory and an obstacle list, and:
 *   1. draws K perturbation sequences delta_u ~ N(0, diag(sigma^2))      Sec. III-A, Eq. (2)
 *   2. rolls each through the quadrotor model with its rate controller,
 *      allocation, rotor saturation and (optionally) rotor lag, by RK4     Eqs. (2), (6)-(13)
 *   3. scores each rollout (input, input-change, tracking, obstacles)     Eqs. (3), (16)-(22)
 *   4. turns costs into softmin weights with temperature lambda           Eq. (4)
 *   5. forms u_nom += sum_k w_k delta_u^k                                 Eq. (5)
 *   6. emits u_nom_0 (and the feasible [F_clip, omega_clip] at x_hat,
 *      Eqs. (12)-(15)), shifts u_nom by one step and refills the last
 *      slot with u_init                                                   Algorithm 1
 *      -- or, when updates come faster than the prediction step, advances
 *      u_nom by that fraction of a step by linear interpolation         Sec. IV-B
 * Upstream of an update, mppi_predict moves the state estimate forward over the
 * computation delay with the command being executed                      Sec. IV-E
 *
 * Conventions
 *  - Every function returns mppi_status: MPPI_OK (0) or a negative error code.
 *    No C++ exception crosses the ABI.  mppi_last_error() gives the text of the
 *    last error on a context (HIP error strings included).
 *  - Pointers documented as "device" are HIP device pointers (for example from
 *    torch tensors' data_ptr()); the library never frees or retains them.  Pointers
 *    documented as "host" are read during the call only.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  All device
 *    work is enqueued asynchronously on it; nothing on the update path allocates
 *    memory or synchronises the host.  Scratch is allocated by mppi_reserve().
 *  - State layout (17 floats): [p(3) m, q(4) unit quaternion w-first (body to
 *    world, Hamilton), v(3) m/s, omega(3) rad/s body frame, T(4) rotor thrusts N].
 *    Control (4 floats): [F_t N, omega_d(3) rad/s].  Reference rows (13 floats):
 *    [p, q, v, omega].  World z points up; gravity is (0, 0, -g).
 *  - Arithmetic on the device is IEEE binary32 (FMA contraction allowed).
 *  - One context per host thread.  Calls that share a context's scratch on
 *    different streams must be ordered by the caller.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mppi_status;

enum {
    MPPI_OK = 0,
    MPPI_E_INVALID_ARG = -1,     /* bad size, parameter or NULL pointer               */
    MPPI_E_NONFINITE_INPUT = -2, /* NaN/Inf in a host-side parameter                  */
    MPPI_E_ALL_NONFINITE = -3,   /* every rollout cost non-finite: u_nom left as is   */
    MPPI_E_BUDGET = -4,          /* request larger than the server's memory budget    */
    MPPI_E_OOM = -5,             /* device allocation failed                          */
    MPPI_E_HIP = -6,             /* HIP runtime error (see mppi_last_error)           */
    MPPI_E_PENDING = -7,         /* result not ready yet                              */
    MPPI_E_CAPACITY = -8         /* request exceeds the reserved scratch (reserve)    */
};

enum { MPPI_NX = 17, MPPI_NU = 4, MPPI_NREF = 13 };
enum { MPPI_SPHERE = 0, MPPI_VCYLINDER = 1 };
enum { MPPI_N_MAX = 4096, MPPI_M_MAX = 2048 };

/* Vehicle model, Sec. III-B and Table I.  tau_m = 0 selects the paper's
 * algebraic rotor model (clipped thrusts act at once, Eq. (13)); tau_m > 0 adds a
 * first-order rotor lag T' = (T_cmd - T) / tau_m.  k_rate = 0 selects the
 * rate-controller gain 1/dt of Eq. (8).  w_xy_max / w_z_max > 0 clamp the body
 * rates of the applied output only (Sec. IV-A safety limits). */
typedef struct mppi_vehicle {
    float mass;
    float J[3];
    float arm_l;
    float c_tf;
    float g;
    float T_min, T_max;
    float tau_m;
    float k_rate;
    float w_xy_max, w_z_max;
} mppi_vehicle;

/* Cost, Eqs. (16)-(22) and Table II: input weights R, input-change weights R_d,
 * tracking weights (c_p, c_v, c_q, c_w) with the attitude term c_q * d_q^2,
 * d_q = 1 - <q, q_ref>^2 (Eq. (21)); obstacle term per state
 * obs_collision * [inside any obstacle] + obs_w * sum_i max(0, r_i + obs_margin - d_i)^2. */
typedef struct mppi_cost {
    float c_p, c_v, c_q, c_w;
    float R[4];
    float R_d[4];
    float obs_margin, obs_w, obs_collision;
} mppi_cost;

/* Obstacle (Sec. IV-D): sphere (distance |p - c|) or vertical cylinder of
 * infinite height (distance |(p - c)_xy|), radius r. 20 bytes. */
typedef struct mppi_obstacle {
    int32_t type;
    float c[3];
    float r;
} mppi_obstacle;

/* Per-update problem (Algorithm 1 parameters).  sigma holds per-dimension standard
 * deviations of delta_u.  Noise is Philox4x32-10 with key (seed low 32 bits,
 * vehicle_id) and counter (k, j, t, seed high 32 bits), Box-Muller on the pairs
 * of uniforms ((w >> 9) + 0.5) 2^-23; t is the vehicle's update index. */
typedef struct mppi_solve {
    int32_t K;         /* rollouts, >= 1                                  */
    int32_t N;         /* horizon steps, 1..MPPI_N_MAX                    */
    float dt;          /* prediction step, s, > 0                         */
    float lambda;      /* softmin temperature, > 0                        */
    float sigma[4];    /* noise standard deviations, >= 0                 */
    float u_init[4];   /* refill value of the last slot after the shift   */
    uint64_t seed;
    uint32_t vehicle_id;
    uint32_t t;
    float dt_ctrl;     /* time between updates, s, 0 <= dt_ctrl <= dt; 0 means dt.
                          The warm start advances by alpha = dt_ctrl / dt of a step
                          (Sec. IV-B); alpha = 1 is Algorithm 1's shift   */
    uint32_t reserved; /* set to 0                                         */
} mppi_solve;

/* Diagnostics written by the device (all rollouts of one update). */
typedef struct mppi_diag {
    float rho;         /* min_k S_k over finite costs                     */
    float eta;         /* sum_k exp(-(S_k - rho) / lambda)                */
    float ess;         /* effective sample size 1 / sum_k w_k^2           */
    int32_t argmin;    /* smallest k with S_k = rho                       */
    int32_t n_finite;  /* number of finite costs                          */
    int32_t status;    /* MPPI_OK or MPPI_E_ALL_NONFINITE                 */
    int32_t lanes;     /* lanes per sample the rollouts ran with          */
    float reserved;
} mppi_diag;

typedef struct mppi_ctx mppi_ctx;

/* Create a context on HIP device `device`.  Allocates no scratch yet. */
mppi_status mppi_create(int device, mppi_ctx **out);
mppi_status mppi_destroy(mppi_ctx *ctx);

/* Make sure the context's scratch holds an update with up to K rollouts, N steps
 * and M obstacles (delta_u [N][4][K] floats, costs and weights [K]).  The only call
 * that allocates; it synchronises the device when it grows. */
mppi_status mppi_reserve(mppi_ctx *ctx, int32_t K, int32_t N, int32_t M);

/* Host-only argument check used by every entry point (no device access):
 * MPPI_E_INVALID_ARG for K < 1, N < 1 or > MPPI_N_MAX, M < 0 or > MPPI_M_MAX,
 * dt <= 0, lambda <= 0, sigma < 0, mass or inertia <= 0, T_min > T_max, tau_m < 0;
 * MPPI_E_NONFINITE_INPUT for NaN/Inf parameters. */
mppi_status mppi_validate(const mppi_vehicle *veh, const mppi_cost *cost,
                          const mppi_solve *solve, int32_t M);

/* One full MPPI update (Algorithm 1 loop body), asynchronous on `stream`.
 *   x_hat    device, 17 floats                     state estimate
 *   x_ref    device, (N+1) x 13 floats             reference rows j = 0..N
 *   obs      device, M obstacles (may be NULL if M = 0); centres and radii must be
 *            finite (they are read on the device only: a non-finite one gives
 *            unspecified costs, never an access outside the inputs)
 *   u_nom    device, N x 4 floats, in/out          warm start -> updated and shifted
 *   u_apply  device, 8 floats, out                 [u_nom_0 after the update (4),
 *                                                   F_clip, omega_clip at x_hat (4)]
 *            (or pinned host memory through its mppi_device_address, so that the
 *            command reaches the host without a copy)
 *   diag     device, one mppi_diag, out (may be NULL)
 * When every cost is non-finite the device leaves u_nom unchanged, writes the
 * current u_nom_0 to u_apply and sets diag->status = MPPI_E_ALL_NONFINITE.
 * Returns MPPI_E_CAPACITY if K, N or M exceed the reserved scratch. */
mppi_status mppi_update(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh,
                        const mppi_cost *cost, const mppi_solve *solve,
                        const float *x_hat, const float *x_ref,
                        const mppi_obstacle *obs, int32_t M,
                        float *u_nom, float *u_apply, mppi_diag *diag);

/* --- an update that allocates nothing --------------------------------------------- */

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  mppi_update with its scratch
 * (delta_u, costs, the rollout waves' weight statistics, the copy of the warm start,
 * and the diagnostics when diag is NULL) carved out of one static device array of
 * MPPI_STATIC_SCRATCH_BYTES on each GPU, whose address mppi_create takes on its device;
 * the array is held until the process ends.  Needs no mppi_reserve and calls no
 * allocating routine.  Arguments, results (bit for bit those of mppi_update in the same
 * launch shape) and errors are mppi_update's, except that it always runs the stored
 * form (a shape stored with fused = 1 runs with fused = 0) and that it returns
 * MPPI_E_CAPACITY when the update needs more than the array holds: 16 N ld + 4 ld +
 * 32 W + 16 N + 32 bytes, each part rounded up to 256, with ld = K rounded up to 64 and
 * W the rollout launch's waves (ceil(K / 64) x lanes for the wave-specialised shape) --
 * K = 4096, N = 100 takes 6.6 MB.  MPPI_E_HIP if the array's address could not be taken.
 * Nothing in the array has to start at zero: each call writes what it reads.  Every
 * call on one GPU uses that GPU's one array, which keeps the last call's contents, so
 * calls that overlap on one GPU (other streams, contexts or threads) race: order them. */
enum { MPPI_STATIC_SCRATCH_BYTES = 16 << 20 };
mppi_status mppi_update_static(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh,
                               const mppi_cost *cost, const mppi_solve *solve,
                               const float *x_hat, const float *x_ref,
                               const mppi_obstacle *obs, int32_t M,
                               float *u_nom, float *u_apply, mppi_diag *diag);

/* --- the update's stages, exposed for stage-by-stage checking ------------------ */

/* Rollouts and costs (Eqs. (2), (3)): writes delta_u [N][4][ld] (device, row
 * (j, d) holds samples k = 0..K-1 contiguously, ld >= K), S [K] (device) and, if
 * states is not NULL, the trajectories [N+1][17][ld] (device). */
mppi_status mppi_rollout(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh,
                         const mppi_cost *cost, const mppi_solve *solve,
                         const float *x_hat, const float *x_ref,
                         const mppi_obstacle *obs, int32_t M, const float *u_nom,
                         float *du, int32_t ld, float *S, float *states);

/* Softmin weights (Eq. (4)) of S [K] (device): w [K] (device), diag (device). */
mppi_status mppi_weights(mppi_ctx *ctx, void *stream, int32_t K, const float *S,
                         float lambda, float *w, mppi_diag *diag);

/* Weighted update (Eq. (5)): u_out[j][d] = u_in[j][d] + sum_k w[k] du[j][d][k]
 * (all device; du as written by mppi_rollout with leading dimension ld).  If diag
 * is not NULL and diag->status != MPPI_OK, u_out = u_in. u_out may alias u_in. */
mppi_status mppi_weighted_sum(mppi_ctx *ctx, void *stream, int32_t K, int32_t N,
                              const float *w, const float *du, int32_t ld,
                              const float *u_in, float *u_out, const mppi_diag *diag);

/* Apply and advance (Algorithm 1 after Eq. (5); Eqs. (12)-(15); Sec. IV-B):
 * u_apply[0..3] = u_upd[0], u_apply[4..7] = [F_clip, omega_clip] at x_hat; u_nom[j] =
 * (1 - alpha) u_upd[j] + alpha u_upd[j+1] with u_upd[N] = solve->u_init and
 * alpha = solve->dt_ctrl / solve->dt (alpha = 1, or dt_ctrl = 0: exactly
 * u_nom[j] = u_upd[j+1], u_nom[N-1] = u_init).  Device pointers; u_nom must not
 * alias u_upd (MPPI_E_INVALID_ARG). */
mppi_status mppi_apply_shift(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh,
                             const mppi_solve *solve, const float *x_hat,
                             const float *u_upd, float *u_nom, float *u_apply);

/* Delay compensation by prediction (Sec. IV-E): x_out = the state reached from x_hat
 * after `delay` seconds while the command u_hold ([F_t, omega_d], the one being
 * executed during the computation) is held: ceil(delay / dt) equal steps of length
 * h <= dt, each the rate controller of Eqs. (8)-(12) at the step's start (gain 1/dt,
 * or veh->k_rate) followed by one RK4 step of length h.  delay = 0 copies x_hat;
 * delay = dt is mppi_plant_step.  Device pointers (17, 4, 17 floats); x_out may
 * alias x_hat.  MPPI_E_INVALID_ARG for dt <= 0, delay < 0 or delay > 4096 dt;
 * MPPI_E_NONFINITE_INPUT for non-finite dt or delay. */
mppi_status mppi_predict(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh, float dt,
                         float delay, const float *x_hat, const float *u_hold, float *x_out);

/* The noise of one update as the rollout kernel draws it: du [N][4][ld] (device). */
mppi_status mppi_noise(mppi_ctx *ctx, void *stream, const mppi_solve *solve,
                       float *du, int32_t ld);

/* Raw Philox4x32-10 on the device: out[i] = philox(ctr[i], key[i]) for n
 * counters (ctr, out: n x 4 uint32; key: n x 2 uint32; all device). */
mppi_status mppi_philox(mppi_ctx *ctx, void *stream, int32_t n, const uint32_t *ctr,
                        const uint32_t *key, uint32_t *out);

/* One noise-free model step of the plant, x_out = x + f_RK4(x, u, dt) with the
 * rate controller inside (Eq. (2), last line): x, u, x_out device (17, 4, 17). */
mppi_status mppi_plant_step(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh, float dt,
                            const float *x, const float *u, float *x_out);

/* --- launch shape and autotuning ----------------------------------------------- */

/* Shape of the rollout launch: `lanes` consecutive lanes share one sample and divide
 * its obstacle tests (1, 2, 4, 8); `block` threads per workgroup (64, 128, 256);
 * obstacle loop unrolled `unroll` times (1, 4).  fused = 1 selects the single-pass
 * update (Eqs. (4), (5) without delta_u in memory): each wave of the rollout launch
 * ends by forming its own minimum cost rho_w, its weights relative to it and its
 * partial sums of e_k delta_u (the perturbations regenerated from the counter-based
 * noise), and one merge launch rescales the partials by exp(-(rho_w - rho)/lambda);
 * fused = 0 stores delta_u and runs the weights and the GEMV-shaped weighted sum.
 * pipe = 1 (M <= 1536; either fused value) runs the rollouts wave-specialised: per 64
 * samples one workgroup of 4 + lanes waves -- noise, body rates, attitude, translation
 * and tracking cost, and `lanes` obstacle-cost waves -- handing chunks of steps over
 * through LDS (block is then 64 (4 + lanes) and the field is ignored); the arithmetic
 * of pipe = 0 with the same lanes and unroll (costs may differ in the last bits where
 * the compiler fuses operations differently), with a shorter per-step critical path.
 * Every shape computes the same update up to rounding: the order of the obstacle-
 * penalty additions depends on lanes, and the order of the weighted sums on fused. */
typedef struct mppi_launch_config {
    int32_t block;
    int32_t lanes;
    int32_t unroll;
    int32_t fused;
    int32_t pipe;
} mppi_launch_config;

/* The shape mppi_update / mppi_rollout use for (K, N, M): a stored entry for the
 * size class (powers of two of K, N and M), else a heuristic: the wave-specialised
 * rollouts (pipe = 1, stored form) with 1, 2 or 4 lanes for M < 16, < 64 or more (with
 * 4 or 8 lanes the obstacle waves cull by the box of each chunk of steps), and beyond
 * the pipe's obstacle limit the one-wave kernel aiming at one wave per SIMD.
 * Host-only. */
mppi_status mppi_get_config(const mppi_ctx *ctx, int32_t K, int32_t N, int32_t M,
                            mppi_launch_config *out);
/* Store a shape for the size class of (K, N, M).  MPPI_E_INVALID_ARG for a shape
 * outside the lists above.  Host-only. */
mppi_status mppi_set_config(mppi_ctx *ctx, int32_t K, int32_t N, int32_t M,
                            const mppi_launch_config *cfg);
/* Time every shape, both variants, on these inputs (reps runs each of the rollouts
 * through the updated sequence, HIP events on `stream`), store the fastest for the
 * size class and return it in best.  Uses the context's
 * scratch (mppi_reserve first) and synchronises the stream; a set-up call, not for
 * the update loop. */
mppi_status mppi_autotune(mppi_ctx *ctx, void *stream, const mppi_vehicle *veh,
                          const mppi_cost *cost, const mppi_solve *solve, const float *x_hat,
                          const float *x_ref, const mppi_obstacle *obs, int32_t M,
                          const float *u_nom, int32_t reps, mppi_launch_config *best);

/* --- batched updates ------------------------------------------------------------ */

/* One instance of a batch: its own model, cost, problem and device buffers (the same
 * meaning and layouts as the arguments of mppi_update).  diag may be NULL. */
typedef struct mppi_request {
    mppi_vehicle veh;
    mppi_cost cost;
    mppi_solve solve;
    const float *x_hat;
    const float *x_ref;
    const mppi_obstacle *obs;
    int32_t M;
    float *u_nom;
    float *u_apply;
    mppi_diag *diag;
} mppi_request;

/* Launch shape of the batched rollout: workgroup size (64, 128, 256), lanes per
 * sample (1, 2, 4, 8 for every instance, or 0 = per instance: as many as keep the
 * whole batch near one wave per SIMD, capped by the instance's obstacle count),
 * obstacle-loop unroll (1, 4), persistent workgroups per compute unit (1..16), and
 * whether to replay a captured HIP graph (1) or launch the kernels one by one (0).
 * Each instance reports the lanes it ran with in its mppi_diag. */
typedef struct mppi_batch_config {
    int32_t block;
    int32_t lanes;
    int32_t unroll;
    int32_t blocks_per_cu;
    int32_t use_graph;
} mppi_batch_config;

/* Grow the batch scratch (delta_u, costs, weights, descriptors, work queue) to hold
 * this list of requests.  The only batch call that allocates; synchronises the device
 * when it grows. */
mppi_status mppi_batch_reserve(mppi_ctx *ctx, const mppi_request *reqs, int32_t n);

/* MPPI updates of n independent instances with uneven K, N and M in one launch
 * sequence on `stream` (Algorithm 1 loop body for each; the same results, bit for
 * bit, as mppi_update with the same lanes per sample, stored form, pipe = 0, see
 * mppi_diag.lanes).  A persistent rollout kernel
 * takes (instance, sample tile) items longest first from a device queue; weights,
 * weighted sums and shifts follow per instance.  With use_graph the sequence is a HIP
 * graph captured once per launch shape and replayed.  Host-side planning is copied
 * from pinned memory on `stream`; the call waits only for the previous batch's copy.
 * MPPI_E_CAPACITY if the list does not fit the reserved scratch. */
mppi_status mppi_batch_update(mppi_ctx *ctx, void *stream, const mppi_request *reqs, int32_t n);

/* Time every batched launch shape on this list (reps rollout passes each), keep the
 * fastest as the context's batch shape and return it.  Synchronises the stream. */
mppi_status mppi_batch_autotune(mppi_ctx *ctx, void *stream, const mppi_request *reqs, int32_t n,
                                int32_t reps, mppi_batch_config *best);
/* The context's batch shape; until set or tuned it is {256, 0, 1, 8, 1} (lanes per
 * instance, the plain obstacle loop, eight persistent workgroups per compute unit, the
 * graph replayed). */
mppi_status mppi_batch_get_config(const mppi_ctx *ctx, mppi_batch_config *out);
mppi_status mppi_batch_set_config(mppi_ctx *ctx, const mppi_batch_config *cfg);

/* --- serving ---------------------------------------------------------------------- */

/* A request loop for many vehicles (continuous batching).  The server owns each
 * vehicle's warm-start sequence on the device (N_max x 4 floats, initialised to
 * u_init) and its update counter t; requests carry the state estimate, reference and
 * obstacles on the host and are copied at submit.  A worker thread admits queued
 * requests whenever one of n_streams slots is free and the request fits that slot's
 * share of budget_bytes (its delta_u, costs, weights and inputs), one request per
 * vehicle in flight (the next update starts from the previous result), in arrival
 * order, and launches them as one batch (mppi_batch_update) on the slot's stream --
 * a lone request as mppi_update, whose default shape runs the wave-specialised
 * rollouts (each slot reserves one K_max x N_max x M_max instance for it, beyond
 * budget_bytes); batches on different slots overlap on the device.  A request with horizon N uses
 * the first N rows of its vehicle's warm start and advances them.  With a delay, the
 * request's state estimate is first moved forward by mppi_predict's model steps with
 * the vehicle's last served command held (u_init before its first request); each
 * served command is recorded for the vehicle's next request (Sec. IV-E). */
typedef struct mppi_server mppi_server;

typedef struct mppi_server_cfg {
    int32_t device;
    int32_t n_vehicles;
    int32_t K_max, N_max, M_max;   /* per request                                   */
    int32_t n_streams;             /* concurrent batches, >= 1                      */
    int32_t max_batch;             /* requests per batch, >= 1                      */
    int32_t reserved;
    int64_t budget_bytes;          /* device scratch for in-flight requests         */
    mppi_vehicle veh;
    mppi_cost cost;
    float u_init[4];
} mppi_server_cfg;

typedef struct mppi_server_request {
    uint32_t vehicle_id;           /* < n_vehicles                                  */
    int32_t K, N, M;
    float dt, lambda;
    float sigma[4];
    float dt_ctrl;                 /* as mppi_solve.dt_ctrl (0: shift by a step)   */
    float delay;                   /* s to predict x_hat forward before the update;
                                      0: none; < 0: the running median of the last
                                      256 submit-to-result latencies              */
    uint64_t seed;
    const float *x_hat;            /* host, 17 floats                               */
    const float *x_ref;            /* host, (N+1) x 13 floats                       */
    const mppi_obstacle *obs;      /* host, M obstacles                             */
} mppi_server_request;

typedef struct mppi_server_result {
    uint64_t ticket;
    uint32_t vehicle_id;
    uint32_t t;                    /* the vehicle's update index this request used  */
    float u_apply[8];              /* as mppi_update's u_apply                      */
    mppi_diag diag;
    double submit_s, launch_s, done_s;   /* server clock, seconds since creation    */
    int32_t K, N;
    float delay;                   /* delay the state estimate was predicted over  */
    int32_t pipe;                  /* 1: run alone by mppi_update with pipe = 1;
                                      0: by mppi_batch_update or the one-wave kernel */
} mppi_server_result;

typedef struct mppi_server_stats {
    int64_t submitted, completed, batches, rejected;
    int64_t rollout_steps;         /* sum of K N over completed requests            */
    int64_t max_in_flight;
    double busy_s;                 /* time with at least one batch in flight        */
} mppi_server_stats;

mppi_status mppi_server_create(const mppi_server_cfg *cfg, mppi_server **out);
/* Waits for queued and in-flight requests, then frees everything. */
mppi_status mppi_server_destroy(mppi_server *srv);
/* Shape of the batched launches on every slot (see mppi_batch_config). */
mppi_status mppi_server_set_batch_config(mppi_server *srv, const mppi_batch_config *cfg);
/* Queue a request (inputs are copied).  MPPI_E_INVALID_ARG for bad parameters or
 * sizes above the server's maxima, MPPI_E_BUDGET if it can never fit a slot. */
mppi_status mppi_server_submit(mppi_server *srv, const mppi_server_request *req,
                               uint64_t *ticket);
/* Result of a finished request (then forgotten), or MPPI_E_PENDING. */
mppi_status mppi_server_poll(mppi_server *srv, uint64_t ticket, mppi_server_result *out);
/* Block until the request has finished, then as mppi_server_poll. */
mppi_status mppi_server_wait(mppi_server *srv, uint64_t ticket, mppi_server_result *out);
/* Block until nothing is queued or in flight. */
mppi_status mppi_server_drain(mppi_server *srv);
mppi_status mppi_server_stats_get(mppi_server *srv, mppi_server_stats *out);
double mppi_server_clock(const mppi_server *srv);
/* Warm starts, last served commands and update counters: size = n_vehicles x
 * (N_max x 4 + 4 floats) + n_vehicles uint32.
 * Both drain first; restore makes the next updates continue exactly (counter-based
 * noise). */
mppi_status mppi_server_snapshot(mppi_server *srv, void *host_buf, size_t *size);
mppi_status mppi_server_restore(mppi_server *srv, const void *host_buf, size_t size);

/* --- profiling ---------------------------------------------------------------- */

/* Device time of mppi_update's two launches -- rollout_ms: the rollouts with each
 * wave's weight statistics (reduced by the single pass's last workgroup); sum_ms: the
 * weighted sum (stored delta_u, whose workgroups reduce the statistics first, or the
 * single-pass partial sums) with the apply and advance -- and of mppi_batch_update's
 * rollout stage and remaining stages, measured
 * with HIP events on the call's stream while enabled.  While profiling, batches are
 * launched kernel by kernel (no graph replay) so that the events can bracket the
 * rollout stage. */
typedef struct mppi_profile {
    int64_t updates;
    double rollout_ms, sum_ms;
    int64_t batches;
    double batch_rollout_ms, batch_rest_ms;
    int64_t obstacle_tests;   /* sample-state-obstacle distance tests performed (both paths);
                                 obstacles out of every lane's reach in a wave are skipped */
} mppi_profile;

mppi_status mppi_profile_enable(mppi_ctx *ctx, int32_t on);
/* The device address of pinned host memory (allocated with hipHostMalloc, as pinned
 * tensors are), for small outputs the host reads right after the stream synchronises,
 * such as u_apply: the kernel writes them over the host link and no copy is queued.
 * Host-only; MPPI_E_INVALID_ARG for NULL or memory the runtime does not map. */
mppi_status mppi_device_address(const void *host_ptr, void **dev_ptr);
/* Waits for the recorded events, returns the totals since enable and resets them. */
mppi_status mppi_profile_read(mppi_ctx *ctx, mppi_profile *out);

const char *mppi_status_str(mppi_status s);
const char *mppi_last_error(const mppi_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_H */
