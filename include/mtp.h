/*
 * mtp.h -- C ABI of the MI355X (gfx950) Model Tensor Planning replan engine.
 *
 * One replan is the loop body of Alg. 2 of "Model Tensor Planning" (Le et al.,
 * arXiv 2505.01059) repeated n_iters times:
 *   sample the random multipartite graph Z (Def. 1) and P paths (Alg. 1);
 *   interpolate them (Def. 2 B-spline, Def. 3 Akima);
 *   draw G-1 local Gaussian samples around the mean and add the mean itself;
 *   roll every candidate out and sum its per-step cost (Eq. 1);
 *   keep the E cheapest, weight them by a softmax and refit mean / std.
 * The action is the first control of the cheapest candidate of the last
 * iteration.
 *
 * Conventions shared by every call:
 *   - Every call returns mtp_status; nothing throws, aborts or prints.
 *   - Arguments are validated before anything is enqueued; on error the object
 *     is unchanged and mtp_last_error() says why.  A failed HIP call returns
 *     MTP_ERR_DEVICE and the error sticks to the object until it is destroyed.
 *   - "d_" pointers are device memory on the current HIP device, "h_" pointers
 *     host memory.  The caller owns the workspace and the stream; both must
 *     outlive the plan.  The plan copies the config and its host tables at
 *     create and never allocates device memory itself (the batch and server
 *     objects below take caller workspaces too).
 *   - Work is enqueued asynchronously on the plan's stream; only calls that
 *     return host data (mtp_get_action, ...) synchronise that stream.
 *   - A plan is used by one host thread at a time.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit
 * seed, counter = (block, item, replan index r, tag << 16 | iteration k):
 *   tag 1 graph waypoints (item = layer, element w*n + j),
 *   tag 2 path indices    (item = tensor path p, element l),
 *   tag 3 local noise     (item = local sample g, element j*4*ceil(T/4) + t),
 * element e sits in word e % 4 of block e / 4.  Waypoints are
 * u_min + (u_max-u_min) * (w >> 8) * 2^-24, indices (w * W) >> 32, normals by
 * Box-Muller on word pairs (0,1) and (2,3).
 *
 * Candidate order (Alg. 2, stacking step): [local 0..G-2 | tensor paths
 * 0..P-1 | nominal mean], so B = P + G and index B-1 is the mean.
 */
#ifndef MTP_H_
#define MTP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTP_ABI_VERSION 3

typedef enum {
  MTP_OK = 0,
  MTP_ERR_INVALID_ARG = 1,  /* bad config or argument; nothing was enqueued      */
  MTP_ERR_UNSUPPORTED = 2,  /* valid but not built (e.g. chain length not instantiated) */
  MTP_ERR_WORKSPACE = 3,    /* workspace missing, too small or misaligned          */
  MTP_ERR_DEVICE = 4,       /* a HIP call failed; sticky until destroy             */
  MTP_ERR_BUSY = 5,         /* server full / budget exceeded; retry later          */
  MTP_ERR_NOT_READY = 6     /* no result available yet                             */
} mtp_status;

typedef enum {
  MTP_INTERP_BSPLINE = 0,  /* Def. 2, degree bspline_degree, uniform knots                  */
  MTP_INTERP_AKIMA = 1,    /* Def. 3, knots i/L                                             */
  MTP_INTERP_LINEAR = 2    /* straight lines between waypoints on knots i/(L-1) (Thm. 1)   */
} mtp_interp;

typedef enum {
  MTP_DYN_POINT_MASS = 0,    /* planar double integrator, d=4, n=2, semi-implicit Euler */
  MTP_DYN_CHAIN = 1,         /* planar n-link pendulum chain, d=2n, RK4                 */
  MTP_DYN_CHAIN_CONTACT = 2  /* chain + penalty ground contact + per-sample masses/friction */
} mtp_dynamics;

/*
 * Planner configuration (Alg. 2 inputs).  L = n_layers is the graph depth
 * (the paper's M), W = n_width the waypoints per layer (the paper's N).
 * n_gauss counts the local samples including the nominal mean (>= 1).
 *
 * task_params (host, copied at create), float32, per dynamics:
 *   POINT_MASS:    [goal_x, goal_y, goal_weight, obstacle_penalty, ctrl_weight,
 *                   n_obs, (cx, cy, r) * n_obs]
 *   CHAIN:         [gravity, goal_weight, ctrl_weight, target_x, target_y,
 *                   mass_1..mass_n, length_1..length_n]
 *   CHAIN_CONTACT: CHAIN's layout followed by [ground_y, k_contact, d_contact, v_slip];
 *                  its masses are ignored in favour of sample_params.
 * sample_params (host, copied at create; CHAIN_CONTACT only): R*B rows of
 *   [mass_1..mass_n, friction_coefficient], row r*B + b for candidate b under
 *   randomised model r; the candidate's cost is the mean over its R rollouts
 *   (online domain randomisation, Section 4).
 */
typedef struct {
  uint32_t abi_version;      /* MTP_ABI_VERSION */
  int32_t dynamics;          /* mtp_dynamics */
  int32_t interp;            /* mtp_interp */
  int32_t n_links;           /* chains: number of links (= ctrl_dim); point mass: 0 */
  int32_t state_dim;         /* d */
  int32_t ctrl_dim;          /* n */
  int32_t horizon;           /* T >= 1 */
  int32_t n_layers;          /* L: >= degree+1 (B-spline), >= 2 (Akima, linear), <= 16 */
  int32_t n_width;           /* W: 1..256 */
  int32_t n_tensor;          /* P >= 0 */
  int32_t n_gauss;           /* G >= 1 */
  int32_t n_elites;          /* E: 1..min(B, 4096) */
  int32_t n_iters;           /* K: 1..65535 CEM iterations per replan */
  int32_t bspline_degree;    /* p: 1..5 (B-spline only) */
  float temperature;         /* lambda > 0; +inf means uniform elite weights */
  float smoothing;           /* alpha in [0, 1) */
  float sigma_min;           /* >= 0, floor on the refitted std */
  float sigma_init;          /* >= 0, initial std and the std given to shifted-in steps */
  float u_min, u_max;        /* control box, u_min < u_max */
  float dt;                  /* > 0 */
  uint64_t seed;             /* Philox key */
  const float* task_params;  /* host */
  int32_t n_task_params;
  const float* sample_params;  /* host, CHAIN_CONTACT only, R*B*(n+1) floats */
  int32_t n_debug_states;    /* record x_{t+1} of candidates 0..n_debug_states-1 under every
                                randomised model (0 = off) */
  int32_t n_replicas;        /* R >= 1 randomised models per candidate (R > 1: CHAIN_CONTACT only);
                                0 is read as 1 */
  int32_t sample_wor;        /* 0: tensor path indices drawn with replacement (Alg. 1);
                                1: without replacement (Section 3.2), needs P <= W^L */
  int32_t diagnostics;       /* bit 0: record the cost entropy of every CEM iteration (Section 5.1) */
} mtp_config;

/*
 * Device views into a plan's workspace, for inspection and staged checks.
 * Layouts (sample index fastest):
 *   Z          float [L][W][n]
 *   I          uint8 [L][P]           path index of tensor path p at layer l
 *   U          float [T][n][ld_U]     control u_t,j of candidate b at U[(t*n+j)*ld_U + b]
 *   cost       float [B]              summed rollout cost (+inf if not finite)
 *   elite_idx  int32 [E]              ascending cost, ties by lower index
 *   elite_cost float [E]
 *   weights    float [E]              softmax weights of the elites
 *   mu, sigma  float [T][n]
 *   x0         float [d]              start state of the current replan
 *   action     float [n]
 *   X_dbg      float [R][T][d][n_debug_states] or NULL: x_{t+1} of candidates 0..n_debug_states-1
 *                                     under each of the R randomised models (R = 1 unless n_replicas > 1)
 *   entropy    float [K]              cost entropy H = -sum_b P_b log P_b, P = softmax(cost) over the
 *                                     finite costs, of every iteration of the last replan
 *                                     (written only when cfg.diagnostics bit 0 is set)
 */
typedef struct {
  void *Z, *I, *U, *cost, *elite_idx, *elite_cost, *weights, *mu, *sigma, *x0, *action, *X_dbg, *entropy;
  size_t ld_U;
} mtp_buffers;

typedef struct mtp_plan mtp_plan;

/* Bytes of device workspace a plan needs (256-byte aligned base required); 0 if cfg is invalid.
 * Sizes the buffers of Alg. 2's loop body: graph Z (Def. 1), paths I (Alg. 1),
 * candidates U, costs S (Eq. 1), elites, mean / std. */
size_t mtp_workspace_bytes(const mtp_config* cfg);

/* Check a config (Alg. 2's inputs: graph L x W of Def. 1, B, beta as counts,
 * T, alpha, lambda, sigma floor, E) without creating anything; on failure
 * writes a reason into `why` (NUL-terminated, at most why_len bytes; may be NULL). */
mtp_status mtp_validate_config(const mtp_config* cfg, char* why, size_t why_len);

/* Bytes of the per-replan (transient) buffers of one instance: graph, paths,
 * candidates, costs, elites.  A server lends this much from its pool to every
 * replan in flight; 0 if cfg is invalid. */
size_t mtp_transient_bytes(const mtp_config* cfg);

/* Bytes of the resident buffers of one instance (control block, start state,
 * warm-start mean / std, tables, per-sample parameters): what a server takes
 * from its pool for as long as the robot is registered; 0 if cfg is invalid. */
size_t mtp_resident_bytes(const mtp_config* cfg);

/* Alg. 2's initialisation: validate cfg, lay the plan out in the caller's
 * workspace, upload its tables (spline basis of Def. 2 / Def. 3, task and
 * sample parameters) on `hip_stream` (NULL = default stream) and initialise
 * mu = (u_min+u_max)/2, sigma = sigma_init, replan index 0. */
mtp_status mtp_plan_create(const mtp_config* cfg, void* d_workspace, size_t ws_bytes,
                           void* hip_stream, mtp_plan** out);

/* Alg. 2's planning step: the loop body (graph, paths, interpolation, local
 * samples, rollout and cost, top-E, softmax refit) n_iters times from start state d_x0 (d floats,
 * read by the replan's first kernel, so it must stay valid until that point in
 * stream order), after shifting the
 * warm-start mean/std forward by shift_steps (0 = no shift; the mean's last row is
 * held, the std's tail reset to sigma_init).  Uses the plan's replan counter as the
 * Philox replan index and increments it.  Asynchronous. */
mtp_status mtp_replan(mtp_plan* p, const float* d_x0, int32_t shift_steps);

/* Alg. 2's planning step as mtp_replan with an explicit replan index; the counter continues from replan_idx+1. */
mtp_status mtp_replan_at(mtp_plan* p, const float* d_x0, int32_t shift_steps, uint32_t replan_idx);

/* Alg. 2's output: the first control of the cheapest candidate of the last
 * iteration, the control the robot executes (n floats) copied to the host;
 * synchronises the stream. */
mtp_status mtp_get_action(mtp_plan* p, float* h_u);

/* Alg. 2's warm start between replans (mean and std carried over, shifted by
 * the next call): export / import it (device arrays of T*n floats) with the
 * replan counter, for checkpoint and resume.  get_state synchronises the stream. */
mtp_status mtp_get_state(const mtp_plan* p, float* d_mu, float* d_sigma, uint32_t* replan_idx);
mtp_status mtp_set_state(mtp_plan* p, const float* d_mu, const float* d_sigma, uint32_t replan_idx);

/* One stage of Alg. 2's loop body, for checks: run one stage of CEM iteration k of replan r on the
 * buffers as they stand (MTP_STAGE_ALL runs one whole iteration).  A test may write
 * a stage's inputs through mtp_get_buffers first.  x0 must have been set by a replan
 * or mtp_set_x0. */
typedef enum {
  MTP_STAGE_CANDIDATES = 0,  /* Z, I, U */
  MTP_STAGE_ROLLOUT = 1,     /* U -> cost (and X_dbg) */
  MTP_STAGE_TOPK = 2,        /* cost -> elite_idx, elite_cost, weights */
  MTP_STAGE_UPDATE = 3,      /* U, elites, weights -> mu, sigma, action */
  MTP_STAGE_ALL = 4
} mtp_stage;
mtp_status mtp_run_stage(mtp_plan* p, int32_t stage, uint32_t replan_idx, int32_t k);
/* The rollouts' start state x0 (Eq. 1) for mtp_run_stage, copied from device memory. */
mtp_status mtp_set_x0(mtp_plan* p, const float* d_x0);

/* How Alg. 2's planning step is launched (the arithmetic is the same): replay
 * a captured hipGraph (1, default) or launch kernels one by one (0). */
mtp_status mtp_set_graph_mode(mtp_plan* p, int32_t use_graph);

/* Measurement of Alg. 2's stages (no arithmetic of its own): per-stage kernel
 * timing with hipEvents recorded on the plan's stream around every
 * stage launch.  While enabled, replans launch their kernels one by one (no graph).
 * mtp_get_stage_times waits for the recorded events and returns, per stage
 * (candidates, rollout, top-E, refit), the summed kernel milliseconds and the
 * number of launches since timing was enabled. */
mtp_status mtp_set_stage_timing(mtp_plan* p, int32_t enable);
mtp_status mtp_get_stage_times(mtp_plan* p, double* h_ms4, uint64_t* h_count4);

/* Device views of the intermediates of Alg. 2's last loop body (layouts above). */
mtp_status mtp_get_buffers(const mtp_plan* p, mtp_buffers* out);

/* 1 if the plan draws each next CEM iteration's tensor-path controls during the
 * current iteration's rollout, else 0 (decided at creation from the config: more
 * than one iteration, tensor paths drawn with replacement, and a
 * rollout grid that leaves at least 32 of the 256 compute units free; on a
 * device with fewer units than that the plan runs the plain sequence).  Such a
 * plan's workspace holds a second [T][n][ldU] candidate buffer; the U buffer of
 * mtp_get_buffers still holds the candidates of the last iteration run.  The
 * results are the same bits either way (Alg. 2: the tensor paths do not depend
 * on the sampling distribution being refitted).  With an even iteration count
 * such a plan also draws across replans: the last iteration of replan r draws
 * the iteration-0 tensor paths of replan r + 1, which that replan takes when it
 * is the next one run (mtp_replan, or mtp_replan_at with index r + 1); any
 * other replan index, or an mtp_run_stage call in between, discards them. */
int32_t mtp_plan_draws_ahead(const mtp_plan* p);
/* Status of Alg. 2's last planning step: bit 0 = every elite cost was +inf (weights fell back to uniform);
 * bit 1 = an elite index out of range (never expected); bit 2 = a wait of the time-sliced rollout
 * timed out (results of that replan are not valid). */
mtp_status mtp_get_flags(mtp_plan* p, uint32_t* h_flags);
/* Release the plan object (the workspace stays the caller's). */
mtp_status mtp_plan_destroy(mtp_plan* p);

/* Error reporting of the conventions above (no passage of the paper). */
const char* mtp_status_str(mtp_status s);
const char* mtp_last_error(const mtp_plan* p);

/* The interpolation operator of Def. 2 (B-spline, Eq. 3-4), Def. 3 (Akima,
 * Eq. 5-7) or the linear paths of Thm. 1, as the host builds it (no device
 * needed): basis gets
 * horizon*8 floats, span gets horizon ints.  B-spline row t holds the degree+1
 * weights of control points span[t] .. span[t]+degree; Akima row t holds the
 * cubic Hermite weights (value i, slope i, value i+1, slope i+1) of interval
 * span[t], slopes in units of the knot spacing; linear row t holds the two
 * weights of waypoints span[t] and span[t]+1. */
mtp_status mtp_interp_table(const mtp_config* cfg, float* h_basis, int32_t* h_span);

/* ---------------------------------------------------------------- batching
 * Many independent instances (uneven candidate counts, horizons, control dims,
 * graphs, interpolation, iteration counts) replanned together by ONE
 * persistent kernel launch replayed from a hipGraph.  Workgroups pull
 * (instance, stage, iteration, tile) items from a device queue; the last tile of
 * an instance's stage publishes its next stage.  Every per-instance reduction
 * has a fixed order, so each instance's result is bit-identical to running it
 * alone as an mtp_plan with the same config and replan index.
 *
 * Packed vectors concatenate the instances in config order: x0 (sum of
 * state_dim floats) and actions (sum of ctrl_dim floats). */
typedef struct mtp_batch mtp_batch;

/* Workspace of n instances of Alg. 2 (each as mtp_workspace_bytes) plus the launch queue. */
size_t mtp_batch_workspace_bytes(const mtp_config* cfgs, int32_t n);
/* Alg. 2's initialisation for every instance (as mtp_plan_create). */
mtp_status mtp_batch_create(const mtp_config* cfgs, int32_t n, void* d_workspace, size_t ws_bytes,
                            void* hip_stream, mtp_batch** out);
/* Alg. 2's planning step for every instance at once: replan from the packed start states (device, read by the launch's
 * first kernel) with per-instance warm-start shifts (host array of n ints; NULL = 0).
 * All instances use the batch's replan counter, which then increments. */
mtp_status mtp_batch_replan(mtp_batch* b, const float* d_x0_packed, const int32_t* h_shift);
/* Part of Alg. 2's planning step for a subset: run CEM iterations [h_k_begin[i], h_k_end[i]) of replan h_r[i] for the
 * n_active instances listed in h_active (host arrays indexed like h_active).  The shift
 * applies to instances whose k_begin is 0; x0 is staged for those too (d_x0_packed may
 * be NULL to keep each instance's x0). */
mtp_status mtp_batch_step(mtp_batch* b, int32_t n_active, const int32_t* h_active, const int32_t* h_k_begin,
                          const int32_t* h_k_end, const int32_t* h_shift, const uint32_t* h_r,
                          const float* d_x0_packed);
/* Alg. 2's output per instance: the actions of the last launch (packed, host); synchronises; MTP_ERR_DEVICE if the
 * launch reported a queue timeout or overflow. */
mtp_status mtp_batch_get_actions(mtp_batch* b, float* h_u_packed);
/* Device views of instance i's Alg. 2 intermediates (as mtp_get_buffers). */
mtp_status mtp_batch_get_buffers(const mtp_batch* b, int32_t i, mtp_buffers* out);
/* Instance i's warm-start mean and std (as mtp_set_state, the replan index aside). */
mtp_status mtp_batch_set_state(mtp_batch* b, int32_t i, const float* d_mu, const float* d_sigma);
/*
 * Schedule of the batched launch.  None of it changes the arithmetic of Alg. 2:
 * every candidate, rollout, selection and refit output is computed by the same
 * code from the same inputs whichever workgroup takes it, so results are
 * bit-identical under every schedule.
 *   wg_per_cu      persistent workgroups per compute unit (0 = the occupancy limit)
 *   order          initial queue order: 0 = config order, 1 = longest estimated work first
 *   cand_tiles     candidate tiles (256 candidates, all joints) per queue item: 1, 2 or 4
 *   roll_tiles     rollout tiles (one workgroup's candidates) per queue item: 1, 2 or 4
 *   refit_outputs  refit outputs (t, j) per queue item: 4, 8, 16, 32 or 64
 *   split_pct      a launch whose active instances have fewer candidate tiles than
 *                  split_pct % of the persistent workgroups runs the finest items
 *                  instead (one joint of one candidate tile, one rollout tile, four
 *                  refit outputs), so that a light load still spreads over the chip;
 *                  0 = never, 100 = fewer tiles than workgroups
 * Defaults: {0, 1, 1, 1, 64, 100}.
 */
typedef struct {
  int32_t wg_per_cu;
  int32_t order;
  int32_t cand_tiles;
  int32_t roll_tiles;
  int32_t refit_outputs;
  int32_t split_pct;
} mtp_batch_schedule;

/* Scheduling of the batched launch: set the workgroups per compute unit and the queue order, keeping the rest. */
mtp_status mtp_batch_set_schedule(mtp_batch* b, int32_t wg_per_cu, int32_t order);
/* Scheduling of the batched launch: set every knob; MTP_ERR_INVALID_ARG (nothing changed) for a value outside
 * the ranges above. */
mtp_status mtp_batch_set_schedule_full(mtp_batch* b, const mtp_batch_schedule* h_schedule);
/* Scheduling of the batched launch: the schedule in force. */
mtp_status mtp_batch_get_schedule(const mtp_batch* b, mtp_batch_schedule* h_schedule);
/* Scheduling of the batched launch: time every workgroups-per-CU x order setting (reps replans each, HIP events) and
 * keep the fastest; writes {wg_per_cu, order} to h_choice and the best milliseconds per replan to h_ms.
 * Every instance is reset to its initial state and replan index 0 afterwards. */
mtp_status mtp_batch_autotune(mtp_batch* b, int32_t reps, int32_t* h_choice, float* h_ms);
/*
 * Scheduling of the batched launch (Alg. 2's planning step for many instances)
 * with a cache.  If cache_path (may be NULL)
 * names a schedule cache holding an entry for (this GPU's architecture name,
 * its compute-unit count, mtp_batch_mix_signature of the batch's configs), that
 * schedule is applied, nothing is launched and *h_from_cache = 1.  Otherwise
 * every knob is searched by coordinate descent (each value of one knob timed
 * with the others held, reps replans per setting after one warm-up, HIP
 * events; a change is kept when it is at least 1 % faster; at most three
 * sweeps over the knobs), the fastest schedule is applied and, with a
 * cache_path, stored there; *h_from_cache = 0, and every instance is reset to
 * its initial state and replan index 0.  h_out / h_ms (may be NULL) receive
 * the schedule and its milliseconds per replan (the cached figure on a hit).
 * Static batches only (the server's batch has no fixed mix).
 */
mtp_status mtp_batch_tune(mtp_batch* b, int32_t reps, const char* cache_path, mtp_batch_schedule* h_out,
                          float* h_ms, int32_t* h_from_cache);
/* Scheduling of the batched launch: signature of a mix for the schedule cache, a 64-bit FNV-1a hash of every
 * config's shape in order (dynamics, interpolation, links, dimensions, horizon,
 * graph, candidate counts, elites, iterations, degree, replicas, sampling,
 * diagnostics, debug states, task-parameter count).  Seeds, weights and other
 * float parameters do not enter.  Host only; 0 for invalid arguments. */
uint64_t mtp_batch_mix_signature(const mtp_config* cfgs, int32_t n);
/* Scheduling of the batched launch: the schedule cache (host only), a JSON file {"format": "mtp-schedules-1", "entries": [{"arch", "cus", "mix",
 * "wg_per_cu", "order", "cand_tiles", "roll_tiles", "refit_outputs", "split_pct", "ms"}, ...]}.
 * lookup: *h_found = 1 and the entry's schedule and ms if the file holds the key; 0 if it does not or the file is
 * missing or unreadable.  store: replaces the key's entry or appends one, keeping every other entry, and writes
 * the file through a temporary and a rename; MTP_ERR_INVALID_ARG for an invalid schedule or an existing file
 * that is not such a cache (left untouched). */
mtp_status mtp_schedule_cache_lookup(const char* path, const char* arch, int32_t cus, uint64_t mix,
                                     mtp_batch_schedule* h_out, float* h_ms, int32_t* h_found);
mtp_status mtp_schedule_cache_store(const char* path, const char* arch, int32_t cus, uint64_t mix,
                                    const mtp_batch_schedule* h_schedule, float ms);
/* As mtp_set_graph_mode, for the persistent launch. */
mtp_status mtp_batch_set_graph_mode(mtp_batch* b, int32_t use_graph);
/* Release the batch object (the workspace stays the caller's). */
mtp_status mtp_batch_destroy(mtp_batch* b);
const char* mtp_batch_last_error(const mtp_batch* b);

/* ---------------------------------------------------------------- serving
 * A request loop for many robots: the receding-horizon outer loop of Alg. 2
 * (replan from the current state, send the first control, shift the warm
 * start one step) run for a fleet, with continuous batching.
 *
 * Memory.  The server owns one caller-supplied device arena
 * (mtp_server_workspace_bytes): launch tables for max_robots slots and a pool
 * of hbm_budget_bytes.  A robot's resident buffers (warm-start mean / std,
 * start state, tables, replan counter) are taken from the pool when it is
 * added and given back when it is removed; every admitted request borrows a
 * transient slab (graph, paths, candidates, costs, elites) from the same pool
 * until its result is delivered.  The server never calls hipMalloc.
 *
 * Requests.  A request (robot, x0, shift) waits in an arrival-ordered queue; it
 * is admitted when its robot has no request in flight and its slab fits in the
 * pool.  Admitted requests run as continuous batches: every launch is one
 * persistent batched launch that advances each admitted request by up to
 * iters_per_launch CEM iterations from wherever it stands, so requests that
 * arrive while others are on the GPU join at the next iteration boundary.  Up
 * to max_inflight launches are queued on the stream ahead of the GPU.  A
 * request's result is bit-identical to the same replan run alone.
 *
 * Threading: submit, poll and stats may be called from any thread; pump, add,
 * remove and get_robot_state from one thread at a time (add and
 * get_robot_state synchronise the server's stream).  Clock: mtp_server_now_ns
 * (steady, nanoseconds). */
typedef struct mtp_server mtp_server;

typedef struct {
  uint64_t ticket;
  int32_t robot;
  int32_t status;            /* MTP_OK, or MTP_ERR_DEVICE if its launch failed */
  uint64_t t_arrival_ns;     /* as given to submit */
  uint64_t t_admit_ns;       /* when a slab was granted */
  uint64_t t_done_ns;        /* when pump saw the result on the host */
  uint32_t replan_idx;       /* the robot's replan counter used */
  int32_t n;                 /* valid entries of u (ctrl_dim <= 32) */
  float u[32];               /* u*: first control of the best candidate of the last iteration */
} mtp_completion;

typedef struct {
  uint64_t submitted, admitted, completed, launches, deferred_for_budget;
  uint64_t dropped;          /* requests of removed robots, never delivered */
  uint64_t pool_bytes, pool_in_use, pool_peak, resident_bytes;
  int32_t queued, in_flight, robots, pad;
} mtp_server_stats;

/* Device arena for a server: launch tables for max_robots robots and a queue of
 * queue_items items (0: 4096 per robot), x0 staging, and the pool of
 * hbm_budget_bytes.  0 if an argument is invalid. */
size_t mtp_server_workspace_bytes(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items);
/* Create an empty server on the caller's arena d_workspace (256-byte aligned,
 * at least mtp_server_workspace_bytes) and stream; iters_per_launch >= 1,
 * 1 <= max_inflight <= 8. */
mtp_status mtp_server_create(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items,
                             int32_t iters_per_launch, int32_t max_inflight, void* d_workspace, size_t ws_bytes,
                             void* hip_stream, mtp_server** out);
/* Same scheduler driving a host-only stand-in for the device (no GPU needed): a
 * launch takes 20 us plus ns_per_sample_step per candidate-step it advances and
 * returns zero actions.  For testing admission, budget and batching logic. */
mtp_status mtp_server_create_simulated(size_t hbm_budget_bytes, int32_t max_robots, uint32_t queue_items,
                                       int32_t iters_per_launch, int32_t max_inflight, double ns_per_sample_step,
                                       mtp_server** out);
/* Register a robot (its planner config, Alg. 2 inputs; copied): takes its
 * resident buffers from the pool, uploads its tables and initialises mean =
 * box centre, std = sigma_init, replan counter 0.  Writes its id.  MTP_ERR_BUSY
 * if every slot is taken, the pool cannot hold its resident buffers or the
 * launch queue cannot hold its items; MTP_ERR_UNSUPPORTED above ctrl_dim 32
 * or state_dim 64. */
mtp_status mtp_server_add_robot(mtp_server* s, const mtp_config* cfg, int32_t* robot_id);
/* Unregister a robot: its queued requests are dropped, a request already on the
 * GPU finishes but its completion is dropped, and its memory returns to the
 * pool when that launch has been retired.  The id may then be reused. */
mtp_status mtp_server_remove_robot(mtp_server* s, int32_t robot);
/* A robot's warm-start mean and std (device arrays of T*n floats, either may be
 * NULL) and its next replan index, for checkpoints and checks; MTP_ERR_BUSY
 * while it has a request admitted. */
mtp_status mtp_server_get_robot_state(mtp_server* s, int32_t robot, float* d_mu, float* d_sigma,
                                      uint32_t* replan_idx);
/* Queue a replan of `robot` from host state h_x0 (state_dim floats, copied),
 * shifting its warm start by `shift` steps first (Alg. 2's receding horizon). */
mtp_status mtp_server_submit(mtp_server* s, int32_t robot, const float* h_x0, int32_t shift,
                             uint64_t t_arrival_ns, uint64_t* ticket);
/* One scheduling round: retire finished launches (their completed requests become
 * pollable and free their slabs), admit waiting requests, enqueue the next launch if
 * there is work and room.  If wait_us > 0 and nothing could be retired, block up to
 * wait_us for the oldest launch first. */
mtp_status mtp_server_pump(mtp_server* s, int32_t wait_us, int32_t* n_completed);
/* Completed requests (at most max), oldest first. */
mtp_status mtp_server_poll(mtp_server* s, mtp_completion* out, int32_t max, int32_t* n_out);
/* Counters of the request loop (admission, budget, launches). */
mtp_status mtp_server_get_stats(const mtp_server* s, mtp_server_stats* out);
/* The server's clock for arrival and completion times. */
uint64_t mtp_server_now_ns(void);
/* Release the server; its arena stays the caller's.  Synchronises its stream. */
mtp_status mtp_server_destroy(mtp_server* s);
const char* mtp_server_last_error(const mtp_server* s);

/* ------------------------------------------------------------ no allocation
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid it): one replan, as mtp_replan_at
 * on a fresh plan whose warm start is (d_mu, d_sigma), with every buffer
 * besides its inputs and outputs in a static device array of
 * mtp_noalloc_scratch_bytes() (64 MiB) that each device holds for the life of
 * the process.  No hipMalloc, no workspace, no graph.
 *   d_x0     [state_dim] start state (read)
 *   d_mu, d_sigma [T][n] warm-start mean and std: read, shifted by shift_steps,
 *            refitted over n_iters CEM iterations and written back
 *   d_action [n] written: first control of the best candidate of the last iteration
 * Enqueued on hip_stream (NULL = default); the host tables are uploaded with a
 * synchronisation of that stream first.  Every call on one device uses the same
 * array and leaves its contents behind: calls that overlap on a device race.
 * MTP_ERR_WORKSPACE if the config's buffers (mtp_workspace_bytes without the
 * second candidate buffer) exceed the array. */
size_t mtp_noalloc_scratch_bytes(void);
mtp_status mtp_replan_noalloc(const mtp_config* cfg, const float* d_x0, float* d_mu, float* d_sigma,
                              int32_t shift_steps, uint32_t replan_idx, float* d_action, void* hip_stream);

/* Host-side plant of a robot, for closing the receding-horizon loop of Alg. 2
 * around a server or plan (execute u*, replan from the state it leads to): one
 * step x_{t+1} = f(x_t, u_t) of cfg's model in float64 on the host (no device
 * work), h_x and h_x_next state_dim doubles, h_u ctrl_dim floats.  The point
 * mass takes a semi-implicit Euler step, the chains a classical RK4 step with
 * the control held; the contact chain uses the first row of sample_params as
 * its masses and friction. */
mtp_status mtp_plant_step(const mtp_config* cfg, const double* h_x, const float* h_u, double* h_x_next);

/* The rollout of Alg. 2 (Eq. 1) is compiled per chain length: the lengths it is
 * instantiated for (writes up to `cap`, returns the count). */
int32_t mtp_supported_chain_links(int32_t* out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* MTP_H_ */
