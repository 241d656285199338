/*
 * comet.h -- C ABI of the MI355X (gfx950) batched mode-conditioned trajectory-optimisation
 * evaluator and of the greedy contact-mode expansion around it.
 *
 * The method (CoMET): for a fixed contact-mode order the planning problem of Eq. (1)
 * reduces to the smooth constrained TO of Eq. (2); every candidate order is solved by a
 * finite-budget local solver whose result is scored in physical units by Eq. (4) and
 * ranked by the merit of Eq. (5); Alg. 1 expands the best-ranked orders by r-edit
 * neighbourhoods and refines the best feasible ones (Sec. III-B, III-C).
 *
 * Conventions for every call:
 *   - Array pointers are DEVICE pointers owned by the caller (for example the data of
 *     torch tensors on cuda:0).  Struct pointers are HOST pointers.  The library never
 *     frees caller memory and never keeps a caller pointer after a call returns.
 *   - Calls that take a stream are asynchronous on that stream unless stated; a NULL
 *     stream means the default stream of the current device.
 *   - No exception crosses the ABI.  Host-detectable errors (null pointers, sizes beyond
 *     what the context was created for) return COMET_EINVAL before any launch, and
 *     comet_last_error() describes them.  Errors in device data (an out-of-range mode id,
 *     a segment count outside [1, max_segments], too many intervals, a non-finite input)
 *     do not stop the batch: that sequence gets cost = NaN, viol = +inf, feasible = 0 and
 *     a device error counter is incremented; comet_check() reads and clears it.
 *   - Units are SI throughout: m, rad, N, m/s.
 *   - Outputs depend only on the inputs of the same sequence, never on the batch.
 */
#ifndef COMET_H
#define COMET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  COMET_OK = 0,
  COMET_EINVAL = -1, /* bad argument or bad device data (see comet_last_error) */
  COMET_EHIP = -2,   /* a HIP runtime call failed */
  COMET_ENOMEM = -3, /* device allocation failed */
  COMET_ESTATE = -4  /* call not valid in the context's current state */
} comet_status;

/* Tasks: planar pushing (Sec. IV-A) with a fixed step, bimanual flipping of a box in a
 * vertical plane (Sec. IV-B), planar pushing with optimised timing (Sec. III-C: the
 * interval durations become controls; Sec. IV-A runs pushing with an optimised time step
 * under a duration bound), and planar pushing with free-motion segments (the admissible
 * language of Sec. III-A: modes are contact events or free motion, and a contact changes
 * faces only through free motion); their dimensions and layouts are given at
 * comet_evaluate. */
typedef enum {
  COMET_TASK_PUSH = 0,
  COMET_TASK_FLIP = 1,
  COMET_TASK_PUSH_TIMED = 2,
  COMET_TASK_PUSH_FREE = 3,
  COMET_TASK_PUSH_FREE_TIMED = 4
} comet_task;

typedef struct comet_ctx comet_ctx; /* opaque */
typedef struct comet_mlp comet_mlp; /* opaque: learned proposal / warm-start network */

/* Solver parameters of the per-order TO (Sec. III-C).  Defaults: comet_default_params.
 *   al_max, gn_max          augmented-Lagrangian outer / Gauss-Newton inner budget
 *                           (exploration budget t_exp of Alg. 1)
 *   ref_al_max, ref_gn_max  refinement budget t_ref
 *   chol_retries            Cholesky attempts with raised damping before a step is rejected
 *   ls_trials               trial step lengths 1, 1/2, ..., 2^-(ls_trials-1), 1..16
 *   max_rejects             consecutive rejected steps that end an inner loop
 *   mu0, mu_min             initial / smallest penalty parameter mu (phi uses c^2/(2 mu))
 *   rho0, rho_min, rho_max  damping of the local systems S_k = H_k + rho I + A^T A / mu
 *   armijo_c1               sufficient-decrease constant of the trial steps
 *   eta_star, omega_star,   scaled feasibility, stationarity and complementarity
 *   rc_star                 tolerances of the stopping test
 *   eps_feas                feasibility tolerance of the physical-unit score, Eq. (4)
 *   mu0_warm                initial penalty parameter of a solve that starts from a caller
 *                           or learned warm start (the primal is taken to be near a solution,
 *                           so the outer loop starts with a tight penalty; multipliers start
 *                           at zero either way)                                          */
typedef struct {
  int32_t al_max, gn_max, ref_al_max, ref_gn_max;
  int32_t chol_retries, ls_trials, max_rejects, reserved;
  double mu0, mu_min, rho0, rho_min, rho_max, armijo_c1;
  double eta_star, omega_star, rc_star, eps_feas;
  double mu0_warm;
} comet_solver_params;

void comet_default_params(comet_solver_params* p);

/* Create a context for one task on the current HIP device.  Allocates the device work
 * space for up to max_batch sequences of up to max_segments segments and max_intervals
 * control intervals each (synchronous).  Returns COMET_EINVAL for max_segments outside
 * [1, 6] ([1, 8] for the free-motion tasks, whose orders the paper caps at eight segments,
 * Sec. IV-A), max_intervals outside [1, 512] or max_batch < 1, COMET_ENOMEM if the work
 * space does not fit. */
comet_status comet_create(comet_task task, const comet_solver_params* params, int64_t max_batch,
                          int32_t max_segments, int32_t max_intervals, comet_ctx** out);
void comet_destroy(comet_ctx* ctx);

/* Message of the last error on this context (thread-unsafe; the context owns the string).
 * With ctx = NULL: the message of the calling thread's last failed call that takes no
 * context (comet_probe_peaks), or "". */
const char* comet_last_error(const comet_ctx* ctx);

/* Task dimensions: state size nx, control size nu, instance parameters per sequence,
 * number of mode ids, and the context limits. */
comet_status comet_dims(const comet_ctx* ctx, int32_t* nx, int32_t* nu, int32_t* n_inst_params, int32_t* n_modes,
                        int32_t* max_segments, int32_t* max_intervals, int64_t* max_batch);

/* Row scales of the solver's internal constraint scaling (Sec. IV-A: each row type is
 * divided by its median Jacobian-row 2-norm over sample orders).  out: host, n >= 12
 * (fixed-step pushing) or n >= 13 (optimised timing: type 12 is the duration bound).
 * Pushing contexts only (the flipping rows are stated non-dimensionally): COMET_EINVAL
 * otherwise. */
comet_status comet_row_scales(const comet_ctx* ctx, double* out, int32_t n);

/* Synchronise `stream`, read and clear the device error counter.  Returns COMET_EINVAL
 * (with the count in comet_last_error) if any sequence since the last check had invalid
 * device data. */
comet_status comet_check(comet_ctx* ctx, void* stream);

/* Evaluate B candidate orders: one mode-conditioned TO per sequence (Eq. 2), scored by
 * Eq. (4).  Pushing task: nx = 4 (x, y, theta, s), nu = 3 (F_n, F_t, v_s), one instance
 * parameter (pusher friction), 12 mode ids = 3*face + slip (face 0..3 with outward normal
 * at angle face*pi/2; slip 0 stick, 1 slide+, 2 slide-).
 *   x0    [B, nx]      start state (float32)
 *   goal  [B, 3]       goal pose (x, y, theta), theta not wrapped
 *   inst  [B, 1]       instance parameters
 *   nseg  [B]          number of segments K, 1..max_segments (int32)
 *   modes [B, Smax]    mode id of each segment, Smax = max_segments; entries >= K ignored
 *   knots [B, Smax]    control intervals of each segment (>= 1); their sum N <= max_intervals
 *   warm  [B, Nmax+1, nx+nu] or NULL: initial primal (rows (x_k, u_k), Nmax = max_intervals);
 *                      NULL = schedule-derived initial guess (Sec. IV-A)
 *   refine 0 = exploration budget (al_max, gn_max), 1 = refinement budget
 *   cost  [B]          J at the returned trajectory (float32)
 *   viol  [B]          max(|g|_inf, |[h]_+|_inf) in physical units, Eq. (4)
 *   feasible [B]       1 iff viol <= eps_feas (uint8)
 *   traj  [B, Nmax+1, nx+nu] or NULL: row k = (x_k, u_k), row N has u = 0, rows > N zero
 *   stats [B, 4] or NULL: (outer iterations, inner iterations, Cholesky failures, status)
 *                      status 1 converged, 0 budget exhausted, 2 non-finite, 3 invalid input
 * B = 0 is a no-op.  B > max_batch returns COMET_EINVAL.
 *
 * Flipping task (COMET_TASK_FLIP): box 0.2 x 0.1 m, 0.5 kg, on the table line y = 0 under
 * gravity, pushed by two point fingers; quasi-static: the table reaction is the balance of
 * gravity and the finger forces.
 *   x0    [B, 8]   (px, py, th, vx, vy, om, s1, s2): centre, angle, twist, finger face
 *                  coordinates; the start is taken at rest on face 3 (the -y face)
 *   goal  [B, 2]   (px, th) at the final knot; the final twist is zero
 *   inst  [B, 1]   table friction coefficient
 *   controls (nu = 9): (ax, ay, al, f1n, f1t, sd1, f2n, f2t, sd2): accelerations of the
 *                  twist, normal / tangential force and face-coordinate rate per finger
 *   mode id = (f1 * 13 + f2) * 5 + g, 845 ids: finger code 0 free, 1 + 3 face + slip
 *                  (slip 0 stick, 1 slide+, 2 slide-); table g: 0 stick, 1 slide+,
 *                  2 slide-, 3 pivot about the left corner of the support face (counter-
 *                  clockwise), 4 pivot about its right corner (clockwise).  A pivot run
 *                  followed by a table-supported segment lands on the neighbouring face;
 *                  an order whose consecutive pivots change direction is invalid.
 *   rows are stated non-dimensionally (forces / mg, moments / (mg * 0.2 m)); viol is in
 *                  these units; cost = sum dt (0.01 |accel|^2 + sum |f_i|^2 / (mg)^2 +
 *                  0.01 sum sd_i^2)
 *   traj  [B, Nmax+1, 17] rows (x_k, u_k); warm likewise.
 *
 * Pushing with optimised timing (COMET_TASK_PUSH_TIMED): the pushing task with the
 * duration h_k of every interval as a fourth control, nu = 4 (F_n, F_t, v_s, h); every
 * defect steps by h_k instead of 0.1 s, each interval carries the bounds
 * 0.02 s <= h_k <= 0.2 s, and cost = sum h_k ((F_n^2 + F_t^2) / f_max^2 + (v_s / v_ref)^2
 * + 0.01) charges the elapsed time; the schedule-derived start has h_k = 0.1 s.
 *   traj  [B, Nmax+1, 8] rows (x_k, u_k); warm likewise.  With the learned network the
 *                  eighth warm-start channel carries the interval duration.
 *
 * Pushing with free motion (COMET_TASK_PUSH_FREE): the slider of the pushing task and a
 * point pusher whose position is part of the state.
 *   x0    [B, 5]  start (x, y, theta, p_x, p_y): slider pose, pusher position in the
 *                 slider frame
 *   goal  [B, 3]  slider pose (x, y, theta); the pusher may end anywhere
 *   inst  [B]     pusher-slider friction coefficient
 *   modes ids 0..11 contact on face id / 3 with slip id % 3 (stick, slide+, slide-), face
 *                 j with outward normal at angle j pi/2; ids 12..15 free motion in front of
 *                 face id - 12 (the half-plane where n . p >= a/2)
 *   controls u = (F_n, F_t, v_x, v_y): contact force and the pusher's velocity in the
 *                 slider frame, p_{k+1} = p_k + 0.1 s v; the slider's twist follows the
 *                 limit surface of the pushing task with the moment M = p x F.  Contact
 *                 rows: the pusher on the face at p_k (n . p_k = a/2) and moving along it
 *                 (n . v = 0), stick (t . v = 0) or slide (F_t = +-mu F_n, +-t . v >= 0),
 *                 F_n >= 0 and the cone when sticking, |t . p| <= a/2 at both knots.
 *                 Free rows: F_n = F_t = 0 and no penetration, n . p >= a/2 at both knots.
 *                 An order whose first segment is a contact needs the pusher on that face
 *                 at the start; any order is evaluated (the language is the expansion's).
 *   cost  sum 0.1 ((F_n^2 + F_t^2) / f_max^2 + |v|^2 / v_ref^2)
 *   traj  [B, Nmax+1, 9] rows (x_k, u_k); warm likewise.  The schedule-derived start puts
 *                 the pusher at the centre of the scheduled face during a contact segment
 *                 and 2 cm in front of the face during a free segment.
 *
 * Pushing with free motion and optimised timing (COMET_TASK_PUSH_FREE_TIMED; the paper's
 * pushing transcription optimises the time step, Sec. IV-A): the free-motion task with the
 * duration h_k of every interval as a fifth control, u = (F_n, F_t, v_x, v_y, h); every
 * defect steps by h_k, each interval carries 0.02 s <= h_k <= 0.2 s, cost = sum h_k
 * ((F_n^2 + F_t^2) / f_max^2 + |v|^2 / v_ref^2 + 0.01); the start has h_k = 0.1 s and the
 * same language, segment cap and keys as COMET_TASK_PUSH_FREE.
 *   traj  [B, Nmax+1, 10] rows (x_k, u_k); warm likewise. */
comet_status comet_evaluate(comet_ctx* ctx, void* stream, int64_t B, const float* x0, const float* goal,
                            const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                            const float* warm, int32_t refine, float* cost, float* viol, uint8_t* feasible,
                            float* traj, int32_t* stats);

/* comet_evaluate without a context, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * pushing tasks only (COMET_TASK_PUSH, COMET_TASK_PUSH_TIMED; others COMET_EINVAL).  The
 * solver's work space lives in a static device array of 64 MiB that every GPU the library
 * runs on holds until the process ends; this call allocates nothing (its first call on a
 * device looks up that device's copy of the array and the device's properties).
 *   params          solver parameters, NULL = comet_default_params (exploration budget)
 *   max_segments    column count of modes / knots (1..6)
 *   max_intervals   row count Nmax of traj (1..512): every order must have <= Nmax intervals
 *   other arguments as comet_evaluate (no warm start, exploration budget).
 * Limit: the work space of B orders and max_intervals rows must fit 64 MiB -- about
 * 265 bytes per (order rounded up to 64) x interval, e.g. 2,048 orders of up to 120
 * intervals; larger requests return COMET_EINVAL before any launch (message from
 * comet_last_error(NULL)).  Results equal comet_evaluate's bit for bit.  Invalid device data
 * is reported through the outputs only (cost NaN, viol +inf, status 3): there is no error
 * counter to read.  All calls on one GPU share its array, so calls that overlap in time on
 * one GPU (other streams, other threads) race and must be serialised by the caller.
 * Asynchronous on `stream`; B = 0 is a no-op. */
comet_status comet_evaluate_noalloc(comet_task task, const comet_solver_params* params, void* stream, int64_t B,
                                    int32_t max_segments, int32_t max_intervals, const float* x0, const float* goal,
                                    const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                                    float* cost, float* viol, uint8_t* feasible, float* traj, int32_t* stats);

/* Launch schedule of the solver kernel.  The kernel is persistent: each lane solves one
 * order at a time and takes the next one from a device work queue when its solve ends
 * (Sec. III-C: a reusable pool of slots with independent stopping).
 *   waves_per_cu    resident 64-lane waves launched per compute unit; 0 = the occupancy
 *                   limit of the kernel (never more than one wave per 64 sequences)
 *   sort_by_length  1 = the queue hands out orders by decreasing interval count, so the
 *                   lanes of a wave sweep similar lengths (ragged batches)
 * A new context starts with {0, 1}.  Results do not depend on the schedule (each order's
 * arithmetic is the same in every lane). */
typedef struct {
  int32_t waves_per_cu, sort_by_length;
} comet_schedule;

comet_status comet_set_schedule(comet_ctx* ctx, const comet_schedule* sched);
/* Current schedule, the kernel's occupancy limit (waves per CU) and the CU count. */
comet_status comet_get_schedule(const comet_ctx* ctx, comet_schedule* sched, int32_t* occupancy_waves_per_cu,
                                int32_t* n_cu);

/* Autotuner: run comet_evaluate on the given batch (outputs written as by comet_evaluate,
 * warm = NULL, refine = 0) once per candidate schedule -- waves_per_cu in {1, 2, 4} x the
 * occupancy limit, sort_by_length in {0, 1} -- time each solver launch with HIP events,
 * keep the fastest in the context and return it (and its time in ms).  Synchronises
 * `stream`; not allowed under stream capture (COMET_ESTATE). */
comet_status comet_autotune(comet_ctx* ctx, void* stream, int64_t B, const float* x0, const float* goal,
                            const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                            float* cost, float* viol, uint8_t* feasible, float* traj, int32_t* stats,
                            comet_schedule* best, float* best_ms);

/* Device time (milliseconds) of the last comet_evaluate on this context, measured with
 * HIP events around its solver kernel on the caller's stream; valid after that stream
 * has been synchronised.  Used for roofline accounting. */
comet_status comet_last_kernel_ms(comet_ctx* ctx, float* ms);

/* ---------------------------------------------------------------------------------
 * Greedy contact-mode expansion (Alg. 1, Sec. III-B) on the device.
 *
 * Orders are keys: K << 60 | m_0 << 50 | m_1 << 40 | ... | m_5 << 0 (10 bits per mode id;
 * with free motion K << 60 | m_0 << 56 | m_1 << 52 | ... | m_7 << 28, 4 bits per id, up to
 * eight segments), so comparing keys compares the segment count, then the ids
 * lexicographically.  The language is every order of 1..kcap segments over the task's mode
 * ids, restricted by the task's rules where it has them (below).  With free motion the seed
 * pass enumerates the admissible orders themselves (the product space of eight segments
 * has 16^8 orders), so a seed of eight segments is the whole language: 205,632 orders.
 *   kcap               segment cap (<= max_segments)
 *   seed_max_segments  seed batch F_0 = every order with at most this many segments, in key order
 *   radius             r of the r-edit neighbourhood (1 or 2): an edit inserts, deletes or
 *                      substitutes one segment; neighbours are enumerated substitutions
 *                      (position, then id), deletions (position), insertions (position, then
 *                      id), and for r = 2 each one-edit neighbour's list in that order
 *   rounds             expansion rounds after the seed (s_max)
 *   frontier_W         at most this many best-ranked evaluated orders are expanded per round
 *   knots_per_segment  intervals per segment; 0 = split n_total intervals as evenly as
 *                      possible, the remainder going to the earliest segments
 *   k_ref              feasible orders re-solved with the refinement budget at the end
 *   batch_B            batch width B (<= max_batch); eval_budget caps the evaluated orders
 *   mu_merit           mu of the merit M = J + mu max(v - eps_feas, 0), Eq. (5)
 * Ranking is by (M, key) with NaN as +inf; refinement ranks feasible orders by (J, key) and
 * returns the smallest refined J among refined-feasible orders (ties by key).
 *   policy             COMET_POLICY_EXPAND (0): Alg. 1 as above.  COMET_POLICY_UNIFORM (1):
 *                      the uniform-sampling baseline of Sec. IV-B: every batch,
 *                      the first one included, is drawn instead of generated, complete orders
 *                      without replacement; seed_max_segments, radius and frontier_W are
 *                      unused.  Round s makes sample_draws draws, numbered from s *
 *                      sample_draws; draw c takes outputs 8c .. 8c+6 of the SplitMix64 stream
 *                      seeded with sample_seed (output i = mix(seed + (i+1) * 0x9E3779B97F4A7C15),
 *                      mix: z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27,
 *                      z *= 0x94D049BB133111EB, z ^= z >> 31): K = 1 + out(8c) mod kcap and
 *                      id j = out(8c+1+j) mod (number of ids), j < K.  A draw outside the
 *                      task's language, already evaluated, or equal to an earlier draw of the
 *                      round is dropped; the batch is the first min(room, kept) remaining draws
 *                      in draw order.  So each segment count is equally likely and, given the
 *                      count, every admissible order is.  With free motion (whose admissible
 *                      eight-segment orders are 1 in 28,500 of the product space) draw c takes
 *                      t = out(8c+1) mod (number of admissible orders of K segments) and the
 *                      t-th of them in key order instead, without rejection.  Refinement and
 *                      the returned plan are as for the expansion.
 *   sample_draws       draws per round (policy 1; 1 .. 2^27)
 *   policy COMET_POLICY_MCTS (2): the UCT allocation of the baselines (Sec. IV-A, IV-B) on the
 *                      same evaluator and refinement, batch_B selections per update (the
 *                      pool P), exploration constant uct_c (the paper's 0.8), rollouts from
 *                      the SplitMix64 stream of sample_seed (as above).  The tree is over
 *                      order prefixes: actions "stop" (length >= 1) then "append id"
 *                      (length < kcap) for the ids, in order, that keep the prefix in the
 *                      language; an untried action is expanded first (stop first), else the
 *                      child of largest W/N + uct_c sqrt(ln N_parent / N) (first on ties);
 *                      visits are counted at selection (virtual loss); a new "append" child
 *                      of length d is completed to K = d + out(8r) mod (kcap - d + 1)
 *                      segments, segment j taking admissible id number out(8r+1+j) mod
 *                      (count) (r = rollout number).  Evaluated orders are cached and the
 *                      budget counts distinct orders; the selection that would exceed it is
 *                      undone and ends the batch.  Rewards after each batch: pushing J_best/J
 *                      for feasible orders (0 otherwise), flipping M_best/M (merit, Eq. (5)).
 *                      Ends at the budget, when nothing is untried and a batch brings no new
 *                      order, or after 64 batches in a row without one.  Runs as a host loop
 *                      with one device evaluation per batch (not captured); no learned
 *                      network (EINVAL).  rounds, seed_max_segments, radius, frontier_W and
 *                      sample_draws are unused.
 *   uct_c              UCT exploration constant (policy 2; finite, >= 0) */
typedef enum { COMET_POLICY_EXPAND = 0, COMET_POLICY_UNIFORM = 1, COMET_POLICY_MCTS = 2 } comet_policy;
typedef struct {
  int32_t kcap, seed_max_segments, radius, rounds, frontier_W, knots_per_segment, k_ref, n_total;
  int32_t learned_warm;   /* with a learned network: 1 = also seed initial trajectories, 0 = order only */
  int32_t policy;         /* comet_policy */
  int64_t batch_B, eval_budget;
  double mu_merit;
  uint64_t sample_seed;   /* policy 1: draws; policy 2: rollouts */
  int64_t sample_draws;   /* policy 1 */
  double uct_c;           /* policy 2 */
} comet_expand_params;

typedef struct {
  int64_t evaluated;             /* orders evaluated (|V|) */
  int32_t rounds_done;           /* evaluation rounds with a non-empty batch */
  int32_t n_feasible;            /* evaluated orders with v <= eps_feas */
  int64_t first_feasible_index;  /* 1-based position in evaluation order of the first feasible order, 0 = none */
  double t_first_feasible_ms;    /* device wall clock from the start of the expansion to the first feasible
                                    completed solve (-1 = none): time to first feasible plan */
  double t_total_ms;             /* device time of the whole expansion including refinement */
  int32_t n_refined, reserved;
} comet_expand_stats;

/* Run seed, s_max expansion rounds and refinement for one instance (x0 [nx], goal [3]
 * (pushing) or [2] (flipping), inst [n_inst]: device pointers).  The order language is the
 * task's: pushing, every sequence of the 12 ids; flipping, the admissible orders (fingers
 * never share a face, change faces only through a free segment, a pivot keeps a finger in
 * contact, no two consecutive equal segments, consecutive pivots keep their direction, no
 * finger on the face on the table -- the support face, and in a pivot the landing face);
 * pushing with free motion, the orders of its 16 ids where no two consecutive segments are
 * equal, a contact keeps its face until a free segment, contact on face j is entered from
 * and left to the free region in front of face j, and free regions connect to the regions
 * of the neighbouring faces (Sec. III-A); the seed and every generated neighbour are
 * filtered by it, and a two-edit neighbour only through an admissible one-edit order.
 * The learned network serves every task (its encoding and warm-start block must be wide
 * enough for the task: see comet_mlp_encode).  The loop runs as one captured HIP graph on an internal
 * stream ordered after `stream`; the call synchronises and fills `stats` (host).  Outputs
 * (device): best_nseg [1] (0 = no feasible plan), best_modes / best_knots [max_segments],
 * best_cost / best_viol [1] (refined), best_traj [max_intervals+1, nx+nu] or NULL.
 * learned: NULL for the plain method, else a proposal network that ranks generated
 * neighbours and seeds their initial trajectories (the plain refinement re-solves every plan).
 * EINVAL on inconsistent parameters (see comet_expand_params), ENOMEM if the work space
 * (|V| <= eval_budget + batch_B, frontier_W x neighbourhood candidates <= 2^27) does not fit. */
comet_status comet_expand(comet_ctx* ctx, void* stream, const float* x0, const float* goal, const float* inst,
                          const comet_expand_params* params, comet_mlp* learned, int32_t* best_nseg,
                          int32_t* best_modes, int32_t* best_knots, float* best_cost, float* best_viol,
                          float* best_traj, comet_expand_stats* stats);
/* (a learned network encodes orders of the context's task, see comet_mlp_encode; it must
 * have been trained on that task's results) */

/* One batch-construction step of Alg. 1 on given scores: rank the n evaluated orders
 * (keys [n] uint64, merit [n] double, device) by (merit, key), traverse at most frontier_W of
 * them and admit their unseen r-edit neighbours in enumeration order until `room` orders are
 * admitted (in the context task's language).  Writes out_keys [room] and out_n [1] (device,
 * int64).  Synchronises `stream`. */
comet_status comet_expand_next(comet_ctx* ctx, void* stream, int64_t n, const uint64_t* keys, const double* merit,
                               const comet_expand_params* params, int64_t room, uint64_t* out_keys,
                               int64_t* out_n);

/* Evaluated set of the last comet_expand on this context, in evaluation order: up to cap
 * keys, J and v (device buffers, any may be NULL) and the full count in n_out (device int64).
 * Synchronises `stream`. */
comet_status comet_expand_trace(comet_ctx* ctx, void* stream, int64_t cap, uint64_t* keys, double* J, double* v,
                                int64_t* n_out);

/* ---------------------------------------------------------------------------------
 * Learned proposal / warm-start network (BF16 matrix-core kernels, FP32 accumulation).
 * in_dim -> `layers` hidden layers of width `hidden` (exact-erf GELU) -> out_dim.  Output
 * row: [0] feasibility logit, [1] predicted log(1 + J), [2 .. 2 + 120 S) warm start: for
 * each of S = min(8, (out_dim - 2) / 120) segment slots, 15 samples at normalised times
 * i/14 of 8 channels (pushing: the 7 trajectory channels (x, y, theta, s, F_n, F_t, v_s)
 * and a zero channel; timed pushing: the same with the interval duration as channel 7;
 * flipping: the 8 states; free motion: (x, y, theta, p_x, p_y, F_n, F_t) and, with
 * optimised timing, the duration as channel 7).  A network for the pushing, timed-pushing
 * and flipping tasks has S = 6 (out_dim 736: 722 padded to a multiple of 8), for free
 * motion S = 8 (out_dim >= 962, e.g. 968).  Flat parameter
 * layout: for each linear layer in order, W [out][in] row-major then b [out] (FP32).
 * Initialisation: W ~ U(-1/sqrt(in), 1/sqrt(in)) from a counter-based hash of (seed, index),
 * b = 0.  Training: AdamW (beta 0.9 / 0.999, eps 1e-8) on FP32 masters; GEMM operands
 * (weights, inputs, activations, back-propagated gradients) are rounded to BF16.
 * in_dim, hidden and out_dim must be multiples of 8 (16-byte operand vectors), else
 * COMET_EINVAL; out_dim >= 722.  For comet_mlp_forward, _encode, _targets and
 * _decode_warm, B = 0 is a no-op after the scalar arguments are checked (array pointers
 * may then be NULL); comet_mlp_train_step needs 1 <= B <= max_batch. */
comet_status comet_mlp_create(int32_t in_dim, int32_t hidden, int32_t layers, int32_t out_dim, int64_t max_batch,
                              uint64_t seed, comet_mlp** out);
void comet_mlp_destroy(comet_mlp* mlp);
comet_status comet_mlp_num_params(const comet_mlp* mlp, int64_t* n);
/* get (set = 0) or set (set = 1) the FP32 master parameters from / to a device buffer of
 * num_params floats; setting also resets the optimiser state.  Asynchronous on `stream`. */
comet_status comet_mlp_params(comet_mlp* mlp, void* stream, int32_t set, float* flat);
/* gradients of the last train step (device buffer of num_params floats) */
comet_status comet_mlp_grads(comet_mlp* mlp, void* stream, float* flat);
/* out [B, out_dim] = network(x [B, in_dim] BF16 bits), B <= max_batch */
comet_status comet_mlp_forward(comet_mlp* mlp, void* stream, int64_t B, const uint16_t* x_bf16, float* out);
/* One AdamW step on a batch: y_feas [B] in {0,1}, y_cost [B] (log(1+J), used where feasible),
 * y_traj / traj_mask [B, 120 S] with S the network's warm-start segments (outputs beyond
 * 2 + 120 S get no gradient; y_traj 8-byte and traj_mask 16-byte aligned, B * out_dim <
 * 2^31, else COMET_EINVAL).
 * loss (device, 3 floats, may be NULL): mean BCE,
 * cost MSE over feasible samples, warm-start MSE over the mask, before the step. */
comet_status comet_mlp_train_step(comet_mlp* mlp, void* stream, int64_t B, const uint16_t* x_bf16,
                                  const float* y_feas, const float* y_cost, const float* y_traj,
                                  const float* traj_mask, float lr, float weight_decay, float* loss);
/* Input encoding of orders (same arguments as comet_evaluate, Smax = smax) into in_dim
 * BF16 values per order, a pose block of 16 then S segment slots of 64 (absent segments
 * all zero, values beyond 16 + 64 S zero): S = 6 and in_dim >= 400, smax <= 6 (pushing,
 * timed pushing, flipping), S = 8 and in_dim >= 528, smax <= 8 (free motion).
 *   COMET_TASK_PUSH: pose = start and goal (x, y, cos, sin), goal - start (x, y, theta),
 *     pusher friction; slot = one-hot mode id (12), intervals / 15, present flag.
 *   COMET_TASK_FLIP: pose = start (px, py, cos, sin), goal (px, 0, cos, sin), goal - start
 *     (px, 0, theta), table friction; slot = one-hot finger-1 code (13), one-hot finger-2
 *     code (13), one-hot table mode (5), intervals / 15, present flag.
 *   COMET_TASK_PUSH_TIMED: as COMET_TASK_PUSH.
 *   COMET_TASK_PUSH_FREE, COMET_TASK_PUSH_FREE_TIMED: the pushing pose block and the
 *     pusher's start position (p_x, p_y) at 12 and 13; slot = one-hot mode id (16),
 *     intervals / 15, present flag.
 * The network proposes orders and warm starts; it is an addition to the paper's method
 * (the paper has no learned component), so no passage defines it.  Other tasks: COMET_EINVAL. */
comet_status comet_mlp_encode(comet_task task, void* stream, int64_t B, const float* x0, const float* goal,
                              const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                              int32_t smax, int32_t in_dim, uint16_t* x_bf16);
/* Training targets from evaluator results (traj [B, nmax+1, row] in comet_evaluate's
 * layout, row = 7 pushing / 8 timed pushing / 17 flipping / 9 free motion / 10 free motion
 * with optimised timing; feasible; cost): y_feas, y_cost = log(1 + J) (0 if infeasible),
 * y_traj [B, 120 S] per-segment samples (S slots x 15 times i/14 x 8 channels; S = 6, or 8
 * for free motion, with smax <= S) by linear interpolation of the rows, traj_mask [B, 120 S]
 * = 1 on the learned channels of present segments of feasible orders.  Learned channels:
 * pushing, the 7 row entries (channel 7 zero); timed pushing, the 8 row entries (channel 7
 * the duration); flipping, the 8 state entries; free motion, row entries 0..6 (states and
 * forces; channel 7 zero), with optimised timing also the duration (row entry 9) as
 * channel 7.  A sequence whose segment count is outside [1, smax], or
 * whose live knot counts are not each >= 1 with a sum <= nmax, is treated as empty: its
 * y_traj and traj_mask rows are zero. */
comet_status comet_mlp_targets(comet_task task, void* stream, int64_t B, const float* traj, int32_t nmax,
                               const int32_t* nseg, const int32_t* knots, int32_t smax, const uint8_t* feasible,
                               const float* cost, float* y_feas, float* y_cost, float* y_traj, float* traj_mask);
/* Warm-start trajectories [B, nmax+1, row] (comet_evaluate's warm layout) from network
 * outputs [B, out_dim]: each segment's samples interpolated to its knots.
 *   COMET_TASK_PUSH: all 7 entries interpolated; row 0 takes x0, the last row's controls
 *     are zero.  `modes` may be NULL.
 *   COMET_TASK_PUSH_TIMED: as COMET_TASK_PUSH with 8 entries, the duration (entry 7)
 *     clamped to [0.02, 0.2] s.
 *   COMET_TASK_FLIP: the 8 states interpolated, row 0 takes x0; controls from the states
 *     and `modes` (required): accelerations and face-coordinate rates by forward
 *     differences over dt = 0.1 s, a contact finger pushes with mg/2 normal force (a
 *     sliding one on its cone edge in the slip direction), a free finger zero; the last
 *     row's controls are zero.
 *   COMET_TASK_PUSH_FREE (row 9), COMET_TASK_PUSH_FREE_TIMED (row 10): states and forces
 *     interpolated (with optimised timing also the duration, entry 9, clamped to
 *     [0.02, 0.2] s), row 0 takes x0; the pusher velocity of interval k is
 *     (p_{k+1} - p_k) / h_k of the decoded positions (h_k = 0.1 s with the fixed step);
 *     the last row's controls are zero.  `modes` may be NULL.  out_dim >= 962.
 * For the other tasks out_dim >= 722.  A sequence with invalid segment or knot counts (as
 * for comet_mlp_targets) gets zero rows with x0 in row 0. */
comet_status comet_mlp_decode_warm(comet_task task, void* stream, int64_t B, const float* out, int32_t out_dim,
                                   const float* x0, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                                   int32_t smax, int32_t nmax, float* warm);

/* Microbenchmarks of the device's peak rates, the denominators of roofline figures
 * (measured on the current device and stream; synchronises; allocates 2 GiB of scratch
 * for the copy and frees it).  out: host, 4 doubles:
 *   [0] FP32 vector FMA rate, TFLOP/s (non-packed instructions: packed FP32 is disabled in
 *       this library)
 *   [1] FP64 vector FMA rate, TFLOP/s
 *   [2] BF16 matrix-core rate (v_mfma_f32_16x16x32_bf16, dense), TFLOP/s
 *   [3] device-to-device copy, GB/s (bytes read + written)
 * COMET_ENOMEM if the scratch does not fit, COMET_EHIP on a runtime failure. */
comet_status comet_probe_peaks(void* stream, double* out);

#ifdef __cplusplus
}
#endif
#endif
