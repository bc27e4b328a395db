/* gx.h -- C interface of the MI355X population-parallel local-search engine.
 *
 * The engine runs the per-generation evolution step of cuGenOpt (arXiv
 * 2603.19163, Alg. 1): one HIP workgroup evolves one solution of a
 * permutation, binary or integer encoding; each generation samples C
 * composite moves (k in {1,2,3} operators, Tab. "operators"), evaluates their
 * exact integer objective deltas against instance data staged in LDS, takes
 * the wavefront argmin, applies simulated-annealing acceptance and collects
 * adaptive-operator-selection statistics; every E generations the operator
 * and K-step weights are updated (Eq. ema, Alg. 2).  Initialisation follows
 * Sec. "Population Management" (oversampled pool with row/column-sum
 * heuristics).  All arithmetic is integer, and all randomness comes from a
 * counter-based generator keyed by (seed) with counter (generation, solution,
 * candidate/slot, instance key), so results are bit-reproducible and
 * independent of launch shape, batching and scheduling.
 *
 * Conventions
 *  - Every call returns gx_status (GX_OK = 0, negative on error) and never
 *    throws; gx_last_error(ctx) describes the last failure on that context.
 *  - The caller owns every host buffer it passes; the library owns every
 *    device allocation it makes and frees it in the matching *_free call or
 *    in gx_destroy.
 *  - All work is ordered on the context's HIP stream (the stream given to
 *    gx_create, or one the context creates).  Calls that return results to
 *    host memory synchronise that stream first.
 *  - A gx_ctx is not thread-safe; use one context per host thread.
 *  - The library never falls back to a CPU path: without a usable gfx950
 *    device gx_create fails with GX_E_DEVICE.
 */
#ifndef GX_H
#define GX_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gx_status;
enum {
  GX_OK = 0,
  GX_E_INVALID = -1,      /* an argument is out of its documented domain */
  GX_E_UNSUPPORTED = -2,  /* valid, but beyond the library's kernel limits */
  GX_E_NOMEM = -3,        /* device or host allocation failed */
  GX_E_DEVICE = -4,       /* a HIP runtime error (message in gx_last_error) */
  GX_E_NOT_READY = -5,    /* gx_poll: work still running */
  GX_E_BUSY = -6,         /* admission refused for now (server) */
  GX_E_CANCELLED = -7
};

/* Problem kinds; the encoding follows from the kind (Sec. "Encoding Types"). */
typedef enum {
  GX_TSP = 1,       /* permutation; symmetric travelling salesman */
  GX_QAP = 2,       /* permutation; quadratic assignment, p[i] = location of facility i */
  GX_KNAPSACK = 3,  /* binary; 0/1 knapsack, penalised overweight */
  GX_VRPTW = 4,     /* permutation of customers (giant tour) split into routes */
  GX_INTCOLOR = 5,  /* integer in [lb, ub]; graph colouring (monochromatic edges) */
  GX_VRPTW_ROWS = 6 /* multi-row permutation: one route per row (Sec. "Solution Structure") */
} gx_problem;

/* Operators (paper, Tab. "operators"); bit i of op_mask enables operator id
 * i, and AOS keeps one weight per id.  Ids are contiguous per encoding:
 * permutation 0-4, plus 5-7 the LNS operators on single-row permutations
 * (TSP, QAP, VRPTW giant tour) and the row operators on multi-row ones;
 * binary 8-9, integer 10-11.  op_mask 0 takes every operator of the encoding
 * but the LNS ones, which run only when named. */
#define GX_N_OPS 12
enum {
  GX_OP_2OPT = 1u << 0,    /* element level: segment reversal */
  GX_OP_SWAP = 1u << 1,    /* element level */
  GX_OP_INSERT = 1u << 2,  /* element level: move one element */
  GX_OP_OROPT = 1u << 3,   /* segment level: move a block of 2 or 3 elements, orientation kept */
  GX_OP_3OPT = 1u << 4,    /* segment level: three cuts a < b < c, blocks [a, b) and [b, c) exchanged */
  /* LNS (single-row permutations; Sec. "Built-in Operator Hierarchy"): a step
   * destroys L = min(n, 2 + n/16, 64) entries and rebuilds them; its draws
   * beyond the step's words w1..w3 are word i mod 4 of the Philox4x32-10
   * block with counter (w1, w2, w3, i/4) and key (0x4C4E5331, 0x4C4E5332).
   * Initial weights 0.006 / 0.004 / 0.001 and a weight cap of 0.02 / 0.01 /
   * 0.005 (Tab. weight_preset, n <= 100 / <= 250 / > 250): the EMA update
   * clamps an LNS weight to [min(w_floor, cap), cap]. */
  GX_OP_LNS_SEGMENT = 1u << 5, /* shuffle the L entries from a uniform start (Fisher-Yates) */
  GX_OP_LNS_SCATTER = 1u << 6, /* shuffle the entries at L distinct uniform positions (Floyd's sampling) */
  GX_OP_LNS_GUIDED = 1u << 7,  /* the L entries from a uniform start in order of their heuristic key
                                  (row sums of the first data matrix), ascending, or descending when
                                  the top bit of w2 is set; ties by entry */
  /* row level (GX_VRPTW_ROWS); p is drawn uniformly among the entries before
   * the final marker and names the row holding it (its marker included) */
  GX_OP_ROWSWAP = 1u << 5,  /* that row and the next trade places (nothing for the last row) */
  GX_OP_ROWSPLIT = 1u << 6, /* when the last row is empty, its marker moves to p: the row ends
                               before p's entry and the rest opens a row (else nothing) */
  GX_OP_ROWMERGE = 1u << 7, /* the row's marker moves before the final one: the next row's
                               customers join it and the last row is left empty (nothing when
                               the next row is the empty last row, or there is none) */
  GX_OP_FLIP = 1u << 8,    /* binary, element level: flip one bit */
  GX_OP_SEGFLIP = 1u << 9, /* binary, segment level: flip L = 2..7 consecutive bits */
  GX_OP_RESET = 1u << 10,  /* integer, element level: draw a new value in [lb, ub] */
  GX_OP_SEGRESET = 1u << 11 /* integer, segment level: set L = 2..7 consecutive elements to one new value */
};

/* Where a TSP instance's distances live during the evolve kernel. */
enum {
  GX_STAGE_AUTO = 0,
  GX_STAGE_LDS_D16 = 1,  /* int16 distance matrix copied into LDS (n <= 181) */
  GX_STAGE_LDS_XY = 2,   /* coordinates in LDS, exact integer distance recomputed */
  GX_STAGE_GLB_D16 = 3,  /* int16 distance matrix read through L2 */
  GX_STAGE_GLB_D32 = 4   /* int32 distance matrix read through L2 */
};

typedef struct gx_ctx gx_ctx;
typedef struct gx_instance gx_instance;
typedef struct gx_job gx_job;

/* Create a context on device `device_ordinal`.  `hip_stream` is a hipStream_t
 * to order all work on, or NULL for a stream the context creates and owns.
 * Fails with GX_E_DEVICE if the device is not a gfx950. */
gx_status gx_create(int device_ordinal, void *hip_stream, gx_ctx **out);
/* Free every device allocation of the context (instances, jobs) and the context. */
gx_status gx_destroy(gx_ctx *ctx);
/* Text of the last error on `ctx` (valid until the next call on it); never NULL. */
const char *gx_last_error(const gx_ctx *ctx);

typedef struct {
  int32_t cus;                 /* compute units */
  int32_t lds_per_block;       /* bytes of LDS one workgroup may use */
  int32_t wave_size;
  int32_t l2_bytes;
  char arch[64];
} gx_device_info;
gx_status gx_get_device_info(gx_ctx *ctx, gx_device_info *out);

/* Instance description.  All arrays are int32, row-major, in host memory
 * (is_device_ptr = 0) or device memory on the context's device
 * (is_device_ptr = 1); they are copied before gx_instance_upload returns.
 *   TSP      a = coordinates n x 2 (a_is_coords = 1) or a symmetric distance
 *            matrix n x n with zero diagonal and entries in [0, 2^24)
 *            (a_is_coords = 0).  Distance between coordinates is the nearest
 *            integer of the Euclidean distance.  Coordinates in [0, 2^14).
 *   QAP      a = flow F n x n, b = distance D n x n, both symmetric, entries
 *            in [0, 2^14); f(p) = sum_ij F[i][j] D[p_i][p_j].  n <= 64.
 *   KNAPSACK a = weights (n), b = values (n), entries in [0, 2^20];
 *            f(x) = -sum v x + (max v + 1) * max(0, sum w x - capacity).
 *   VRPTW    n = number of customers; a = coordinates (n+1) x 2, depot in
 *            row 0; b = demand, ready, due, each (n+1) (3 x (n+1) array);
 *            capacity, vehicles, service_time, horizon.  Customers are
 *            visited in tour order and a new route opens whenever the load
 *            would exceed capacity; f = wD * distance + wR * routes
 *            + wM * (length of the longest route) + 100 * total lateness
 *            + 10000 * max(0, routes - vehicles), with (wD, wR, wM) =
 *            obj_weights (paper, Sec. "Multi-Objective Optimization Modes":
 *            the weighted mode over distance, vehicle count and the longest
 *            route; each weight in [0, 2^20]; all zero means (1, 0, 0), the
 *            single objective).  n <= 250; coordinates in [0, 2^14), demand
 *            in [0, capacity], times in [0, 2^19].
 *            Lexicographic mode (paper, Sec. "Multi-Objective Optimization
 *            Modes"; Tab. lexicographic_mode) when lex_order[0] != 0: a
 *            solution's objective is the vector (penalty, level 1, level 2,
 *            level 3), penalty = 100 * lateness + 10000 * fleet excess (+ 100 *
 *            load above capacity in the multi-row form), level
 *            i the objective lex_order[i] (1 distance, 2 routes, 3 longest
 *            route; a 0 ends the list; no repeats).  b is better than a when
 *            its penalty is lower, or the penalties are equal and at the
 *            first level where the two differ by more than lex_tol[i]
 *            (in [0, 2^30]) b's value is the lower one; otherwise neither is
 *            better.  Within a set (the candidates of a generation, the
 *            population) the best is found by a scan in index order in
 *            which a later element replaces the one kept when better.  The
 *            scalar reported for a solution (cur_f, best_f, the best
 *            objective) is its penalty plus its level-1 value; island
 *            migration and elite injection pick best and worst solutions by
 *            the same relation.  obj_weights must be zero in this mode;
 *            solves on such an instance take aos_scope 0 and cannot be
 *            restored (gx_job_restore).
 *   VRPTW_ROWS  the VRPTW data and modes (above) in the multi-row form of
 *            Sec. "Solution Structure" (Tab. generality runs CVRP and VRPTW
 *            so): `vehicles` rows (>= 1, <= 250), one route each.  A
 *            solution holds n + vehicles entries: entry e < n is customer
 *            e + 1, entries n .. n + vehicles - 1 are row markers; the rows
 *            come one after another, each followed by its marker, and the
 *            final entry is a marker (the paper's rows of per-row length,
 *            stored back to back).  A row is a route from the depot through
 *            its customers in order and back; an empty row is no route.  f as
 *            for VRPTW with routes = non-empty rows (the fleet term is then
 *            0) plus 100 * (load above capacity, summed over rows).
 *            capacity <= 2^22.  Operators: the permutation ones act on the
 *            entries before the final marker, the row ones on whole rows.
 *            Initial pool slot 0 is the sweep solution of Sec. "Partition
 *            Encoding Heuristic Initialization" (customers by polar angle
 *            about the depot fill the rows in turn up to the capacity, each
 *            row then ordered by due time, ready time, index); the others
 *            shuffle the entries before the final marker.
 *   INTCOLOR a = edge list n_edges x 2 (no self loops); values in [lb, ub];
 *            f = number of edges whose ends share a value.
 * instance_key enters every random counter of solves on this instance: keep
 * it stable for a request, independent of where it runs in a batch. */
typedef struct {
  int32_t kind, n, is_device_ptr;
  const int32_t *a, *b;
  int32_t a_is_coords, capacity, vehicles, service_time, horizon, lb, ub, n_edges;
  uint32_t instance_key;
  int32_t obj_weights[3];   /* VRPTW objective weights (above); zero for the other kinds */
  int32_t lex_order[3];     /* VRPTW lexicographic mode (above); zero: the weighted mode */
  int32_t lex_tol[3];
} gx_instance_desc;
gx_status gx_instance_upload(gx_ctx *ctx, const gx_instance_desc *desc, gx_instance **out);
gx_status gx_instance_free(gx_ctx *ctx, gx_instance *inst);

/* Solve parameters (Alg. 1 and Alg. 2; Sec. "Adaptive Operator Selection";
 * Sec. "Problem-Profile-Driven Prior Strategy"); integer only; 0 selects the
 * default in brackets.
 *  seed            key of the counter-based generator
 *  generations     generations G to run (>= 1 for gx_solve)
 *  population      P solutions, one workgroup each [0: CUs x resident workgroups per CU]
 *  candidates      C sampled composite moves per solution per generation [128], <= 65536
 *  op_mask         GX_OP_* bits [all operators of the encoding]
 *  t0_q16          initial temperature, Q16 [a quarter of |f|/n of the best start]
 *  alpha_q32       cooling factor per generation, Q32 (required, >= 1)
 *  aos_epoch       generations E between AOS weight updates [10]
 *  aos_alpha_q16   EMA factor of the weight update, Q16 [49152 = 0.75]
 *  w_floor_q16     weight floor, Q16 [1024 = 1/64]
 *  stagnation_epochs  epochs without improvement of the instance best before
 *                  the K-step weights reset to (0.8, 0.15, 0.05) [5]
 *  aos_credit      0 every candidate credits its operators, 1 only the accepted move [0]
 *  oversample_k    pool of oversample_k * P starting solutions [4]
 *  staging         GX_STAGE_* for TSP [GX_STAGE_AUTO]
 *  aos_scope       0 the weights of the instance, updated from the counts of
 *                  all P solutions (Alg. 2); 1 each solution keeps its own
 *                  weights, counts and stagnation count, updated the same way
 *                  from its own candidates and its own best objective
 *                  (aos_epoch * candidates <= 2^30) [0]
 *  init_weight_q16 raw initial weight of operator id i, Q16 in [1, 2^24]; 0
 *                  takes the Tab. weight_preset value (1.0; or-opt 0.8 / 0.7 /
 *                  0.3 and 3-opt 0.5 / 0.3 / 0.05 for n <= 100, <= 250, > 250);
 *                  the enabled operators' raw weights are then normalised
 *  weight_cap_q16  per-sequence weight cap of operator id i, Q16 in [1, 2^16]
 *                  (Sec. "Two-Level Weight Structure": the Eq. ema update
 *                  clamps weight i to [w_floor, min(1, cap_i)], to [cap_i,
 *                  cap_i] when cap_i is below the floor); 0 takes the default:
 *                  the LNS cap of Tab. weight_preset for the LNS operators,
 *                  1.0 for the others
 * Island model and elite injection (paper, Sec. "Island Model and Elite
 * Injection"), applied at the end of an AOS epoch e, after the weight update:
 *  islands         I islands of P / I consecutive solutions (P a multiple of
 *                  I, at least 2 per island, I <= 64) [0: one population]
 *  migrate_epochs  migration when e is a multiple of it [0: never]: the
 *                  elites (best-so-far solutions) replace the worst current
 *                  solutions of the receiving islands, all chosen before the
 *                  first copy; mode 0 ring (island i's best to island i+1),
 *                  1 top-N (the population's N best to every island), 2 hybrid
 *                  (ring when e / migrate_epochs is odd, top-N when even) [0]
 *  migrate_n       N of top-N, <= 8 and below the island size [1]
 *  elite_epochs    elite injection when e is a multiple of it: the
 *                  population's best replaces its worst [0: never]
 * "best" is the smallest (best objective, index), "worst" the largest
 * (current objective, index); a replaced solution takes the elite as its
 * current solution, and as its own best when that improves it. */
typedef struct {
  uint64_t seed;
  uint32_t generations, population, candidates, op_mask;
  uint64_t t0_q16;
  uint32_t alpha_q32, aos_epoch, aos_alpha_q16, w_floor_q16;
  uint32_t stagnation_epochs, aos_credit, oversample_k, staging;
  uint32_t islands, migrate_epochs, migrate_mode, migrate_n;
  uint32_t elite_epochs, aos_scope;
  uint32_t init_weight_q16[GX_N_OPS];
  uint32_t weight_cap_q16[GX_N_OPS];
} gx_solve_params;

/* Population the library would use for P = 0 on this instance: the CUs times
 * the workgroups one CU holds at the evolve kernel's registers and LDS (at
 * most 32 per CU).  The paper sizes P from the L2 capacity (Eq. pop_sizing);
 * this sizing is the gfx950 build's own. */
gx_status gx_autosize_population(gx_ctx *ctx, const gx_instance *inst, const gx_solve_params *p,
                                 uint32_t *population_out);

/* Allocate a job and run the initialisation (Sec. "Population Management":
 * oversampled pool of oversample_k * P starts, the row/column-sum heuristics
 * of Sec. "Attribute-Agnostic Heuristic Initialization", selection of the
 * best P; initial temperature and weights) on the stream.  Fails with
 * GX_E_INVALID or GX_E_UNSUPPORTED as gx_solve does. */
gx_status gx_job_create(gx_ctx *ctx, const gx_instance *inst, const gx_solve_params *p, gx_job **out);
/* Enqueue `n_generations` more generations of Alg. 1, with the epoch update
 * of Alg. 2 every aos_epoch generations (asynchronous).  GX_E_INVALID for a
 * batched job or a total beyond 2^32 - 2 generations. */
gx_status gx_job_advance(gx_ctx *ctx, gx_job *job, uint32_t n_generations);
/* gx_job_create followed by gx_job_advance(generations) (Alg. 1 run for a
 * generation budget in place of the paper's time limit).  *out receives the
 * job, which the caller frees with gx_job_free.  GX_E_INVALID for null
 * arguments, generations = 0, alpha_q32 = 0, an op_mask with no operator of
 * the encoding or a parameter out of its range above; GX_E_UNSUPPORTED when
 * the instance needs more LDS than a workgroup has. */
gx_status gx_solve(gx_ctx *ctx, const gx_instance *inst, const gx_solve_params *p, gx_job **out);
/* Solve without allocating: for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Runs the same solve as gx_solve (same result for the same
 * instance and parameters) with all of its device state in a static
 * workspace of 64 MiB that each device holds for the life of the process,
 * and writes the best solution (n int32) to best_solution and its objective
 * to best_objective, both caller-owned device memory.  Asynchronous on the
 * context's stream (gx_wait(ctx, NULL) waits for it).  Every call on one
 * device shares that device's workspace: calls must not overlap on a device
 * (calls on one context's stream follow each other; calls from other
 * contexts or streams of the same device race).  GX_E_UNSUPPORTED when the
 * solve needs more than the workspace (about 4 (2 + oversample_k) P n bytes
 * plus the instance-independent records) or int32 distances the instance
 * does not already hold; other errors as gx_solve.  Calls no allocator. */
gx_status gx_solve_static(gx_ctx *ctx, const gx_instance *inst, const gx_solve_params *p, int32_t *best_solution,
                          int64_t *best_objective);
/* Wait for everything enqueued on the context's stream (and record the
 * job's evolve time, gx_job_info.evolve_ms). */
gx_status gx_wait(gx_ctx *ctx, gx_job *job);
/* GX_OK if the job's enqueued work has finished, GX_E_NOT_READY otherwise. */
gx_status gx_poll(gx_ctx *ctx, gx_job *job);
/* Best solution found (the paper returns the best of the population: the
 * minimum of (best objective, solution index)) into solution_out[capacity >=
 * n] (may be NULL) and its objective into *objective_out; synchronises the
 * stream.  GX_E_INVALID when capacity < n. */
gx_status gx_fetch_best(gx_ctx *ctx, gx_job *job, int32_t *solution_out, int32_t capacity,
                        int64_t *objective_out);
/* Portfolio selection (paper, Sec. "Multi-GPU" runs: independent solves of
 * one instance with different seeds, the best kept; here the solves share one
 * device, e.g. the jobs of one gx_solve_batch call): among count >= 1 jobs of
 * the same instance, the one whose best objective is smallest (ties: the
 * lowest position in jobs; in the VRPTW lexicographic mode the jobs' best
 * objective vectors are compared by that mode's relation, in job order, a
 * later job replacing the one kept only when strictly better); its index
 * into *index_out, its objective into
 * *objective_out and its best solution into solution_out[capacity >= n].
 * GX_E_INVALID for null arguments, count < 1 or jobs of different instances.
 * Synchronises the stream. */
gx_status gx_portfolio_best(gx_ctx *ctx, gx_job *const *jobs, int32_t count, int32_t *solution_out,
                            int32_t capacity, int64_t *objective_out, int32_t *index_out);

/* Run facts of a job (synchronises the stream).  op_steps and k_count count
 * every evaluated candidate's operators and k (zero with aos_credit = 1). */
typedef struct {
  uint32_t population, candidates, generations_done, staging;
  uint64_t move_evals;        /* P * C * generations run */
  uint64_t accepted;
  uint32_t evolve_launches;   /* evolve-kernel launches so far */
  float evolve_ms;            /* device time between the first and last evolve launch of the
                                 last gx_job_advance (HIP events on the context stream) */
  uint64_t op_steps[GX_N_OPS]; /* operator steps evaluated over the run, per operator id */
  uint64_t k_count[3];        /* candidates with k = 1, 2, 3 operators over the run */
} gx_job_info;
gx_status gx_job_info_get(gx_ctx *ctx, gx_job *job, gx_job_info *out);

/* Run totals of the adaptive-operator-selection statistics (Sec. "Statistics
 * Collection and Weight Update": per operator its uses u and improvements v,
 * per k the same) as credited under aos_credit, summed over every generation
 * and solution so far; synchronises the stream. */
typedef struct {
  uint64_t move_evals, accepted;
  uint64_t u_op[GX_N_OPS], v_op[GX_N_OPS], u_k[3], v_k[3];
  uint32_t generations_done, population;
} gx_run_stats;
gx_status gx_job_stats(gx_ctx *ctx, gx_job *job, gx_run_stats *out);
/* Population P of a job (the autosized one when population was 0). */
gx_status gx_job_population(gx_ctx *ctx, gx_job *job, uint32_t *population_out);

/* Scalars of the job state at a generation boundary (Alg. 1 temperature,
 * Alg. 2 weights, epoch statistics and stagnation count). */
typedef struct {
  uint32_t g, stag;
  uint64_t T_q16;
  int64_t epoch_ref;          /* instance best at the start of the current epoch */
  uint32_t w_op[GX_N_OPS], w_k[3], pad_;
  uint64_t u_op[GX_N_OPS], v_op[GX_N_OPS], u_k[3], v_k[3];   /* statistics of the current epoch */
  uint64_t accepted;
} gx_state_scalars;
/* Copy the job state to host buffers (any array may be NULL); synchronises.
 * cur and best are P x n int32, cur_f and best_f P int64. */
gx_status gx_snapshot(gx_ctx *ctx, gx_job *job, gx_state_scalars *sc, int32_t *cur, int64_t *cur_f,
                      int32_t *best, int64_t *best_f);
/* Per-solution AOS state (aos_scope = 1): weights, stagnation count, the
 * solution's best at the start of the epoch, the epoch's counts. */
typedef struct {
  uint32_t w_op[GX_N_OPS], w_k[3], stag;
  int64_t epoch_ref;
  uint32_t u_op[GX_N_OPS], v_op[GX_N_OPS], u_k[3], v_k[3];
} gx_sol_aos;
/* The P per-solution records into out[P]; synchronises. */
gx_status gx_snapshot_aos(gx_ctx *ctx, gx_job *job, gx_sol_aos *out);
/* Objective vectors of a job on a VRPTW instance in the lexicographic mode
 * (paper, Sec. "Multi-Objective Optimization Modes"): cur_v and best_v are
 * P x 4 int64 (penalty, level 1, level 2, level 3; unused levels 0) of the
 * current and best-so-far solutions, ref_v (4 int64) the instance best's
 * vector at the last epoch end (the stagnation reference).  Any pointer may
 * be NULL; host memory.  GX_E_INVALID for a job not in that mode;
 * synchronises. */
gx_status gx_snapshot_lex(gx_ctx *ctx, gx_job *job, int64_t *cur_v, int64_t *best_v, int64_t *ref_v);
/* Resume from a snapshot: overwrite a non-batched job's state at a generation
 * boundary with sc, cur, cur_f, best, best_f (all required, as gx_snapshot
 * fills them) and, with aos_scope = 1, the P records of aos (else ignored).
 * Continuing the job then gives the generations the snapshotted job would
 * have run (same instance and parameters).  GX_E_INVALID for a batched job,
 * a null array, sc->g beyond the job's generation budget, or a permutation
 * or value that is not a solution of the instance; GX_E_UNSUPPORTED for a
 * job in the lexicographic mode; synchronises. */
gx_status gx_job_restore(gx_ctx *ctx, gx_job *job, const gx_state_scalars *sc, const int32_t *cur,
                         const int64_t *cur_f, const int32_t *best, const int64_t *best_f, const gx_sol_aos *aos);
gx_status gx_job_free(gx_ctx *ctx, gx_job *job);

/* Batched solve: `count` instances with their own parameters, run together
 * in one persistent launch per AOS epoch (the launch sequence is captured
 * into a HIP graph).  Each job's result equals the result of gx_solve on the
 * same instance and parameters.  jobs_out[i] receives job i. */
gx_status gx_solve_batch(gx_ctx *ctx, const gx_instance *const *insts, const gx_solve_params *params,
                         int32_t count, gx_job **jobs_out);

/* ---- Serving: continuous batching of solve requests.
 * A server owns a device arena and a scheduler thread.  Requests are admitted
 * in arrival order as soon as their device footprint (instance data, solution
 * state, initial pool) fits the arena and a resident slot is free; requests
 * that do not fit wait without blocking smaller ones behind them.  Requests
 * are grouped into lanes by kind, staging and LDS class, each lane with its own
 * stream; a lane's scheduling quantum advances every resident request of the
 * lane by several AOS epochs (16 for TSP, knapsack and colouring, 4 for QAP and
 * VRPTW), each one fused launch over all their solutions, so requests that
 * arrive while others run overlap with them on the device.  Finished requests return their best
 * solution and free their memory.  A result depends only on the request
 * (instance, parameters, seed, instance key), never on what else is resident,
 * so it equals gx_solve on the same request. */
typedef struct gx_server gx_server;
typedef struct {
  uint64_t hbm_budget_bytes;   /* arena for resident requests [1 GiB] */
  uint32_t max_resident;       /* requests resident at once [1024] */
  uint32_t max_lds_bytes;      /* LDS per workgroup a request may need [65536] */
  uint32_t max_items;          /* solutions (workgroups) resident at once; further
                                  requests wait in arrival order [40 x CUs] */
  uint32_t quantum_epochs;     /* AOS epochs a lane advances per quantum [16 for TSP,
                                  knapsack and colouring, 4 for QAP and VRPTW] */
  uint32_t reserved;
} gx_server_cfg;
typedef struct {
  uint64_t submitted, admitted, completed, cancelled;
  uint64_t quanta, move_evals;
  uint32_t resident, pending;
  uint64_t arena_used_bytes, arena_bytes;
  double busy_seconds;         /* wall time with at least one request resident */
} gx_server_stats;
/* Start a server on the context's device (it uses a stream of its own). */
gx_status gx_server_create(gx_ctx *ctx, const gx_server_cfg *cfg, gx_server **out);
/* Thread-safe.  Copies the instance (host pointers only); validates it and the
 * parameters (population must be given, >= 1); GX_E_UNSUPPORTED if the request
 * can never fit the arena or the LDS limit.  *ticket identifies the request. */
gx_status gx_server_submit(gx_server *srv, const gx_instance_desc *desc, const gx_solve_params *p,
                           uint64_t *ticket);
/* Thread-safe.  GX_E_NOT_READY while queued or running; GX_E_CANCELLED after a
 * cancel; GX_OK with the best solution (capacity >= n), its objective, and the
 * submit and completion times (steady clock, ns).  A completed or cancelled
 * ticket is forgotten after it has been reported once (then GX_E_INVALID). */
gx_status gx_server_poll(gx_server *srv, uint64_t ticket, int32_t *solution_out, int32_t capacity,
                         int64_t *objective_out, uint64_t *t_submit_ns, uint64_t *t_done_ns);
/* Thread-safe.  Drops a queued or running request; other requests are unaffected. */
gx_status gx_server_cancel(gx_server *srv, uint64_t ticket);
gx_status gx_server_stats_get(gx_server *srv, gx_server_stats *out);
/* Stops the scheduler, waits for in-flight work and frees the arena. */
gx_status gx_server_destroy(gx_server *srv);

/* Exponential tables of the acceptance test (host copies, for checking):
 * hi[i] = round(2^31 e^-i) for i < 16, lo[j] = round(2^31 e^-(j/256)) for j < 256. */
gx_status gx_exp_tables(uint32_t hi[16], uint32_t lo[256]);

/* Device arithmetic on caller-given inputs, so that the primitives the
 * kernels use can be compared with an independent implementation.  `in` and
 * `out` are host arrays of `count` elements (count <= 2^26); the call
 * synchronises the context's stream.
 *  GX_CHECK_PHILOX  Philox4x32-10 (Salmon et al., SC'11; the random source of
 *                   Alg. 1's rand()): key = k0 | k1 << 32; in[2i], in[2i+1] =
 *                   counter words c0 | c1 << 32, c2 | c3 << 32; out[4i..4i+1]
 *                   the block from the per-lane form the candidate draws use,
 *                   out[4i+2..4i+3] from the form of the single draws, each
 *                   as r0 | r1 << 32, r2 | r3 << 32.
 *  GX_CHECK_DIST    nearest-integer Euclidean distance (the TSP objective):
 *                   in[i] = x1 | y1 << 16 | x2 << 32 | y2 << 48, coordinates in
 *                   [0, 2^14) (GX_E_INVALID otherwise); out[2i] from the
 *                   int16-pair path, out[2i+1] from the int32 path.
 *  GX_CHECK_ACCEPT  acceptance threshold of Alg. 1 for a worse move:
 *                   in[2i] = delta > 0, in[2i+1] = T_q16; out[i] = the value
 *                   p a 31-bit draw must stay below, or UINT64_MAX when the
 *                   move is rejected outright (T = 0 or delta / T >= 16). */
enum { GX_CHECK_PHILOX = 1, GX_CHECK_DIST = 2, GX_CHECK_ACCEPT = 3 };

/* Device ceilings the evolve kernels are measured against, each timed with
 * HIP events on the context's stream (best of three launches after a
 * warm-up, 8 workgroups of 256 threads per CU): random 4-byte LDS reads (64
 * KiB per workgroup), Philox4x32-10 blocks of the per-lane form, full-rate
 * 32-bit multiply-adds, random 4-byte reads from a 4 MiB buffer (fits the
 * L2), and a 2 GiB read stream from HBM.  Allocates and frees its buffers;
 * synchronises the stream. */
typedef struct gx_peaks {
  double lds_gather_bytes_per_s, philox_blocks_per_s, valu_lane_ops_per_s, valu_instr_per_s;
  double l2_gather_bytes_per_s, hbm_read_bytes_per_s;
  int32_t cus, pad_;
} gx_peaks;
gx_status gx_measure_peaks(gx_ctx *ctx, gx_peaks *out);
gx_status gx_device_check(gx_ctx *ctx, int32_t what, uint64_t key, const uint64_t *in, uint64_t *out,
                          int64_t count);

#ifdef __cplusplus
}
#endif
#endif
