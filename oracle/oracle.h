/* oracle.h -- plain CPU reference of the population-parallel local search
 * (cuGenOpt, arXiv 2603.19163, Alg. 1 per-generation evolution, Alg. 2 / Eq. ema
 * adaptive operator selection, Sec. "Population Management" initialisation).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only tests, the smoke check and the benchmark's CPU-baseline
 * leg load liboracle.so.  It is deliberately slow: every candidate is a real
 * copy of the solution, every objective a full recomputation from its
 * definition.
 */
#ifndef GX_ORACLE_H
#define GX_ORACLE_H
#include <stdint.h>

/* Operator ids (Tab. "operators"): permutation 0 2-opt, 1 swap, 2 insert,
 * 3 or-opt, 4 3-opt; ids 5-7 are the LNS operators on single-row
 * permutations (5 segment shuffle, 6 scatter shuffle, 7 guided rebuild; Sec.
 * "Built-in Operator Hierarchy") and the row operators on multi-row solutions
 * (5 row_swap, 6 row_split, 7 row_merge); binary 8 flip, 9 seg_flip; integer
 * 10 random_reset, 11 seg_reset. */
#define OR_MAX_OPS 12

/* kind 1 TSP, 2 QAP, 3 knapsack, 4 VRPTW as a giant tour split by capacity,
 * 5 colouring, 6 VRPTW in the multi-row form (Sec. "Solution Structure"): n
 * customers and `vehicles` rows; a solution holds n + vehicles entries, the
 * customers (entry c is node c + 1) and one marker per row (entries n ..
 * n + vehicles - 1), each row's customers followed by its marker. */
typedef struct {
  int32_t kind, n;
  const int32_t *a, *b;
  int32_t a_is_coords, capacity, vehicles, service_time, horizon, lb, ub, n_edges;
  uint32_t key;
  int32_t obj_w[3];   /* VRPTW: weights of distance, routes, longest route; all 0 = (1, 0, 0) */
  /* VRPTW lexicographic mode (Sec. "Multi-Objective Optimization Modes"):
   * objectives in priority order (1 distance, 2 routes, 3 longest route; 0
   * ends the list; lex_order[0] = 0 is the weighted mode) and the tolerance
   * of each level */
  int32_t lex_order[3], lex_tol[3];
} or_inst_desc;

typedef struct {
  uint64_t seed;
  uint32_t generations, population, candidates, op_mask;
  uint64_t t0_q16;
  uint32_t alpha_q32, epoch, aos_alpha_q16, w_floor_q16, stagnation_epochs, credit, oversample_k;
  /* Sec. "Island Model and Elite Injection": islands (0 or 1: none), migration
   * every migrate_epochs epochs (0: never) in mode 0 ring, 1 top-N, 2 hybrid,
   * N = migrate_n (0: 1), elite injection every elite_epochs epochs (0: never) */
  uint32_t islands, migrate_epochs, migrate_mode, migrate_n, elite_epochs;
  /* Alg. 2 scope of the weight statistics: 0 the instance (counts of all
   * solutions pooled), 1 each solution on its own (or_sol_aos below) */
  uint32_t aos_scope;
  /* initial raw operator weights, Q16; 0 selects the Tab. weight_preset value */
  uint32_t init_w[OR_MAX_OPS];
  /* per-operator weight caps (Q16, <= 65536); 0 selects the default: the LNS
   * cap of Tab. weight_preset for the LNS operators, 1.0 for the others */
  uint32_t cap_w[OR_MAX_OPS];
} or_params;

/* Per-solution adaptive-operator-selection state (aos_scope = 1). */
typedef struct {
  uint32_t w_op[OR_MAX_OPS], w_k[3], stag;
  int64_t epoch_ref;                  /* the solution's best at the start of the epoch */
  uint32_t u_op[OR_MAX_OPS], v_op[OR_MAX_OPS], u_k[3], v_k[3];
} or_sol_aos;

/* Epoch-boundary state of one solve.  Arrays are caller-owned. */
typedef struct {
  uint32_t g, stag;
  uint64_t T_q16;
  int64_t epoch_ref;                  /* instance best at the start of the epoch */
  uint32_t w_op[OR_MAX_OPS], w_k[3];
  uint32_t pad_;
  uint64_t u_op[OR_MAX_OPS], v_op[OR_MAX_OPS], u_k[3], v_k[3]; /* current-epoch counts */
  uint64_t accepted;                  /* accepted moves over the whole run */
  uint64_t tot_u_op[OR_MAX_OPS], tot_v_op[OR_MAX_OPS], tot_u_k[3], tot_v_k[3]; /* run totals of the counts */
  int32_t *cur;                       /* P x n */
  int64_t *cur_f;                     /* P     */
  int32_t *best;                      /* P x n */
  int64_t *best_f;                    /* P     */
  or_sol_aos *saos;                   /* P entries when aos_scope = 1, else NULL */
  /* lexicographic mode: objective vectors (penalty, then the priority levels)
   * of the current and best solutions (P x 4) and of the instance best at the
   * start of the epoch */
  int64_t *cur_v, *best_v;
  int64_t ref_v[4];
} or_state;

typedef struct or_inst or_inst;

void    or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void    or_philox_many(const uint32_t *ctr, int64_t count, const uint32_t key[2], uint32_t *out);
int32_t or_nint_dist(int32_t x1, int32_t y1, int32_t x2, int32_t y2);
uint64_t or_isqrt(uint64_t v);
uint32_t or_accept_threshold(uint64_t delta, uint64_t t_q16, int *reject_outright);
uint64_t or_cool(uint64_t t_q16, uint32_t alpha_q32);

or_inst *or_inst_new(const or_inst_desc *d);   /* NULL on invalid input */
void     or_inst_free(or_inst *);
int64_t  or_objective(const or_inst *, const int32_t *x);
int32_t  or_dist(const or_inst *, int32_t u, int32_t v);  /* TSP / VRPTW distances */
int      or_apply_op(const or_inst *, int32_t *x, int op, uint32_t w1, uint32_t w2, uint32_t w3);
void     or_initial_weights(const or_inst *, uint32_t op_mask, const uint32_t *init_w, uint32_t w_op[OR_MAX_OPS]);
void     or_aos_update(const or_inst *, const or_params *, uint32_t op_mask, or_state *st, int64_t inst_best_now);
int      or_lns_len(int n);                     /* entries an LNS step destroys */
uint32_t or_lns_cap(const or_inst *);           /* Q16 weight cap of the LNS operators (0: none) */
void     or_migrate(const or_inst *in, const or_params *, int n, or_state *st, uint32_t epoch);  /* epoch: 1-based count */
int      or_heuristic_perms(const or_inst *, int32_t *out, int cap); /* returns count */
int      or_init(const or_inst *, const or_params *, or_state *st);
void     or_random_solution(const or_inst *, const or_params *, uint32_t pool_index, int32_t *x);
int      or_wpick(uint32_t u16, const uint32_t *w, int cnt);  /* Q16 roulette */
int      or_lex_mode(const or_inst *);
void     or_lex_vector(const or_inst *, const int32_t *x, int64_t v[4]);
int      or_lex_better(const or_inst *, const int64_t a[4], const int64_t b[4]);
int      or_lex_best(const or_inst *, const or_state *st, int population);   /* ordered scan of the bests */
int      or_run(const or_inst *, const or_params *, or_state *st, uint32_t n_gens);
/* the same generations on `threads` threads (solutions split between them
 * inside each epoch); equal to or_run */
int      or_run_par(const or_inst *, const or_params *, or_state *st, uint32_t n_gens, int threads);
uint32_t or_effective_mask(const or_inst *, uint32_t op_mask);

#endif
