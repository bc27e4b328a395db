/* oracle.c -- plain CPU reference of the population-parallel local search of
 * cuGenOpt (arXiv 2603.19163).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  It shares no
 * source with the HIP path.  Everything is written from the paper's
 * definitions in the most direct form:
 *   - each candidate is a real copy of the solution with its k operators
 *     applied in order (Alg. 1, "copy(s)" then "execute sigma_i on s_t");
 *   - every objective is recomputed in full from its definition (Alg. 1,
 *     "evaluate s_t; delta_t = f(s_t) - f(s)");
 *   - argmin, acceptance, AOS statistics, cooling (Alg. 1), the EMA weight
 *     update with clamp, normalisation and stagnation reset (Eq. ema, Alg. 2,
 *     Sec. "Stagnation Detection"), oversampled initialisation with row/column
 *     sum heuristics (Sec. "Population Management").
 * Where the paper leaves a choice open (random source, integer objectives,
 * tie-breaks, the meaning of "batch", constants of the AOS update) the code
 * makes one explicit choice, marked "reading:" where it is made.
 */
#include "oracle.h"
#include "exp_tables.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

enum { K_TSP = 1, K_QAP = 2, K_KNAP = 3, K_VRPTW = 4, K_COLOR = 5, K_VRPROWS = 6 };
enum { OP_2OPT = 0, OP_SWAP = 1, OP_INSERT = 2, OP_OROPT = 3, OP_3OPT = 4, OP_ROWSWAP = 5, OP_ROWSPLIT = 6,
       OP_ROWMERGE = 7, OP_FLIP = 8, OP_SEGFLIP = 9, OP_RESET = 10, OP_SEGRESET = 11 };
/* on single-row permutations ids 5-7 are the LNS operators */
enum { OP_LNS_SEG = 5, OP_LNS_SCATTER = 6, OP_LNS_GUIDED = 7 };

struct or_inst {
  or_inst_desc d;
  int32_t *dist;   /* TSP: n x n; VRPTW: (n+1) x (n+1) */
  int32_t dn;      /* side of dist */
  int64_t lambda;  /* knapsack penalty weight */
  int32_t nc;      /* multi-row VRPTW: customers (the solution holds nc + vehicles entries, d.n) */
  int64_t *hkey;   /* permutations: heuristic key of each entry (row sums of the first data matrix) */
};

/* ------------------------------------------------------------------ RNG
 * reading: the paper only says rand(); the oracle uses Philox4x32-10
 * (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* the same block for `count` counters ctr[4i .. 4i+3] into out[4i .. 4i+3] */
void or_philox_many(const uint32_t *ctr, int64_t count, const uint32_t key[2], uint32_t *out) {
  for (int64_t i = 0; i < count; ++i) or_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

static void draw(const or_params *p, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                 uint32_t r[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
  or_philox4x32_10(ctr, key, r);
}

/* floor(w * m / 2^32): an integer in [0, m) */
static uint32_t rmap(uint32_t w, uint32_t m) { return (uint32_t)(((uint64_t)w * m) >> 32); }

/* Weighted choice from Q16 weights: u = floor(u16 * S / 2^16), smallest i with u < cumsum_i. */
int or_wpick(uint32_t u16, const uint32_t *w, int cnt) {
  uint64_t s = 0;
  for (int i = 0; i < cnt; ++i) s += w[i];
  uint64_t u = ((uint64_t)u16 * s) >> 16;
  uint64_t c = 0;
  for (int i = 0; i < cnt; ++i) {
    c += w[i];
    if (u < c) return i;
  }
  return cnt - 1;
}

/* ------------------------------------------------------------ distances */
uint64_t or_isqrt(uint64_t v) {  /* digit-by-digit integer square root */
  uint64_t res = 0, bit = (uint64_t)1 << 62;
  while (bit > v) bit >>= 2;
  while (bit) {
    if (v >= res + bit) { v -= res + bit; res = (res >> 1) + bit; }
    else res >>= 1;
    bit >>= 2;
  }
  return res;
}

/* reading: integer objective; distance = nearest integer of the Euclidean
 * distance, floor(sqrt(s) + 1/2) = (isqrt(4 s) + 1) / 2 exactly. */
int32_t or_nint_dist(int32_t x1, int32_t y1, int32_t x2, int32_t y2) {
  int64_t dx = (int64_t)x1 - x2, dy = (int64_t)y1 - y2;
  uint64_t s = (uint64_t)(dx * dx + dy * dy);
  return (int32_t)((or_isqrt(4 * s) + 1) >> 1);
}

int32_t or_dist(const or_inst *in, int32_t u, int32_t v) {
  return in->dist[(int64_t)u * in->dn + v];
}

/* ------------------------------------------------------------ instances */
or_inst *or_inst_new(const or_inst_desc *d) {
  if (!d || d->n < 1 || !d->a) return NULL;
  or_inst *in = (or_inst *)calloc(1, sizeof(or_inst));
  in->d = *d;
  int n = d->n;
  if (d->kind == K_TSP) {
    in->dn = n;
    in->dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        in->dist[(int64_t)i * n + j] =
            d->a_is_coords ? or_nint_dist(d->a[2 * i], d->a[2 * i + 1], d->a[2 * j], d->a[2 * j + 1])
                           : d->a[(int64_t)i * n + j];
  } else if (d->kind == K_VRPTW || d->kind == K_VRPROWS) {
    if (!d->b || (d->kind == K_VRPROWS && d->vehicles < 1)) { free(in); return NULL; }
    if (d->obj_w[0] == 0 && d->obj_w[1] == 0 && d->obj_w[2] == 0) in->d.obj_w[0] = 1;
    int m = n + 1;
    in->dn = m;
    in->dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        in->dist[(int64_t)i * m + j] =
            or_nint_dist(d->a[2 * i], d->a[2 * i + 1], d->a[2 * j], d->a[2 * j + 1]);
    if (d->kind == K_VRPROWS) {   /* the solution: n customers and one marker per row */
      in->nc = n;
      in->d.n = n + d->vehicles;
    }
  } else if (d->kind == K_QAP || d->kind == K_KNAP) {
    if (!d->b) { free(in); return NULL; }
    if (d->kind == K_KNAP) {
      int64_t mv = 0;
      for (int i = 0; i < n; ++i) if (d->b[i] > mv) mv = d->b[i];
      /* reading: penalty weight lambda = max value + 1, so an overweight
       * selection is always worse than dropping an item */
      in->lambda = mv + 1;
    }
  } else if (d->kind == K_COLOR) {
    if (d->ub < d->lb) { free(in); return NULL; }
  } else {
    free(in);
    return NULL;
  }
  if (d->kind == K_TSP || d->kind == K_QAP || d->kind == K_VRPTW) {
    /* the row sums of the heuristic initialisation: TSP distances, QAP flows,
     * VRPTW travel times among the customers */
    in->hkey = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        in->hkey[i] += d->kind == K_TSP ? in->dist[(int64_t)i * n + j]
                       : d->kind == K_QAP ? d->a[(int64_t)i * n + j]
                                          : in->dist[(int64_t)(i + 1) * in->dn + (j + 1)];
  }
  return in;
}

void or_inst_free(or_inst *in) {
  if (!in) return;
  free(in->hkey);
  free(in->dist);
  free(in);
}

/* ------------------------------------------------------------ objectives
 * All minimised, int64, recomputed from the definition. */
static int64_t obj_tsp(const or_inst *in, const int32_t *x) {
  int n = in->d.n;
  int64_t f = 0;
  for (int i = 0; i < n; ++i) f += or_dist(in, x[i], x[(i + 1) % n]);
  return f;
}

static int64_t obj_qap(const or_inst *in, const int32_t *x) {
  int n = in->d.n;
  const int32_t *F = in->d.a, *D = in->d.b;
  int64_t f = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      f += (int64_t)F[(int64_t)i * n + j] * D[(int64_t)x[i] * n + x[j]];
  return f;
}

static int64_t obj_knap(const or_inst *in, const int32_t *x) {
  int n = in->d.n;
  int64_t W = 0, V = 0;
  for (int i = 0; i < n; ++i)
    if (x[i]) { W += in->d.a[i]; V += in->d.b[i]; }
  int64_t over = W - in->d.capacity;
  return -V + in->lambda * (over > 0 ? over : 0);
}

/* reading: giant tour over customers 1..n, split greedily into routes by
 * capacity; wait until ready, lateness penalised 100 per unit, each vehicle
 * beyond the fleet 10000.  Sec. "Multi-Objective Optimization Modes", weighted
 * mode: the three objectives (total distance, number of routes, length of the
 * longest route) enter with the instance's integer weights; the default
 * (1, 0, 0) is the single distance objective. */
/* parts[0..4]: total distance, routes, longest route, total lateness,
 * routes beyond the fleet */
static void vrptw_parts(const or_inst *in, const int32_t *x, int64_t parts[5]) {
  int n = in->d.n;
  const int32_t *dem = in->d.b, *ready = in->d.b + (n + 1), *due = in->d.b + 2 * (n + 1);
  int64_t dist = 0, late = 0, t = 0, load = 0, route_len = 0, longest = 0;
  int routes = 0, prev = 0;
  for (int p = 0; p < n; ++p) {
    int c = x[p] + 1;
    if (routes == 0 || load + dem[c] > in->d.capacity) {
      if (routes > 0) {
        int64_t back = or_dist(in, prev, 0);
        dist += back; t += back; route_len += back;
        if (t > in->d.horizon) late += t - in->d.horizon;
        if (route_len > longest) longest = route_len;
      }
      routes++; load = 0; t = 0; prev = 0; route_len = 0;
    }
    int64_t dd = or_dist(in, prev, c);
    dist += dd; t += dd; route_len += dd;
    if (t < ready[c]) t = ready[c];
    if (t > due[c]) late += t - due[c];
    t += in->d.service_time;
    load += dem[c];
    prev = c;
  }
  if (routes > 0) {
    int64_t back = or_dist(in, prev, 0);
    dist += back; t += back; route_len += back;
    if (t > in->d.horizon) late += t - in->d.horizon;
    if (route_len > longest) longest = route_len;
  }
  int64_t extra = routes - in->d.vehicles;
  parts[0] = dist; parts[1] = routes; parts[2] = longest; parts[3] = late; parts[4] = extra > 0 ? extra : 0;
}

/* Sec. "Solution Structure": a multi-row solution keeps one route per row
 * (Tab. generality runs CVRP and VRPTW in this form).  Entries below nc are
 * customers (entry c is node c + 1), the others row markers; a row is the run
 * of customers before its marker and goes from the depot through them in
 * order and back.  reading: an empty row is no route; lateness as for the
 * giant tour; a row's load above the capacity costs 100 per unit (the row
 * form's penalty, where the giant tour's split keeps every route within the
 * capacity).  parts as vrptw_parts, plus parts[5] = load above capacity. */
static void rows_parts(const or_inst *in, const int32_t *x, int64_t parts[6]) {
  const int N = in->d.n, m = in->nc + 1;
  const int32_t *dem = in->d.b, *ready = in->d.b + m, *due = in->d.b + 2 * m;
  int64_t dist = 0, late = 0, longest = 0, over = 0;
  int routes = 0, start = 0;
  for (int p = 0; p < N; ++p) {
    if (x[p] < in->nc) continue;            /* a customer */
    if (p > start) {                        /* the row of entries start .. p-1 */
      int64_t t = 0, load = 0, len = 0;
      int prev = 0;
      for (int i = start; i < p; ++i) {
        int c = x[i] + 1;
        int64_t dd = or_dist(in, prev, c);
        dist += dd; len += dd; t += dd;
        if (t < ready[c]) t = ready[c];
        if (t > due[c]) late += t - due[c];
        t += in->d.service_time;
        load += dem[c];
        prev = c;
      }
      int64_t back = or_dist(in, prev, 0);
      dist += back; len += back; t += back;
      if (t > in->d.horizon) late += t - in->d.horizon;
      if (len > longest) longest = len;
      if (load > in->d.capacity) over += load - in->d.capacity;
      routes++;
    }
    start = p + 1;
  }
  parts[0] = dist; parts[1] = routes; parts[2] = longest; parts[3] = late; parts[4] = 0; parts[5] = over;
}

/* the parts of either VRPTW form (parts[5]: load above capacity, 0 for the giant tour) */
static void vrp_parts(const or_inst *in, const int32_t *x, int64_t parts[6]) {
  if (in->d.kind == K_VRPROWS) rows_parts(in, x, parts);
  else { vrptw_parts(in, x, parts); parts[5] = 0; }
}

static int64_t obj_vrptw(const or_inst *in, const int32_t *x) {
  int64_t q[6];
  vrp_parts(in, x, q);
  return (int64_t)in->d.obj_w[0] * q[0] + (int64_t)in->d.obj_w[1] * q[1] + (int64_t)in->d.obj_w[2] * q[2] +
         100 * q[3] + 10000 * q[4] + 100 * q[5];
}

/* Sec. "Multi-Objective Optimization Modes", lexicographic mode.  reading:
 * the penalty (lateness, fleet excess and, in the row form, load above capacity,
 * as in the weighted mode) comes
 * first and is compared exactly; then the objectives in the caller's
 * priority order, where two values within the level's tolerance are equal
 * and the next level decides.  v = (penalty, level 1, level 2, level 3),
 * unused levels 0. */
int or_lex_mode(const or_inst *in) {
  return (in->d.kind == K_VRPTW || in->d.kind == K_VRPROWS) && in->d.lex_order[0] != 0;
}

void or_lex_vector(const or_inst *in, const int32_t *x, int64_t v[4]) {
  int64_t q[6];
  vrp_parts(in, x, q);
  v[0] = 100 * q[3] + 10000 * q[4] + 100 * q[5];
  for (int i = 0; i < 3; ++i) {
    int id = in->d.lex_order[i];
    v[1 + i] = id ? q[id - 1] : 0;
  }
}

/* a strictly better than b */
int or_lex_better(const or_inst *in, const int64_t a[4], const int64_t b[4]) {
  if (a[0] != b[0]) return a[0] < b[0];
  for (int i = 0; i < 3 && in->d.lex_order[i]; ++i) {
    int64_t tol = in->d.lex_tol[i];
    if (a[1 + i] + tol < b[1 + i]) return 1;
    if (b[1 + i] + tol < a[1 + i]) return 0;
  }
  return 0;
}

/* reading: where the paper compares two solutions' objectives over a set
 * (the argmin over candidates, the best of a population), the lexicographic
 * mode scans the set in index order and keeps the first element no later
 * element is strictly better than the one kept so far. */
int or_lex_best(const or_inst *in, const or_state *st, int population) {
  int b = 0;
  for (int s = 1; s < population; ++s)
    if (or_lex_better(in, st->best_v + 4 * (size_t)s, st->best_v + 4 * (size_t)b)) b = s;
  return b;
}

static int64_t obj_color(const or_inst *in, const int32_t *x) {
  int64_t f = 0;
  for (int e = 0; e < in->d.n_edges; ++e)
    f += x[in->d.a[2 * e]] == x[in->d.a[2 * e + 1]];
  return f;
}

int64_t or_objective(const or_inst *in, const int32_t *x) {
  switch (in->d.kind) {
    case K_TSP: return obj_tsp(in, x);
    case K_QAP: return obj_qap(in, x);
    case K_KNAP: return obj_knap(in, x);
    case K_VRPTW: case K_VRPROWS: return obj_vrptw(in, x);
    default: return obj_color(in, x);
  }
}

/* ------------------------------------------------------------ operators
 * Tab. "operators": element level swap / insert / reverse (permutation),
 * flip (binary), random_reset (integer); segment level or-opt.
 * Applied to a real array.  Returns the op id that was applied. */
static void reverse_range(int32_t *x, int lo, int hi) {
  while (lo < hi) { int32_t t = x[lo]; x[lo] = x[hi]; x[hi] = t; ++lo; --hi; }
}

static void perm_op(int32_t *x, int n, int op, uint32_t w1, uint32_t w2, uint32_t w3);
static void row_op(const or_inst *in, int32_t *x, int op, uint32_t w1);
static void lns_op(const or_inst *in, int32_t *x, int op, uint32_t w1, uint32_t w2, uint32_t w3);

int or_apply_op(const or_inst *in, int32_t *x, int op, uint32_t w1, uint32_t w2, uint32_t w3) {
  int n = in->d.n;
  /* the row form: the permutation operators act on the entries before the
   * final marker (which stays last), the row operators on whole rows */
  if (in->d.kind == K_VRPROWS) {
    if (op >= OP_ROWSWAP) row_op(in, x, op, w1);
    else perm_op(x, n - 1, op, w1, w2, w3);
    return op;
  }
  if (op >= OP_LNS_SEG && op <= OP_LNS_GUIDED) {
    lns_op(in, x, op, w1, w2, w3);
    return op;
  }
  if (op == OP_FLIP) { x[rmap(w1, n)] ^= 1; return op; }
  if (op == OP_RESET) {
    uint32_t i = rmap(w1, n);
    x[i] = in->d.lb + (int32_t)rmap(w2, (uint32_t)(in->d.ub - in->d.lb + 1));
    return op;
  }
  /* Tab. operators, segment level: seg_flip flips, seg_reset sets to one new
   * value, the L consecutive elements starting at a.  reading: L = 2 +
   * floor(w3 * 6 / 2^32) (2..7), at most n; a = floor(w1 * (n - L + 1) / 2^32); the
   * value as for random_reset */
  if (op == OP_SEGFLIP || op == OP_SEGRESET) {
    uint32_t L = 2 + rmap(w3, 6);
    if (L > (uint32_t)n) L = (uint32_t)n;
    const uint32_t a = rmap(w1, (uint32_t)n - L + 1);
    const int32_t v = in->d.lb + (int32_t)rmap(w2, (uint32_t)(in->d.ub - in->d.lb + 1));
    for (uint32_t p = a; p < a + L; ++p) {
      if (op == OP_SEGFLIP) x[p] ^= 1;
      else x[p] = v;
    }
    return op;
  }
  perm_op(x, n, op, w1, w2, w3);
  return op;
}

/* The permutation operators on x[0 .. n-1]. */
static void perm_op(int32_t *x, int n, int op, uint32_t w1, uint32_t w2, uint32_t w3) {
  if (n < 2) return;                         /* every permutation move is the identity */
  /* Tab. operators, segment level, 3-opt.  reading: the segment exchange, the
   * 3-opt reconnection that keeps every segment's orientation: three distinct
   * cut positions a < b < c of {0..n} (drawn as a uniform triple: w1 over n+1
   * values, w2 over the other n, w3 over the remaining n-1, in increasing
   * order of value), and s[a..b) and s[b..c) trade places. */
  if (op == OP_3OPT) {
    uint32_t c1 = rmap(w1, (uint32_t)n + 1), c2 = rmap(w2, (uint32_t)n), c3 = rmap(w3, (uint32_t)n - 1);
    c2 += (c2 >= c1);
    uint32_t lo = c1 < c2 ? c1 : c2, hi = c1 < c2 ? c2 : c1;
    c3 += (c3 >= lo);
    c3 += (c3 >= hi);
    uint32_t a = lo, b = hi, c = c3;          /* sort the three cuts */
    if (c < a) { uint32_t t = c; c = b; b = a; a = t; }
    else if (c < b) { uint32_t t = c; c = b; b = t; }
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * n);
    int o = 0;
    for (uint32_t p = 0; p < a; ++p) tmp[o++] = x[p];
    for (uint32_t p = b; p < c; ++p) tmp[o++] = x[p];
    for (uint32_t p = a; p < b; ++p) tmp[o++] = x[p];
    for (uint32_t p = c; p < (uint32_t)n; ++p) tmp[o++] = x[p];
    memcpy(x, tmp, sizeof(int32_t) * n);
    free(tmp);
    return;
  }
  if (op == OP_2OPT || op == OP_SWAP) {
    uint32_t i = rmap(w1, n), j = rmap(w2, n - 1);
    j += (j >= i);
    if (op == OP_SWAP) { int32_t t = x[i]; x[i] = x[j]; x[j] = t; }
    else reverse_range(x, i < j ? i : j, i < j ? j : i);   /* reverse = 2-opt */
    return;
  }
  /* insert (segment length 1) and or-opt (length 2 or 3, orientation kept):
   * remove s[i..i+L-1] and put it back so that it starts at index q */
  int L = (op == OP_INSERT) ? 1 : 2 + (int)rmap(w3, 2);
  if (L > n - 1) L = n - 1;
  uint32_t i = rmap(w1, (uint32_t)(n - L + 1));
  uint32_t q = rmap(w2, (uint32_t)(n - L));
  q += (q >= i);
  int32_t seg[3];
  for (int s = 0; s < L; ++s) seg[s] = x[i + s];
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * n);
  int m = 0;
  for (int p = 0; p < n; ++p)
    if (p < (int)i || p >= (int)i + L) tmp[m++] = x[p];   /* the remainder, n-L items */
  int o = 0;
  for (int p = 0; p < n - L + 1; ++p) {
    if (p == (int)q) for (int s = 0; s < L; ++s) x[o++] = seg[s];
    if (p < n - L) x[o++] = tmp[p];
  }
  free(tmp);
  return;
}

/* Tab. "operators", row level: row_swap, row_split and row_merge act on whole
 * rows of a multi-row solution (rows one after another, each closed by its
 * marker; the final entry is a marker).  reading: w1 draws a position p
 * uniformly among the N - 1 entries before the final marker, which names the
 * row that holds it (the row p's entry belongs to, its marker included):
 *   row_swap:  that row and the next one trade places, each with its marker;
 *              nothing when it is the last row;
 *   row_split: when the last row is empty, its marker (entry N - 2) is taken
 *              out and put back at index p, so that the row ends before p's
 *              entry and p's entry opens a new row with the rest of the row;
 *              nothing when the last row holds customers or p = N - 2;
 *   row_merge: the row's marker is taken out and put back just before the
 *              final marker, so that the next row's customers join the row
 *              and the rows after it move up, leaving the last row empty;
 *              nothing when the row is the last one or the next one is the
 *              empty last row.
 * The operators only look at the solution they are applied to (the candidate
 * as the earlier steps left it). */
static void move_entry(int32_t *x, int from, int to) {   /* take x[from] out, put it back at index `to` */
  int32_t v = x[from];
  if (from < to) memmove(x + from, x + from + 1, sizeof(int32_t) * (size_t)(to - from));
  else memmove(x + to + 1, x + to, sizeof(int32_t) * (size_t)(from - to));
  x[to] = v;
}

static void row_op(const or_inst *in, int32_t *x, int op, uint32_t w1) {
  const int N = in->d.n, nc = in->nc;
  const int p = (int)rmap(w1, (uint32_t)(N - 1));
  int e1 = p;                                   /* the marker that closes p's row */
  while (x[e1] < nc) ++e1;
  if (op == OP_ROWSPLIT) {
    if (N >= 2 && x[N - 2] >= nc && p < N - 2) move_entry(x, N - 2, p);
    return;
  }
  if (op == OP_ROWMERGE) {
    if (e1 < N - 2) move_entry(x, e1, N - 2);
    return;
  }
  if (e1 == N - 1) return;                      /* row_swap of the last row */
  int s = p;                                    /* the first entry of p's row */
  while (s > 0 && x[s - 1] < nc) --s;
  int e2 = e1 + 1;                              /* the marker that closes the next row */
  while (x[e2] < nc) ++e2;
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(e2 - s + 1));
  int o = 0;
  for (int i = e1 + 1; i <= e2; ++i) tmp[o++] = x[i];
  for (int i = s; i <= e1; ++i) tmp[o++] = x[i];
  memcpy(x + s, tmp, sizeof(int32_t) * (size_t)o);
  free(tmp);
}

/* Sec. "Built-in Operator Hierarchy": the LNS operators -- segment shuffle,
 * scatter shuffle, guided rebuild -- destroy a part of the solution whose
 * size follows the problem size and rebuild it.  On single-row permutations
 * (ids 5-7).  readings:
 *  - destroyed part L(n) = min(n, 2 + floor(n / 16), 64) entries;
 *  - draws beyond the step's three words: x_i is word i mod 4 of the
 *    Philox4x32-10 block with counter (w1, w2, w3, floor(i / 4)) and key
 *    (0x4C4E5331, 0x4C4E5332), so that a step stays a function of its words;
 *  - segment shuffle: the L entries from a = floor(w1 (n - L + 1) / 2^32)
 *    shuffled by Fisher-Yates: for i = L-1 down to 1 entry i and entry
 *    floor(x_{L-1-i} (i + 1) / 2^32) of the segment trade places;
 *  - scatter shuffle: L distinct positions by Floyd's sampling (for
 *    j = n-L .. n-1 in turn, r = floor(x_{j-n+L} (j + 1) / 2^32) joins the
 *    set, or j when r is already in it), in increasing order; their entries
 *    shuffled as above with the words x_{L + L-1-i};
 *  - guided rebuild: the L entries from a (drawn as for the segment shuffle)
 *    put back in order of their heuristic key (the row sums of the heuristic
 *    initialisation), ascending when the top bit of w2 is 0 and descending
 *    otherwise, ties by entry value ascending. */
int or_lns_len(int n) {
  int L = 2 + n / 16;
  if (L > 64) L = 64;
  return L < n ? L : n;
}

static uint32_t lns_word(uint32_t w1, uint32_t w2, uint32_t w3, int i) {
  const uint32_t ctr[4] = {w1, w2, w3, (uint32_t)(i >> 2)}, key[2] = {0x4C4E5331u, 0x4C4E5332u};
  uint32_t r[4];
  or_philox4x32_10(ctr, key, r);
  return r[i & 3];
}

static void lns_op(const or_inst *in, int32_t *x, int op, uint32_t w1, uint32_t w2, uint32_t w3) {
  const int n = in->d.n, L = or_lns_len(n);
  if (L < 2) return;
  int pos[64];
  if (op == OP_LNS_SCATTER) {
    int cnt = 0;
    for (int j = n - L; j < n; ++j) {
      int r = (int)rmap(lns_word(w1, w2, w3, j - n + L), (uint32_t)(j + 1)), have = 0;
      for (int q = 0; q < cnt; ++q) have |= pos[q] == r;
      pos[cnt++] = have ? j : r;
    }
    for (int i = 1; i < L; ++i) {             /* increasing order */
      int v = pos[i], q = i;
      while (q > 0 && pos[q - 1] > v) { pos[q] = pos[q - 1]; --q; }
      pos[q] = v;
    }
  } else {
    const int a = (int)rmap(w1, (uint32_t)(n - L + 1));
    for (int i = 0; i < L; ++i) pos[i] = a + i;
  }
  if (op == OP_LNS_GUIDED) {
    const int desc = (int)(w2 >> 31);
    int32_t v[64];
    for (int i = 0; i < L; ++i) v[i] = x[pos[i]];
    for (int i = 1; i < L; ++i) {             /* insertion sort by (key, value) */
      int32_t e = v[i];
      int q = i;
      while (q > 0) {
        int64_t kp = in->hkey[v[q - 1]], ke = in->hkey[e];
        if (desc) { kp = -kp; ke = -ke; }
        if (kp > ke || (kp == ke && v[q - 1] > e)) { v[q] = v[q - 1]; --q; }
        else break;
      }
      v[q] = e;
    }
    for (int i = 0; i < L; ++i) x[pos[i]] = v[i];
    return;
  }
  const int base = op == OP_LNS_SCATTER ? L : 0;
  for (int i = L - 1; i >= 1; --i) {
    int j = (int)rmap(lns_word(w1, w2, w3, base + L - 1 - i), (uint32_t)(i + 1));
    int32_t t = x[pos[i]]; x[pos[i]] = x[pos[j]]; x[pos[j]] = t;
  }
}

/* ------------------------------------------------------------ encodings */
static uint32_t encoding_ops(int kind) {
  if (kind == K_KNAP) return (1u << OP_FLIP) | (1u << OP_SEGFLIP);
  if (kind == K_COLOR) return (1u << OP_RESET) | (1u << OP_SEGRESET);
  if (kind == K_VRPROWS)
    return (1u << OP_2OPT) | (1u << OP_SWAP) | (1u << OP_INSERT) | (1u << OP_OROPT) | (1u << OP_3OPT) |
           (1u << OP_ROWSWAP) | (1u << OP_ROWSPLIT) | (1u << OP_ROWMERGE);
  return (1u << OP_2OPT) | (1u << OP_SWAP) | (1u << OP_INSERT) | (1u << OP_OROPT) | (1u << OP_3OPT);
}

/* reading: the LNS operators are taken when op_mask names them; the default
 * set of a single-row permutation is its element and segment operators */
static int lns_kind(int kind) { return kind == K_TSP || kind == K_QAP || kind == K_VRPTW; }

uint32_t or_effective_mask(const or_inst *in, uint32_t op_mask) {
  uint32_t e = encoding_ops(in->d.kind);
  if (lns_kind(in->d.kind) && op_mask) e |= (1u << OP_LNS_SEG) | (1u << OP_LNS_SCATTER) | (1u << OP_LNS_GUIDED);
  return op_mask ? (op_mask & e) : e;
}

/* Tab. "weight_preset", LNS cap: the largest weight the EMA update gives an
 * LNS operator, 0.02 / 0.01 / 0.005 (Q16, rounded) by scale; the lower bound
 * of its clamp is the smaller of the floor and the cap.  0: no LNS. */
uint32_t or_lns_cap(const or_inst *in) {
  if (!lns_kind(in->d.kind)) return 0;
  const int n = in->d.n;
  return n <= 100 ? 1311u : (n <= 250 ? 655u : 328u);
}

/* the per-sequence caps of a solve: the caller's, else the LNS cap for the
 * LNS operators and 1.0 for the others */
static void op_caps(const or_inst *in, const or_params *p, uint32_t caps[OR_MAX_OPS]) {
  const uint32_t lc = or_lns_cap(in);
  for (int i = 0; i < OR_MAX_OPS; ++i)
    caps[i] = p->cap_w[i] ? p->cap_w[i] : ((lc && i >= OP_LNS_SEG && i <= OP_LNS_GUIDED) ? lc : 65536u);
}

static int enabled_list(uint32_t mask, int *ids) {
  int c = 0;
  for (int i = 0; i < OR_MAX_OPS; ++i) if (mask & (1u << i)) ids[c++] = i;
  return c;
}

/* Sec. "Problem-Profile-Driven Prior Strategy", Tab. "weight_preset":
 * O(1) operators start at 1.0; or-opt at 0.8 / 0.7 / 0.3 and 3-opt at
 * 0.50 / 0.30 / 0.05 for n <= 100, <= 250, > 250 (Q16, rounded; n is the
 * solution's length, customers and markers in the row form); LNS at
 * 0.006 / 0.004 / 0.001; reading: the row operators, which the table does
 * not list, start at 1.0; a nonzero
 * init_w[i] replaces the preset of operator i; then the weights are
 * normalised (Q16). */
void or_initial_weights(const or_inst *in, uint32_t op_mask, const uint32_t *init_w, uint32_t w[OR_MAX_OPS]) {
  uint32_t m = or_effective_mask(in, op_mask);
  int n = in->d.n;
  uint64_t raw[OR_MAX_OPS] = {0}, s = 0;
  for (int i = 0; i < OR_MAX_OPS; ++i) {
    if (!(m & (1u << i))) continue;
    raw[i] = 65536;
    if (i == OP_OROPT) raw[i] = n <= 100 ? 52429 : (n <= 250 ? 45875 : 19661);
    if (i == OP_3OPT) raw[i] = n <= 100 ? 32768 : (n <= 250 ? 19661 : 3277);
    if (lns_kind(in->d.kind) && i >= OP_LNS_SEG && i <= OP_LNS_GUIDED)
      raw[i] = n <= 100 ? 393 : (n <= 250 ? 262 : 66);
    if (init_w && init_w[i]) raw[i] = init_w[i];
    s += raw[i];
  }
  for (int i = 0; i < OR_MAX_OPS; ++i) {
    if (!(m & (1u << i))) { w[i] = 0; continue; }
    uint64_t v = (raw[i] << 16) / s;
    w[i] = (uint32_t)(v < 1 ? 1 : v);
  }
}

/* ------------------------------------------------------------ acceptance
 * Alg. 1: accept if delta < 0 or rand() < e^{-delta/T}.  reading: delta = 0
 * always accepted (e^0 = 1); e^{-x} taken from two integer tables on
 * z = floor(delta * 2^24 / T_q16) = floor(256 * delta / T), the quotient
 * taken exactly for every delta < 2^63 and T_q16 < 2^64 (128-bit numerator). */
uint32_t or_accept_threshold(uint64_t delta, uint64_t t_q16, int *reject) {
  *reject = 0;
  if (t_q16 == 0) { *reject = 1; return 0; }
  unsigned __int128 z = ((unsigned __int128)delta << 24) / t_q16;
  if (z >= 4096) { *reject = 1; return 0; }
  return (uint32_t)(((uint64_t)OR_EXP_HI[z >> 8] * OR_EXP_LO[z & 255]) >> 31);
}

/* Alg. 1: T <- alpha T, with T in Q16 and alpha in Q32: floor(T * alpha / 2^32). */
uint64_t or_cool(uint64_t t, uint32_t alpha) {
  uint64_t hi = t >> 32, lo = t & 0xFFFFFFFFu;
  return hi * alpha + ((lo * alpha) >> 32);
}

/* ------------------------------------------------------------ AOS update
 * Eq. ema: w <- a w + (1-a)(v/(u+eps) + w_floor); clamp to [w_floor, 1];
 * normalise; Alg. 2 also updates the K-step weights the same way and resets
 * them to (0.8, 0.15, 0.05) after stagnation. */
/* Eq. ema, then the clamp to [w_floor, min(w_cap, cap_i)] with w_cap = 1.0
 * and cap_i the per-sequence cap of operator i (Sec. "Two-Level Weight
 * Structure"); reading: when cap_i is below the floor the clamp is [cap_i,
 * cap_i].  caps: per operator id, NULL for the K-step group. */
static void ema_group(const or_params *p, uint32_t *w, const uint64_t *u, const uint64_t *v,
                      const int *ids, int cnt, const uint32_t *caps) {
  uint64_t A = p->aos_alpha_q16, FL = p->w_floor_q16, s = 0;
  for (int c = 0; c < cnt; ++c) {
    int i = ids[c];
    uint64_t r = (v[i] << 16) / (u[i] + 1);
    uint64_t nw = (A * w[i] + (65536 - A) * (r + FL)) >> 16;
    const uint64_t hi = caps ? caps[i] : 65536, lo = hi < FL ? hi : FL;
    if (nw < lo) nw = lo;
    if (nw > hi) nw = hi;
    w[i] = (uint32_t)nw;
    s += nw;
  }
  for (int c = 0; c < cnt; ++c) {
    int i = ids[c];
    uint64_t nw = ((uint64_t)w[i] << 16) / s;
    w[i] = (uint32_t)(nw < 1 ? 1 : nw);
  }
}

static const uint32_t WK_DEFAULT[3] = {52429, 9830, 3277};

/* the update with the epoch's improvement of the instance best given */
static void aos_update_flag(const or_params *p, uint32_t mask, const uint32_t *caps, or_state *st, int improved) {
  int ids[OR_MAX_OPS];
  int cnt = enabled_list(mask, ids);
  ema_group(p, st->w_op, st->u_op, st->v_op, ids, cnt, caps);
  int kid[3] = {0, 1, 2};
  ema_group(p, st->w_k, st->u_k, st->v_k, kid, 3, NULL);
  /* reading: "consecutive no-improvement" counted in epochs of the instance best */
  if (improved) st->stag = 0;
  else st->stag++;
  if (st->stag >= p->stagnation_epochs) {
    memcpy(st->w_k, WK_DEFAULT, sizeof(WK_DEFAULT));
    st->stag = 0;
  }
  memset(st->u_op, 0, sizeof(st->u_op));
  memset(st->v_op, 0, sizeof(st->v_op));
  memset(st->u_k, 0, sizeof(st->u_k));
  memset(st->v_k, 0, sizeof(st->v_k));
}

void or_aos_update(const or_inst *in, const or_params *p, uint32_t mask, or_state *st, int64_t inst_best_now) {
  int improved = inst_best_now < st->epoch_ref;
  st->epoch_ref = inst_best_now;
  uint32_t caps[OR_MAX_OPS];
  op_caps(in, p, caps);
  aos_update_flag(p, mask, caps, st, improved);
}

/* Per-solution scope (aos_scope = 1).  reading: Alg. 2 pools the statistics
 * of all blocks of the instance; the per-solution mode gives each solution
 * (one workgroup) its own operator and K-step weights, updated from its own
 * candidates' counts with the same Eq. ema arithmetic, and its own
 * stagnation counter on its own best objective.  The instance-level weights
 * and epoch counts are then not used and stay as initialised. */
static void sol_aos_update(const or_params *p, uint32_t mask, const uint32_t *caps, or_sol_aos *a, int64_t best_now) {
  int ids[OR_MAX_OPS];
  int cnt = enabled_list(mask, ids);
  uint64_t u[OR_MAX_OPS], v[OR_MAX_OPS], uk[3], vk[3];
  for (int i = 0; i < OR_MAX_OPS; ++i) { u[i] = a->u_op[i]; v[i] = a->v_op[i]; }
  for (int i = 0; i < 3; ++i) { uk[i] = a->u_k[i]; vk[i] = a->v_k[i]; }
  ema_group(p, a->w_op, u, v, ids, cnt, caps);
  int kid[3] = {0, 1, 2};
  ema_group(p, a->w_k, uk, vk, kid, 3, NULL);
  if (best_now < a->epoch_ref) a->stag = 0;
  else a->stag++;
  a->epoch_ref = best_now;
  if (a->stag >= p->stagnation_epochs) {
    memcpy(a->w_k, WK_DEFAULT, sizeof(WK_DEFAULT));
    a->stag = 0;
  }
  memset(a->u_op, 0, sizeof(a->u_op));
  memset(a->v_op, 0, sizeof(a->v_op));
  memset(a->u_k, 0, sizeof(a->u_k));
  memset(a->v_k, 0, sizeof(a->v_k));
}

/* ------------------------------------------------------------ islands
 * Sec. "Island Model and Elite Injection".  Readings: island i holds the
 * consecutive solutions [i S, (i+1) S), S = P / I.  At the end of epoch e
 * (after the AOS update) with e % migrate_epochs == 0, elites -- best-so-far
 * solutions -- replace the worst current solutions of the receiving islands;
 * every source and every target is chosen on the state before the first copy:
 *   ring:   the best of island i replaces the worst of island (i + 1) mod I;
 *   top-N:  the N best of the population replace the N worst of every island
 *           (the k-th best the k-th worst);
 *   hybrid: ring at odd-numbered migrations (e / migrate_epochs odd), top-N
 *           at even ones.
 * Elite injection (e % elite_epochs == 0, after the migration): the best of
 * the population replaces its worst.  best = smallest (best_f, index); worst
 * = largest (cur_f, index).  A replaced solution takes the elite's vector and
 * objective as its current solution, and as its own best when it improves it.
 * reading, lexicographic mode: the same rules with "smaller" replaced by the
 * mode's relation -- best: a later solution replaces the one kept when
 * strictly better; worst: when the one kept is not strictly better than it
 * (as ties go to the later index in the scalar rule); an elite improves a
 * solution when strictly better than its best vector. */
static int mig_better(const or_inst *in, const int64_t *fa, const int64_t *va, const int64_t *fb,
                      const int64_t *vb) {
  return or_lex_mode(in) ? or_lex_better(in, va, vb) : *fa < *fb;
}

static void mig_put(const or_inst *in, or_state *st, int n, int tgt, const int32_t *vec, int64_t f,
                    const int64_t v[4]) {
  memcpy(st->cur + (size_t)tgt * n, vec, sizeof(int32_t) * n);
  st->cur_f[tgt] = f;
  if (or_lex_mode(in)) memcpy(st->cur_v + 4 * (size_t)tgt, v, 4 * sizeof(int64_t));
  if (mig_better(in, &f, v, &st->best_f[tgt], st->best_v + 4 * (size_t)tgt)) {
    st->best_f[tgt] = f;
    memcpy(st->best + (size_t)tgt * n, vec, sizeof(int32_t) * n);
    if (or_lex_mode(in)) memcpy(st->best_v + 4 * (size_t)tgt, v, 4 * sizeof(int64_t));
  }
}

static int in_list(const int *l, int cnt, int v) {
  for (int i = 0; i < cnt; ++i) if (l[i] == v) return 1;
  return 0;
}

/* the cnt best of [lo, hi) by (best_f, index), in that order */
static void best_of_range(const or_inst *in, const or_state *st, int lo, int hi, int cnt, int *out) {
  for (int k = 0; k < cnt; ++k) {
    int b = -1;
    for (int s = lo; s < hi; ++s)
      if (!in_list(out, k, s) &&
          (b < 0 || mig_better(in, &st->best_f[s], st->best_v + 4 * (size_t)s, &st->best_f[b],
                               st->best_v + 4 * (size_t)b)))
        b = s;
    out[k] = b;
  }
}

/* the cnt worst of [lo, hi) by (cur_f, index), worst first */
static void worst_of_range(const or_inst *in, const or_state *st, int lo, int hi, int cnt, int *out) {
  for (int k = 0; k < cnt; ++k) {
    int w = -1;
    for (int s = lo; s < hi; ++s)
      if (!in_list(out, k, s) &&
          (w < 0 || !mig_better(in, &st->cur_f[s], st->cur_v + 4 * (size_t)s, &st->cur_f[w],
                                st->cur_v + 4 * (size_t)w)))
        w = s;
    out[k] = w;
  }
}

void or_migrate(const or_inst *in, const or_params *p, int n, or_state *st, uint32_t e) {
  const int P = (int)p->population;
  const int I = p->islands > 1 ? (int)p->islands : 1, S = P / I;
  if (p->migrate_epochs && e % p->migrate_epochs == 0 && I >= 2) {
    int mode = (int)p->migrate_mode;
    if (mode == 2) mode = ((e / p->migrate_epochs) & 1) ? 0 : 1;
    const int N = mode == 0 ? 1 : (p->migrate_n ? (int)p->migrate_n : 1);
    const int n_src = mode == 0 ? I : N;
    int *src = (int *)malloc(sizeof(int) * n_src), *tgt = (int *)malloc(sizeof(int) * I * N);
    int32_t *vec = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_src * n);
    int64_t *f = (int64_t *)malloc(sizeof(int64_t) * n_src);
    int64_t *v = (int64_t *)calloc((size_t)n_src * 4, sizeof(int64_t));
    if (mode == 0) {
      for (int i = 0; i < I; ++i) {
        best_of_range(in, st, i * S, (i + 1) * S, 1, &src[i]);
        const int j = (i + 1) % I;
        worst_of_range(in, st, j * S, (j + 1) * S, 1, &tgt[i]);
      }
    } else {
      best_of_range(in, st, 0, P, N, src);
      for (int i = 0; i < I; ++i) worst_of_range(in, st, i * S, (i + 1) * S, N, &tgt[i * N]);
    }
    for (int k = 0; k < n_src; ++k) {   /* sources read before any copy */
      memcpy(vec + (size_t)k * n, st->best + (size_t)src[k] * n, sizeof(int32_t) * n);
      f[k] = st->best_f[src[k]];
      if (or_lex_mode(in)) memcpy(v + 4 * (size_t)k, st->best_v + 4 * (size_t)src[k], 4 * sizeof(int64_t));
    }
    if (mode == 0)
      for (int i = 0; i < I; ++i) mig_put(in, st, n, tgt[i], vec + (size_t)i * n, f[i], v + 4 * (size_t)i);
    else
      for (int i = 0; i < I; ++i)
        for (int k = 0; k < N; ++k)
          mig_put(in, st, n, tgt[i * N + k], vec + (size_t)k * n, f[k], v + 4 * (size_t)k);
    free(src); free(tgt); free(vec); free(f); free(v);
  }
  if (p->elite_epochs && e % p->elite_epochs == 0) {
    int b, w;
    best_of_range(in, st, 0, P, 1, &b);
    worst_of_range(in, st, 0, P, 1, &w);
    if (w != b) {
      int64_t vb[4] = {0, 0, 0, 0};
      if (or_lex_mode(in)) memcpy(vb, st->best_v + 4 * (size_t)b, sizeof vb);
      mig_put(in, st, n, w, st->best + (size_t)b * n, st->best_f[b], vb);
    }
  }
}

/* ------------------------------------------------------------ init
 * Sec. "Attribute-Agnostic Heuristic Initialization": row sums and column
 * sums of every n x n data matrix, sorted ascending and descending, give four
 * permutations per matrix.  reading: ties keep the smaller index first. */
typedef struct { int64_t k; int32_t i; } kv;
static int kv_cmp(const void *a, const void *b) {
  const kv *x = (const kv *)a, *y = (const kv *)b;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  return x->i < y->i ? -1 : (x->i > y->i);
}

static int sum_perms(const int32_t *M, int n, int stride, int32_t *out) {
  kv *t = (kv *)malloc(sizeof(kv) * n);
  for (int rc = 0; rc < 2; ++rc) {          /* rows, then columns */
    for (int dir = 0; dir < 2; ++dir) {     /* ascending, then descending */
      for (int i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int j = 0; j < n; ++j)
          s += rc == 0 ? M[(int64_t)i * stride + j] : M[(int64_t)j * stride + i];
        t[i].k = dir == 0 ? s : -s;
        t[i].i = i;
      }
      qsort(t, n, sizeof(kv), kv_cmp);
      for (int i = 0; i < n; ++i) out[i] = t[i].i;
      out += n;
    }
  }
  free(t);
  return 4;
}

/* Sec. "Partition Encoding Heuristic Initialization": customers grouped by
 * place, each route ordered by time window.  reading: a sweep around the
 * depot.  Customers in order of polar angle about the depot, counter-clockwise
 * from the positive x axis (compared exactly: the half-plane dy > 0 or
 * (dy = 0, dx >= 0) first, then the sign of the cross product; ties by
 * squared distance to the depot, then index), fill the rows in turn: a row is
 * closed when the next customer's demand would take its load above the
 * capacity, and the last row takes every customer left.  Each row is then
 * ordered by due time, ties by ready time, then index; rows left over stay
 * empty.  Row r is closed by marker nc + r. */
static int sweep_half(int64_t dx, int64_t dy) { return (dy < 0 || (dy == 0 && dx < 0)) ? 1 : 0; }
static int sweep_cmp(const or_inst *in, int a, int b) {   /* nodes 1..nc */
  const int32_t *xy = in->d.a;
  int64_t ax = xy[2 * a] - xy[0], ay = xy[2 * a + 1] - xy[1];
  int64_t bx = xy[2 * b] - xy[0], by = xy[2 * b + 1] - xy[1];
  int ha = sweep_half(ax, ay), hb = sweep_half(bx, by);
  if (ha != hb) return ha - hb;
  int64_t cr = ax * by - ay * bx;
  if (cr != 0) return cr > 0 ? -1 : 1;
  int64_t da = ax * ax + ay * ay, db = bx * bx + by * by;
  if (da != db) return da < db ? -1 : 1;
  return a < b ? -1 : (a > b);
}
static int window_cmp(const or_inst *in, int a, int b) {
  const int m = in->nc + 1;
  const int32_t *ready = in->d.b + m, *due = in->d.b + 2 * m;
  if (due[a] != due[b]) return due[a] < due[b] ? -1 : 1;
  if (ready[a] != ready[b]) return ready[a] < ready[b] ? -1 : 1;
  return a < b ? -1 : (a > b);
}
/* insertion sort of v[0..cnt-1] by cmp */
static void sort_nodes(const or_inst *in, int32_t *v, int cnt, int (*cmp)(const or_inst *, int, int)) {
  for (int i = 1; i < cnt; ++i) {
    int32_t x = v[i];
    int j = i;
    while (j > 0 && cmp(in, v[j - 1], x) > 0) { v[j] = v[j - 1]; --j; }
    v[j] = x;
  }
}

static int sweep_rows(const or_inst *in, int32_t *out) {
  const int nc = in->nc, R = in->d.vehicles;
  int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * nc), *row = (int32_t *)malloc(sizeof(int32_t) * (nc + 1));
  for (int i = 0; i < nc; ++i) ord[i] = i + 1;
  sort_nodes(in, ord, nc, sweep_cmp);
  int r = 0;
  int64_t load = 0;
  for (int i = 0; i < nc; ++i) {
    int c = ord[i];
    if (load + in->d.b[c] > in->d.capacity && r < R - 1) { ++r; load = 0; }
    row[c] = r;
    load += in->d.b[c];
  }
  int o = 0;
  for (int rr = 0; rr < R; ++rr) {
    int cnt = 0;
    for (int i = 0; i < nc; ++i) if (row[ord[i]] == rr) out[o + cnt++] = ord[i];
    sort_nodes(in, out + o, cnt, window_cmp);
    for (int i = 0; i < cnt; ++i) out[o + i] -= 1;   /* node c is entry c - 1 */
    o += cnt;
    out[o++] = nc + rr;
  }
  free(ord);
  free(row);
  return 1;
}

int or_heuristic_perms(const or_inst *in, int32_t *out, int cap) {
  int n = in->d.n, c = 0;
  if (in->d.kind == K_TSP) {
    if (cap >= 4) c += sum_perms(in->dist, n, n, out);
  } else if (in->d.kind == K_QAP) {
    if (cap >= 8) {
      c += sum_perms(in->d.a, n, n, out);
      c += sum_perms(in->d.b, n, n, out + (size_t)4 * n);
    }
  } else if (in->d.kind == K_VRPTW) {
    /* the customer block of the travel-time matrix */
    if (cap >= 4) c += sum_perms(in->dist + in->dn + 1, n, in->dn, out);
  } else if (in->d.kind == K_VRPROWS) {
    if (cap >= 1) c += sweep_rows(in, out);
  }
  return c;
}

/* A random member of the pool at index q: draw i is word (i mod 4) of the
 * block with counter (0xFFFFFFFF, q, i / 4, instance key).  Permutations by
 * Fisher-Yates from the identity (i = n-1 .. 1 swaps x[i] with x[j], j uniform
 * in [0, i]; in the row form over the first n-1 entries, i = n-2 .. 1); bits from the top bit of the draw; integers uniform in [lb, ub]. */
void or_random_solution(const or_inst *in, const or_params *p, uint32_t q, int32_t *x) {
  int n = in->d.n;
  uint32_t key = in->d.key, r[4];
  if (in->d.kind == K_KNAP || in->d.kind == K_COLOR) {
    for (int i = 0; i < n; ++i) {
      draw(p, 0xFFFFFFFFu, q, (uint32_t)(i >> 2), key, r);
      uint32_t w = r[i & 3];
      x[i] = in->d.kind == K_KNAP ? (int32_t)(w >> 31)
                                  : in->d.lb + (int32_t)rmap(w, (uint32_t)(in->d.ub - in->d.lb + 1));
    }
  } else {
    /* the row form shuffles the entries before the final marker, which stays last */
    const int m = in->d.kind == K_VRPROWS ? n - 1 : n;
    for (int i = 0; i < n; ++i) x[i] = i;
    for (int i = m - 1; i >= 1; --i) {
      draw(p, 0xFFFFFFFFu, q, (uint32_t)(i >> 2), key, r);
      uint32_t j = rmap(r[i & 3], (uint32_t)(i + 1));
      int32_t t = x[i]; x[i] = x[j]; x[j] = t;
    }
  }
}

/* pool order: by f, or in the lexicographic mode by the objective vector
 * level by level (no tolerances: a total order); ties by pool index */
typedef struct { int64_t f, v[4]; int32_t q, lex; } fq;
static int fq_cmp(const void *a, const void *b) {
  const fq *x = (const fq *)a, *y = (const fq *)b;
  if (x->lex) {
    for (int i = 0; i < 4; ++i)
      if (x->v[i] != y->v[i]) return x->v[i] < y->v[i] ? -1 : 1;
  } else if (x->f != y->f) {
    return x->f < y->f ? -1 : 1;
  }
  return x->q < y->q ? -1 : (x->q > y->q);
}

/* Sec. "Oversample Initialization": K*P candidates, evaluated, best P kept.
 * reading: heuristic solutions take the first pool slots, the rest are
 * random; ties in f keep the lower pool index. */
int or_init(const or_inst *in, const or_params *p, or_state *st) {
  int n = in->d.n, P = p->population;
  /* reading: the lexicographic mode runs under instance-level weights; the
   * per-solution scope tracks each solution's improvement by a scalar and is
   * not combined with it */
  if (or_lex_mode(in) && p->aos_scope == 1) return -1;
  int Q = p->oversample_k * P;
  int32_t *pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)Q * n);
  int32_t *heur = (int32_t *)malloc(sizeof(int32_t) * (size_t)8 * n);
  int H = or_heuristic_perms(in, heur, 8);
  if (H > Q) H = Q;
  for (int q = 0; q < Q; ++q) {
    int32_t *x = pool + (size_t)q * n;
    if (q < H) memcpy(x, heur + (size_t)q * n, sizeof(int32_t) * n);
    else or_random_solution(in, p, (uint32_t)q, x);
  }
  fq *ord = (fq *)malloc(sizeof(fq) * Q);
  const int lex = or_lex_mode(in);
  for (int q = 0; q < Q; ++q) {
    memset(&ord[q], 0, sizeof(fq));
    ord[q].q = q;
    ord[q].lex = lex;
    if (lex) {   /* reading: the reported scalar of the lexicographic mode is penalty + level 1 */
      or_lex_vector(in, pool + (size_t)q * n, ord[q].v);
      ord[q].f = ord[q].v[0] + ord[q].v[1];
    } else {
      ord[q].f = or_objective(in, pool + (size_t)q * n);
    }
  }
  qsort(ord, Q, sizeof(fq), fq_cmp);
  for (int s = 0; s < P; ++s) {
    memcpy(st->cur + (size_t)s * n, pool + (size_t)ord[s].q * n, sizeof(int32_t) * n);
    memcpy(st->best + (size_t)s * n, pool + (size_t)ord[s].q * n, sizeof(int32_t) * n);
    st->cur_f[s] = st->best_f[s] = ord[s].f;
    if (lex) {
      memcpy(st->cur_v + 4 * (size_t)s, ord[s].v, 4 * sizeof(int64_t));
      memcpy(st->best_v + 4 * (size_t)s, ord[s].v, 4 * sizeof(int64_t));
    }
  }
  if (lex) memcpy(st->ref_v, ord[0].v, 4 * sizeof(int64_t));
  st->g = 0;
  st->stag = 0;
  st->epoch_ref = ord[0].f;
  if (p->t0_q16) st->T_q16 = p->t0_q16;
  else {  /* reading: T0 = a quarter of the mean per-element cost of the best start */
    uint64_t a = (uint64_t)(ord[0].f < 0 ? -ord[0].f : ord[0].f);
    st->T_q16 = ((a << 16) / (uint64_t)n) >> 2;
  }
  or_initial_weights(in, p->op_mask, p->init_w, st->w_op);
  memcpy(st->w_k, WK_DEFAULT, sizeof(WK_DEFAULT));
  memset(st->u_op, 0, sizeof(st->u_op));
  memset(st->v_op, 0, sizeof(st->v_op));
  memset(st->u_k, 0, sizeof(st->u_k));
  memset(st->v_k, 0, sizeof(st->v_k));
  memset(st->tot_u_op, 0, sizeof(st->tot_u_op));
  memset(st->tot_v_op, 0, sizeof(st->tot_v_op));
  memset(st->tot_u_k, 0, sizeof(st->tot_u_k));
  memset(st->tot_v_k, 0, sizeof(st->tot_v_k));
  st->accepted = 0;
  if (p->aos_scope == 1) {   /* every solution starts from the same weights and its own objective */
    for (int s = 0; s < P; ++s) {
      or_sol_aos *a = &st->saos[s];
      memset(a, 0, sizeof(*a));
      memcpy(a->w_op, st->w_op, sizeof(a->w_op));
      memcpy(a->w_k, WK_DEFAULT, sizeof(a->w_k));
      a->epoch_ref = st->best_f[s];
    }
  }
  free(ord);
  free(heur);
  free(pool);
  return 0;
}

/* ------------------------------------------------------------ generations
 * Alg. 1 for every solution of the population, then cooling; after every
 * epoch of E generations the AOS update of Alg. 2.  reading: the RNG counter
 * of candidate t, operator slot m, is (g, solution, 4t + m, instance key);
 * the acceptance draw uses (g, solution, 0xFFFFFFFF, instance key). */

/* AOS counts one generation of one solution adds (uses u and improvements v
 * per operator and per k), and its accepted moves */
typedef struct {
  uint64_t u_op[OR_MAX_OPS], v_op[OR_MAX_OPS], u_k[3], v_k[3], acc;
} or_counts;

static void credit(or_counts *c, const int *ops, int k, int improved) {
  for (int m = 0; m < k; ++m) { c->u_op[ops[m]]++; if (improved) c->v_op[ops[m]]++; }
  c->u_k[k - 1]++;
  if (improved) c->v_k[k - 1]++;
}

/* The difference a worse winner w makes against the current c in the
 * lexicographic mode, for the acceptance test: the penalty difference when
 * the penalties differ, else the difference at the first level where c is
 * better than w by more than the tolerance. */
static int64_t lex_delta(const or_inst *in, const int64_t w[4], const int64_t c[4]) {
  if (w[0] != c[0]) return w[0] - c[0];
  for (int i = 0; i < 3 && in->d.lex_order[i]; ++i)
    if (c[1 + i] + in->d.lex_tol[i] < w[1 + i]) return w[1 + i] - c[1 + i];
  return 0;
}

/* Alg. 1 body in the lexicographic mode: the candidates' objective vectors
 * are compared with or_lex_better (argmin: ordered scan, ties to the lower
 * t); a winner that the current solution does not beat is accepted, a worse
 * one with the exponential test on lex_delta; a candidate improves when it is
 * strictly better than the current solution. */
static void generation_lex(const or_inst *in, const or_params *p, or_state *st, int sol, uint32_t g, uint64_t T,
                           const int *ids, int nids, int32_t *tmp, int32_t *cand, or_counts *c) {
  int n = in->d.n, C = p->candidates;
  uint32_t key = in->d.key;
  int32_t *x = st->cur + (size_t)sol * n;
  int64_t *cv = st->cur_v + 4 * (size_t)sol, *bvs = st->best_v + 4 * (size_t)sol;
  uint32_t wl[OR_MAX_OPS];
  for (int i = 0; i < nids; ++i) wl[i] = st->w_op[ids[i]];
  int64_t bv[4] = {0, 0, 0, 0}, v[4];
  int best_t = -1, best_k = 0, best_ops[3] = {0, 0, 0};
  for (int t = 0; t < C; ++t) {
    memcpy(tmp, x, sizeof(int32_t) * n);
    uint32_t r[4];
    draw(p, g, (uint32_t)sol, (uint32_t)t << 2, key, r);
    int k = 1 + or_wpick(r[0] >> 16, st->w_k, 3);
    int ops[3];
    for (int m = 0; m < k; ++m) {
      if (m > 0) draw(p, g, (uint32_t)sol, ((uint32_t)t << 2) | (uint32_t)m, key, r);
      ops[m] = ids[or_wpick(r[0] & 0xFFFFu, wl, nids)];
      or_apply_op(in, tmp, ops[m], r[1], r[2], r[3]);
    }
    or_lex_vector(in, tmp, v);
    if (p->credit == 0) credit(c, ops, k, or_lex_better(in, v, cv));
    if (best_t < 0 || or_lex_better(in, v, bv)) {
      memcpy(bv, v, sizeof(bv)); best_t = t; best_k = k;
      memcpy(best_ops, ops, sizeof(ops));
      memcpy(cand, tmp, sizeof(int32_t) * n);
    }
  }
  int acc = 0;
  if (!or_lex_better(in, cv, bv)) acc = 1;
  else {
    int rej;
    uint32_t thr = or_accept_threshold((uint64_t)lex_delta(in, bv, cv), T, &rej);
    if (!rej) {
      uint32_t r[4];
      draw(p, g, (uint32_t)sol, 0xFFFFFFFFu, key, r);
      acc = (r[0] >> 1) < thr;
    }
  }
  if (acc) {
    if (p->credit == 1) credit(c, best_ops, best_k, or_lex_better(in, bv, cv));
    memcpy(x, cand, sizeof(int32_t) * n);
    memcpy(cv, bv, sizeof(bv));
    st->cur_f[sol] = bv[0] + bv[1];
    c->acc++;
    if (or_lex_better(in, cv, bvs)) {
      memcpy(bvs, cv, sizeof(bv));
      st->best_f[sol] = st->cur_f[sol];
      memcpy(st->best + (size_t)sol * n, x, sizeof(int32_t) * n);
    }
  }
}

/* One generation of solution `sol` at generation g and temperature T (Alg. 1
 * body); the credited counts are added to *c.  tmp and cand hold n entries. */
static void generation(const or_inst *in, const or_params *p, or_state *st, int sol, uint32_t g, uint64_t T,
                       const int *ids, int nids, int32_t *tmp, int32_t *cand, or_counts *c) {
  if (or_lex_mode(in)) {
    generation_lex(in, p, st, sol, g, T, ids, nids, tmp, cand, c);
    return;
  }
  int n = in->d.n, C = p->candidates;
  uint32_t key = in->d.key;
  int32_t *x = st->cur + (size_t)sol * n;
  const uint32_t *w_op = p->aos_scope == 1 ? st->saos[sol].w_op : st->w_op;   /* R.w */
  const uint32_t *w_k = p->aos_scope == 1 ? st->saos[sol].w_k : st->w_k;      /* w_K */
  uint32_t wl[OR_MAX_OPS];
  for (int i = 0; i < nids; ++i) wl[i] = w_op[ids[i]];
  int64_t best_d = 0;
  int best_t = -1, best_k = 0, best_ops[3] = {0, 0, 0};
  for (int t = 0; t < C; ++t) {
    memcpy(tmp, x, sizeof(int32_t) * n);           /* s_t <- copy(s) */
    uint32_t r[4];
    draw(p, g, (uint32_t)sol, (uint32_t)t << 2, key, r);
    int k = 1 + or_wpick(r[0] >> 16, w_k, 3);      /* k_t from w_K */
    int ops[3];
    for (int m = 0; m < k; ++m) {
      if (m > 0) draw(p, g, (uint32_t)sol, ((uint32_t)t << 2) | (uint32_t)m, key, r);
      ops[m] = ids[or_wpick(r[0] & 0xFFFFu, wl, nids)];  /* sigma_i from R.w */
      or_apply_op(in, tmp, ops[m], r[1], r[2], r[3]);
    }
    int64_t d = or_objective(in, tmp) - st->cur_f[sol];
    if (p->credit == 0) credit(c, ops, k, d < 0);   /* reading: every candidate credits its operators */
    if (best_t < 0 || d < best_d) {   /* argmin; ties keep the lowest t */
      best_d = d; best_t = t; best_k = k;
      memcpy(best_ops, ops, sizeof(ops));
      memcpy(cand, tmp, sizeof(int32_t) * n);
    }
  }
  int acc = 0;
  if (best_d <= 0) acc = 1;
  else {
    int rej;
    uint32_t thr = or_accept_threshold((uint64_t)best_d, T, &rej);
    if (!rej) {
      uint32_t r[4];
      draw(p, g, (uint32_t)sol, 0xFFFFFFFFu, key, r);
      acc = (r[0] >> 1) < thr;
    }
  }
  if (acc) {
    if (p->credit == 1) credit(c, best_ops, best_k, best_d < 0);   /* reading R2: only the accepted move */
    memcpy(x, cand, sizeof(int32_t) * n);
    st->cur_f[sol] += best_d;
    c->acc++;
    if (st->cur_f[sol] < st->best_f[sol]) {
      st->best_f[sol] = st->cur_f[sol];
      memcpy(st->best + (size_t)sol * n, x, sizeof(int32_t) * n);
    }
  }
}

/* The counts of one generation of one solution into the epoch statistics of
 * its scope and the run totals. */
static void add_counts(const or_params *p, or_state *st, int sol, const or_counts *c) {
  for (int i = 0; i < OR_MAX_OPS; ++i) {
    st->tot_u_op[i] += c->u_op[i];
    st->tot_v_op[i] += c->v_op[i];
    if (p->aos_scope == 1) {
      st->saos[sol].u_op[i] += (uint32_t)c->u_op[i];
      st->saos[sol].v_op[i] += (uint32_t)c->v_op[i];
    } else {
      st->u_op[i] += c->u_op[i];
      st->v_op[i] += c->v_op[i];
    }
  }
  for (int i = 0; i < 3; ++i) {
    st->tot_u_k[i] += c->u_k[i];
    st->tot_v_k[i] += c->v_k[i];
    if (p->aos_scope == 1) {
      st->saos[sol].u_k[i] += (uint32_t)c->u_k[i];
      st->saos[sol].v_k[i] += (uint32_t)c->v_k[i];
    } else {
      st->u_k[i] += c->u_k[i];
      st->v_k[i] += c->v_k[i];
    }
  }
  st->accepted += c->acc;
}

/* At the end of an epoch (g_end a multiple of E): the weight update of the
 * scope, then migration (Alg. 2; Sec. "Island Model and Elite Injection"). */
static void epoch_end(const or_inst *in, const or_params *p, or_state *st, uint32_t g_end, uint32_t mask) {
  int P = p->population;
  uint32_t caps[OR_MAX_OPS];
  op_caps(in, p, caps);
  if (or_lex_mode(in)) {   /* the instance best by the ordered scan; improved when strictly better */
    int b = or_lex_best(in, st, P);
    int improved = or_lex_better(in, st->best_v + 4 * (size_t)b, st->ref_v);
    memcpy(st->ref_v, st->best_v + 4 * (size_t)b, sizeof(st->ref_v));
    st->epoch_ref = st->best_f[b];
    aos_update_flag(p, mask, caps, st, improved);
  } else if (p->aos_scope == 1) {
    for (int s = 0; s < P; ++s) sol_aos_update(p, mask, caps, &st->saos[s], st->best_f[s]);
  } else {
    int64_t ib = st->best_f[0];
    for (int s = 1; s < P; ++s) if (st->best_f[s] < ib) ib = st->best_f[s];
    or_aos_update(in, p, mask, st, ib);
  }
  or_migrate(in, p, in->d.n, st, g_end / p->epoch);
}

/* End of generation g: cooling, then the epoch end when one is reached. */
static void end_generation(const or_inst *in, const or_params *p, or_state *st, uint32_t g, uint32_t mask) {
  st->T_q16 = or_cool(st->T_q16, p->alpha_q32);
  if ((g + 1) % p->epoch == 0) epoch_end(in, p, st, g + 1, mask);
  st->g = g + 1;
}

int or_run(const or_inst *in, const or_params *p, or_state *st, uint32_t n_gens) {
  int n = in->d.n, P = p->population;
  uint32_t mask = or_effective_mask(in, p->op_mask);
  int ids[OR_MAX_OPS];
  int nids = enabled_list(mask, ids);
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * n);
  for (uint32_t it = 0; it < n_gens; ++it) {
    uint32_t g = st->g;
    for (int sol = 0; sol < P; ++sol) {
      or_counts c;
      memset(&c, 0, sizeof c);
      generation(in, p, st, sol, g, st->T_q16, ids, nids, tmp, cand, &c);
      add_counts(p, st, sol, &c);
    }
    end_generation(in, p, st, g, mask);
  }
  free(cand);
  free(tmp);
  return 0;
}

/* ------------------------------------------------------------ parallel runner
 * The same generations as or_run, spread over threads for speed (tests that
 * check long windows).  Within an epoch the solutions do not interact: the
 * weights are fixed and the temperature of generation g depends on g alone,
 * so each thread runs its share of the solutions through the epoch's
 * generations, and the counts are summed before the epoch end. */
typedef struct {
  const or_inst *in;
  const or_params *p;
  or_state *st;
  const int *ids;
  int nids, s0, s1;
  uint32_t g0, L;
  const uint64_t *T;
  or_counts sum;
} or_task;

static void *run_task(void *arg) {
  or_task *t = (or_task *)arg;
  int n = t->in->d.n;
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * n);
  memset(&t->sum, 0, sizeof t->sum);
  for (int sol = t->s0; sol < t->s1; ++sol)
    for (uint32_t i = 0; i < t->L; ++i) {
      or_counts c;
      memset(&c, 0, sizeof c);
      generation(t->in, t->p, t->st, sol, t->g0 + i, t->T[i], t->ids, t->nids, tmp, cand, &c);
      for (int o = 0; o < OR_MAX_OPS; ++o) { t->sum.u_op[o] += c.u_op[o]; t->sum.v_op[o] += c.v_op[o]; }
      for (int q = 0; q < 3; ++q) { t->sum.u_k[q] += c.u_k[q]; t->sum.v_k[q] += c.v_k[q]; }
      t->sum.acc += c.acc;
      if (t->p->aos_scope == 1) {   /* the solution's own counts (owned by this thread) */
        or_sol_aos *a = &t->st->saos[sol];
        for (int o = 0; o < OR_MAX_OPS; ++o) { a->u_op[o] += (uint32_t)c.u_op[o]; a->v_op[o] += (uint32_t)c.v_op[o]; }
        for (int q = 0; q < 3; ++q) { a->u_k[q] += (uint32_t)c.u_k[q]; a->v_k[q] += (uint32_t)c.v_k[q]; }
      }
    }
  free(cand);
  free(tmp);
  return NULL;
}

int or_run_par(const or_inst *in, const or_params *p, or_state *st, uint32_t n_gens, int threads) {
  int P = p->population;
  if (threads < 1) threads = 1;
  if (threads > P) threads = P;
  uint32_t mask = or_effective_mask(in, p->op_mask);
  int ids[OR_MAX_OPS];
  int nids = enabled_list(mask, ids);
  or_task *tasks = (or_task *)calloc((size_t)threads, sizeof(or_task));
  pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
  uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * ((size_t)p->epoch + 1));
  while (n_gens > 0) {
    uint32_t g0 = st->g, E = p->epoch;
    uint64_t nb = ((uint64_t)g0 / E + 1) * E;
    uint32_t g1 = (uint64_t)g0 + n_gens < nb ? g0 + n_gens : (uint32_t)nb;
    uint32_t L = g1 - g0;
    T[0] = st->T_q16;
    for (uint32_t i = 0; i < L; ++i) T[i + 1] = or_cool(T[i], p->alpha_q32);
    for (int k = 0; k < threads; ++k) {
      or_task *t = &tasks[k];
      t->in = in; t->p = p; t->st = st; t->ids = ids; t->nids = nids;
      t->s0 = (int)((int64_t)P * k / threads);
      t->s1 = (int)((int64_t)P * (k + 1) / threads);
      t->g0 = g0; t->L = L; t->T = T;
      if (threads == 1) run_task(t);
      else pthread_create(&th[k], NULL, run_task, t);
    }
    for (int k = 0; k < threads; ++k) {
      if (threads > 1) pthread_join(th[k], NULL);
      const or_counts *c = &tasks[k].sum;
      for (int o = 0; o < OR_MAX_OPS; ++o) {
        st->tot_u_op[o] += c->u_op[o];
        st->tot_v_op[o] += c->v_op[o];
        if (p->aos_scope != 1) { st->u_op[o] += c->u_op[o]; st->v_op[o] += c->v_op[o]; }
      }
      for (int q = 0; q < 3; ++q) {
        st->tot_u_k[q] += c->u_k[q];
        st->tot_v_k[q] += c->v_k[q];
        if (p->aos_scope != 1) { st->u_k[q] += c->u_k[q]; st->v_k[q] += c->v_k[q]; }
      }
      st->accepted += c->acc;
    }
    st->T_q16 = T[L];
    if (g1 % E == 0) epoch_end(in, p, st, g1, mask);
    st->g = g1;
    n_gens -= L;
  }
  free(T);
  free(th);
  free(tasks);
  return 0;
}
