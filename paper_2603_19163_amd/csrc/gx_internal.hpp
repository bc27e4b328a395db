// gx_internal.hpp -- device-resident structures shared by the kernels and the
// host runtime of the gx engine (not part of the public C interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gx {

constexpr int kWave = 64;
constexpr int kOps = 12;
// Each evolve workgroup adds its per-launch counts (2 kOps + 7 of them) into
// one of kShards rows of kEpochSlots 64-bit accumulators, picked by its
// solution index, and lowers the row's smallest best objective (the last
// slot); the epoch kernel folds the rows and clears them for the next launch.
constexpr int kShards = 64;
constexpr int kEpochSlots = 2 * kOps + 8;   // counts (uses, improvements per operator and k; accepted), minimum
constexpr int kMaxQapN = 64;
constexpr uint32_t kQapListPerN = 24;   // QAP entry-list capacity per window: 24 n entries
constexpr int kMaxVrpN = 250;
constexpr int kMaxCoord = 1 << 14;
constexpr int64_t kDeltaBias = int64_t(1) << 47;   // argmin key = ((delta + bias) << 16) | t

enum Kind : int32_t { KTSP = 1, KQAP = 2, KKNAP = 3, KVRP = 4, KCOLOR = 5 };
// operator ids, contiguous per encoding: permutation 0-4; ids 5-7 are the
// LNS operators of single-row permutations and the row operators of
// multi-row solutions; binary 8-9, integer 10-11
enum Op : int32_t { O2OPT = 0, OSWAP = 1, OINS = 2, OOROPT = 3, O3OPT = 4, OROWSWAP = 5, OROWSPLIT = 6,
                    OROWMERGE = 7, OFLIP = 8, OSFLIP = 9, ORESET = 10, OSRESET = 11 };
enum LnsOp : int32_t { OLNSSEG = 5, OLNSSCAT = 6, OLNSGUIDE = 7 };
constexpr uint32_t kLnsMask = (1u << OLNSSEG) | (1u << OLNSSCAT) | (1u << OLNSGUIDE);
constexpr int kLnsMax = 64;   // most entries an LNS step destroys
constexpr int kPermOps = 5;
enum Stage : int32_t { SAUTO = 0, SLDS16 = 1, SLDSXY = 2, SGLB16 = 3, SGLB32 = 4 };
// Evolve-kernel variant: the staging, plus kVarX3 when a permutation job's
// operator set holds 3-opt or, on single-row permutations, an LNS operator
// (their loops are compiled apart from the others, so that jobs without them
// carry none of their branches or wider counters), plus
// kVarLex for a VRPTW instance in the lexicographic mode, plus kVarRows for a
// VRPTW instance in the multi-row form, plus kVarLns (with kVarX3) when a
// single-row permutation job's operator set holds an LNS operator.
constexpr int kVarX3 = 8, kVarLex = 16, kVarRows = 32, kVarLns = 64;
inline int evolve_variant(int kind, uint32_t stage, uint32_t op_mask, uint32_t lex_levels, uint32_t rows) {
  const bool perm = kind == KTSP || kind == KQAP || kind == KVRP;
  const bool lns = perm && !rows && (op_mask & kLnsMask);
  const bool wide = (op_mask & (1u << O3OPT)) || lns;
  return (int)stage | ((perm && wide) ? kVarX3 : 0) | (lns ? kVarLns : 0) |
         ((kind == KVRP && lex_levels) ? kVarLex : 0) | ((kind == KVRP && rows) ? kVarRows : 0);
}

// One uploaded instance.  All pointers are device pointers owned by the instance.
struct DevInst {
  int32_t kind, n, dn, n_edges;
  int32_t capacity, vehicles, service, horizon;
  int32_t lb, ub, has_xy;
  int32_t qap_sums32;         // QAP: 2 n * max F * max D < 2^31 (delta row and pair sums fit int32)
  int32_t qap_h16, pad_q;     // QAP: n * max F * max D < 2^16 (row sums H fit 16 bits: staging 1)
  int32_t vw_d, vw_r, vw_m;   // VRPTW objective weights: distance, routes, longest route
  // VRPTW in the multi-row form: the number of rows (0: a giant tour split by
  // capacity).  A solution then holds n = customers + rows entries: entry
  // e < dn - 1 is customer node e + 1, the others are row markers.
  int32_t rows;
  // VRPTW lexicographic mode: number of levels (0: the weighted mode), each
  // level's objective (1 distance, 2 routes, 3 longest route) and tolerance
  int32_t lex_levels, lex_id[3], lex_tol[3], pad_l;
  int64_t lambda;             // knapsack penalty weight
  const int32_t *xy;          // TSP n x 2 / VRPTW (n+1) x 2 coordinates
  const int16_t *d16;         // TSP n x n / VRPTW dn x dn distances (int16)
  const int32_t *d32;         // TSP n x n distances (int32)
  const int16_t *qf, *qd;     // QAP flow / distance (int16)
  const int32_t *kw, *kv;     // knapsack weights / values
  const int32_t *dem, *rdy, *due;  // VRPTW
  const int32_t *adj_off, *adj;    // colouring CSR (both directions)
  const int32_t *edges;            // colouring edge list
};

// Adaptive-operator-selection state of one solution when the weights are kept
// per solution (aos_scope 1): its weights, stagnation count, its best at the
// start of the epoch, and the counts of the current epoch.  Same layout as
// gx_sol_aos in include/gx.h.
struct SolAos {
  uint32_t w_op[kOps], w_k[3], stag;
  int64_t epoch_ref;
  uint32_t u_op[kOps], v_op[kOps], u_k[3], v_k[3];
};
static_assert(sizeof(SolAos) == 192, "gx_sol_aos layout");

// One solve.  Scalars below `g` change as the solve runs; the epoch kernel
// after every evolve launch updates them.
struct DevJob {
  const DevInst *inst;
  uint64_t seed;
  uint64_t t0_param;
  uint32_t P, C, G, E;
  uint32_t op_mask, credit, aos_A, w_floor;
  uint32_t stag_limit, key, alpha, Q;     // Q = oversample pool size
  uint32_t stage, lds_bytes, islands, mig_epochs;   // island model: see gx_solve_params
  uint32_t mig_mode, mig_n, elite_epochs, aos_scope;   // aos_scope: 0 instance, 1 per solution
  uint32_t init_w[kOps];      // caller's raw initial weights (0: Tab. weight_preset)
  uint32_t w_cap[kOps];       // per-sequence weight caps (Q16; the caller's or the defaults)
  uint32_t lex_levels;        // levels of the lexicographic mode (0: scalar objective)
  uint32_t rows;              // rows of a multi-row VRPTW solution (0: other kinds)
  // ---- mutable state
  uint32_t g, g_stop, stag, done;
  uint64_t T;
  int64_t epoch_ref, inst_best;
  int64_t ref_v[4];           // lexicographic mode: the instance best's vector at the last epoch end
  uint32_t w_op[kOps], w_k[3], pad3;
  unsigned long long u_op[kOps], v_op[kOps], u_k[3], v_k[3];
  unsigned long long accepted;
  unsigned long long tot_u_op[kOps], tot_u_k[3];   // whole-run totals of the credited counts
  unsigned long long tot_v_op[kOps], tot_v_k[3];
  // ---- arrays (device)
  int32_t *cur, *best;        // P x n
  int64_t *cur_f, *best_f;    // P
  int32_t *pool;              // Q x n
  int64_t *pool_f;            // Q
  int64_t *sums;              // 2 x n heuristic row/column sums
  int32_t *best_out;          // n
  unsigned long long *shard;  // kShards x kEpochSlots per-launch accumulators
  SolAos *saos;               // P per-solution AOS records (used with aos_scope 1)
  int64_t *cur_v, *best_v;    // lexicographic mode: P x 4 objective vectors (else null)
  int64_t *pool_v;            // lexicographic mode: Q x 4 vectors of the initial pool
  int64_t best_out_f;
  int32_t best_idx;
  uint32_t lns_cap;           // Q16 weight cap of the LNS operators (0: ids 5-7 are not LNS here)
};

// Permutations of up to kOneBufferN elements are rewritten through the first
// 2 kOneBufferN bytes of the candidate tables when a move is applied (the
// tables are dead then; the bytes above hold the TSP run's counters); longer
// ones through a second tour buffer.
constexpr int kOneBufferN = 1536;

// LDS bytes one evolve workgroup needs for this instance and kernel variant:
// the candidate tables (3968 bytes, or 4736 with the block lengths of 3-opt
// steps) followed by the solution and instance data (rows: the rows of a
// multi-row VRPTW solution, whose n entries include one marker per row).
constexpr uint32_t kTables = 3968, kTablesX3 = 4736;
// LNS scratch per wave, at the end of the workgroup's LDS in the variants
// that may draw LNS steps: three step tables (positions, sources, length)
// and the candidate's entries (VRPTW: the entries of up to kLnsBatch
// candidates, whose splits the lanes then run side by side)
struct LnsTab {
  uint16_t pos[kLnsMax];
  uint8_t src[kLnsMax];
  int32_t L;
  int32_t pad[3];
};
constexpr int kLnsBatch = 16;
__host__ __device__ inline uint32_t lns_wave_bytes(int kind, int n) {
  return 3u * (uint32_t)sizeof(LnsTab) + (kind == KVRP ? (uint32_t)kLnsBatch : 1u) * ((2u * n + 15u) & ~15u);
}
__host__ __device__ inline bool lns_variant(int kind, int var) {
  return (var & kVarLns) && (kind == KTSP || kind == KQAP || kind == KVRP);
}
__host__ __device__ inline uint32_t lds_core_bytes(int kind, int n, int var, int rows) {
  auto al = [](uint32_t b) { return (b + 15u) & ~15u; };
  const int stage = var & 7;
  const uint32_t un = (uint32_t)n, tables = (var & kVarX3) ? kTablesX3 : kTables;
  const uint32_t tours = (n <= kOneBufferN ? 1 : 2) * al(2 * un);
  switch (kind) {
    case KTSP: {
      uint32_t b = tables + tours;
      if (stage == SLDS16) b += al(2 * un * un);
      else if (stage == SLDSXY) b += al(4 * un) + al(2 * un);   // coordinates, edge lengths
      return b;
    }
    case KQAP: {   // F and D(x) rows padded to 8, row sums H (16-bit for staging 1), the two waves'
                   // chunk minima, wave 1's maps, then per wave: deltas, segments, entry lists
      const uint32_t np = (un + 7u) & ~7u, lst = kQapListPerN * un;   // entry-list capacity per window
      return tables + tours + 2 * al(2 * un * np) + al((stage == 1 ? 2u : 4u) * un * un) + 16 + 24 * kWave +
             2 * (16 * kWave + al(lst) + al(2 * lst));
    }
    case KKNAP: return tables + al(un) + 2 * al(4 * un);
    case KVRP: {   // distances and node records over the depot and the customers, chunk minima, and
                   // the chunk's candidate vectors in the lexicographic mode
      const uint32_t dn = un - (uint32_t)rows + 1u;
      return tables + tours + al(2 * dn * dn) + 16 * dn + 16 + ((var & kVarLex) ? 128u * 32u : 0u);
    }
    default: return tables + al(2 * un) + al(4 * (un + 1));   // + adjacency, added by the caller
  }
}
__host__ __device__ inline uint32_t lds_bytes_for(int kind, int n, int var, int rows) {
  const uint32_t lns = lns_variant(kind, var) ? 2u * lns_wave_bytes(kind, n) : 0u;
  return lds_core_bytes(kind, n, var, rows) + lns;
}

}  // namespace gx

// Launch wrappers implemented in gx_kernels.hip (measure_peaks: gx_peaks.hip).
struct gx_peaks;
namespace gxk {
hipError_t measure_peaks(int cus, hipStream_t s, ::gx_peaks *out);
hipError_t set_exp_tables(const uint32_t *hi, const uint32_t *lo);
hipError_t build_tsp_d16_from_xy(const int32_t *xy, int n, int16_t *d16, hipStream_t s);
hipError_t build_d32_from_xy(const int32_t *xy, int n, int32_t *d32, hipStream_t s);
hipError_t init_jobs(gx::DevJob *jobs, int count, uint32_t max_q, int max_n, int max_heur_mats,
                     hipStream_t s);
hipError_t set_stop(gx::DevJob *jobs, int count, uint32_t add, int use_total, hipStream_t s);
hipError_t evolve_plain(gx::DevJob *job, int kind, int stage, uint32_t P, uint32_t lds,
                        hipStream_t s);
hipError_t evolve_group(int kind, int stage, gx::DevJob *jobs, const uint2 *items, uint32_t n_items, uint32_t *next,
                        uint32_t grid, uint32_t lds, hipStream_t s);
hipError_t fetch_best(gx::DevJob *jobs, int count, hipStream_t s);
// mig: some job of the launch may migrate or inject its elite (island model)
hipError_t epoch(gx::DevJob *jobs, const uint32_t *idx, uint32_t count, uint32_t *next, uint32_t n_next, bool mig,
                 hipStream_t s);
hipError_t prepare_kernel_attrs(uint32_t max_lds);
hipError_t occupancy_plain(int kind, int stage, uint32_t lds, int *blocks_per_cu);
hipError_t occupancy_group(int kind, int stage, uint32_t lds, int *blocks_per_cu);
hipError_t device_check(int what, uint64_t key, const uint64_t *in, uint64_t *out, int64_t count, hipStream_t s);
hipError_t write_job(gx::DevJob *dst, const gx::DevJob &src, hipStream_t s);
hipError_t copy_i64(int64_t *dst, const int64_t *src, hipStream_t s);
}  // namespace gxk
