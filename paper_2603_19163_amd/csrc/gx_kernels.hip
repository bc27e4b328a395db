// gx_kernels.hip -- gfx950 kernels of the population-parallel local search.
//
// One workgroup evolves one solution (paper, Sec. "GPU Parallelization
// Strategy": one block per solution): a single 64-lane wavefront, or two for
// QAP, whose deltas are LDS-gather heavy.  Per generation (Alg. 1) every lane
// samples ceil(C/64) composite moves, evaluates their exact integer deltas
// against the solution and instance data held in LDS, the wave takes the
// lexicographic argmin of (delta, candidate) with DPP shuffles, and the
// acceptance test, the move application and the AOS bookkeeping follow in
// uniform control flow.  Candidates are never copied: a composite of k <= 3
// operators is a chain of position maps, and a position of the candidate is
// read as s[psi_1(psi_2(psi_3(p)))].
//
// A launch runs the generations up to the next AOS epoch boundary for every
// solution of every job it covers; each workgroup adds its operator counts
// into one of the job's accumulator rows, and the epoch kernel that follows
// the launch folds them into the EMA weight update (Eq. ema, Alg. 2).
#include "gx_internal.hpp"

#include <climits>
#include <type_traits>

using namespace gx;

__constant__ uint32_t c_exp_hi[16];
__constant__ uint32_t c_exp_lo[256];

namespace {

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon et al., SC'11); counter (generation, solution,
// 4*candidate + slot, instance key), key = the 64-bit seed.
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t r[4]) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  r[0] = c0; r[1] = c1; r[2] = c2; r[3] = c3;
}

// The same block for per-lane counters with a wave-uniform key: each round's
// two three-way XORs are single v_bitop3_b32 instructions (truth table 0x96),
// which the compiler does not form by itself; the round keys stay scalar.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}
__device__ __forceinline__ void philox_lane(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1, uint32_t r[4]) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c0 = xor3_vvs(hi1, c1, k0);
    c1 = lo1;
    c2 = xor3_vvs(hi0, c3, k1);
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  r[0] = c0; r[1] = c1; r[2] = c2; r[3] = c3;
}

// integer in [0, m) from a 32-bit draw: floor(w * m / 2^32)
__device__ __forceinline__ uint32_t rmap(uint32_t w, uint32_t m) { return __umulhi(w, m); }

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }
// threads of an evolve workgroup: two wavefronts for QAP (they share the
// solution and split the delta entries) and for VRPTW (one candidate per
// lane), one for the other kinds
template <int KIND, int VAR = 0>
constexpr int kThreads = (KIND == KQAP || KIND == KVRP) ? 128 : 64;
// LDS written by this wave visible to all of its lanes (a wave's LDS accesses
// are performed in order; this only keeps the compiler from reordering them)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Wave-uniform parameters of one job.
// The roulettes use cumulative weights: cw[i] = sum of the first i + 1
// weights of the encoding's operators, sw their total; ck[i] the same for
// the K-step weights, swk their total.
struct Uni {
  uint32_t n, C, key, k0, k1, credit, alpha;
  int32_t lb, ub;
  uint32_t cw[7], sw;
  uint32_t ck[2], swk;
};

struct Step {
  int op, a, b, c;
};

// weighted choice from Q16 weights: u = floor(u16 * S / 2^16); smallest i with
// u < cumsum_i.  An encoding's operators are contiguous ids (permutations 0-4,
// multi-row permutations 0-7, binary 8-9, integer 10-11) and the others have
// weight 0, so only the encoding's own cumulative sums matter.
template <int ENC>
__device__ __forceinline__ int pick_op(uint32_t u16, const Uni &U) {
  const uint32_t u = (uint32_t)(((uint64_t)u16 * U.sw) >> 16);
  if (ENC == 1 || ENC == 2) {
    constexpr int lo = ENC == 1 ? OFLIP : ORESET;
    return lo + (U.cw[0] <= u);
  }
  int op = (U.cw[0] <= u) + (U.cw[1] <= u) + (U.cw[2] <= u) + (U.cw[3] <= u);
  if (ENC >= 3) op += (U.cw[4] <= u) + (U.cw[5] <= u) + (U.cw[6] <= u);
  return op;
}

// k in {1, 2, 3} from the high 16 bits of a draw
__device__ __forceinline__ int pick_k(uint32_t w0, const Uni &U) {
  const uint32_t u = (uint32_t)(((uint64_t)(w0 >> 16) * U.swk) >> 16);
  return 1 + (U.ck[0] <= u) + (U.ck[1] <= u);
}

// Encodings: 0 permutation, 1 binary, 2 integer, 3 multi-row permutation
// (the permutation operators on the entries before the final row marker, and
// the row operators), 4 permutation with the LNS operators (ids 5-7; the
// kernel variants whose operator set holds them).
// first operator id of an encoding
template <int ENC>
constexpr int enc_lo() { return (ENC == 1 || ENC == 2) ? (ENC == 1 ? OFLIP : ORESET) : 0; }
// last operator id of an encoding
template <int ENC>
constexpr int enc_hi() { return ENC == 0 ? O3OPT : (ENC >= 3 ? OROWMERGE : enc_lo<ENC>() + 1); }
template <int ENC>
constexpr bool enc_perm() { return ENC == 0 || ENC >= 3; }

// X3: the operator set holds 3-opt (the loops without it are compiled
// without its branches).  A row operator's step keeps only its drawn position
// (a, uniform over the entries before the final marker): what it moves
// depends on the rows of the candidate it is applied to and is resolved there.
template <int ENC, bool X3>
__device__ __forceinline__ Step make_step(int op, uint32_t r1, uint32_t r2, uint32_t r3, const Uni &U) {
  Step s;
  s.op = op;
  s.c = 0;
  const uint32_t n = U.n;
  if (enc_perm<ENC>()) {
    // 2-opt / swap: two distinct positions i, j of n, ordered; insert /
    // or-opt: block length L, start i of n - L + 1, target q != i of n - L + 1
    // (one code path for both, selecting the ranges); 3-opt: three distinct
    // cuts a < b < c of 0..n, the blocks [a, b) and [b, c) exchanged, which is
    // the block [a, b) moved to start at q = c - (b - a)
    const bool rv = op < OINS;
    const uint32_t L = rv ? 0u : min((op == OINS) ? 1u : 2u + rmap(r3, 2u), n - 1);
    const uint32_t i = rmap(r1, rv ? n : n - L + 1);
    uint32_t j = rmap(r2, rv ? n - 1 : n - L);
    j += (j >= i);
    s.a = (int)(rv ? min(i, j) : i);
    s.b = (int)(rv ? max(i, j) : j);
    s.c = (int)L;
    if (X3 && op == O3OPT) {
      const uint32_t c1 = rmap(r1, n + 1);
      uint32_t c2 = rmap(r2, n);
      c2 += (c2 >= c1);
      const uint32_t lo = min(c1, c2), hi = max(c1, c2);
      uint32_t t = rmap(r3, n - 1);
      t += (t >= lo);
      t += (t >= hi);
      const uint32_t ca = min(lo, t), cc = max(hi, t), cb = lo + hi + t - ca - cc;
      s.a = (int)ca;
      s.b = (int)(cc - (cb - ca));
      s.c = (int)(cb - ca);
    }
    if (n < 2) s.a = s.b = s.c = 0;
    if (ENC == 3 && op >= OROWSWAP) {
      s.a = (int)rmap(r1, n);
      s.b = s.c = 0;
    }
  } else {
    // flip / random reset: one element; seg_flip / seg_reset: L = 2..7
    // consecutive elements (at most n) from a; a step covers [a, a + c)
    const bool seg = op == OSFLIP || op == OSRESET;
    const uint32_t L = seg ? min(2u + rmap(r3, 6u), n) : 1u;
    s.a = (int)rmap(r1, n - L + 1);
    s.b = ENC == 1 ? 0 : U.lb + (int)rmap(r2, (uint32_t)(U.ub - U.lb + 1));
    s.c = (int)L;
  }
  return s;
}

// Sample candidate t of generation g (Alg. 1: k from w_K, then k operators
// from the operator weights).  Returns k.
template <int ENC, bool X3>
__device__ __forceinline__ int sample(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, Step st[3]) {
  uint32_t r[4];
  philox(g, sol, t << 2, U.key, U.k0, U.k1, r);
  const int k = pick_k(r[0], U);
  st[0] = make_step<ENC, X3>(pick_op<ENC>(r[0] & 0xFFFFu, U), r[1], r[2], r[3], U);
  if (k > 1) {
    philox(g, sol, (t << 2) | 1u, U.key, U.k0, U.k1, r);
    st[1] = make_step<ENC, X3>(pick_op<ENC>(r[0] & 0xFFFFu, U), r[1], r[2], r[3], U);
  }
  if (k > 2) {
    philox(g, sol, (t << 2) | 2u, U.key, U.k0, U.k1, r);
    st[2] = make_step<ENC, X3>(pick_op<ENC>(r[0] & 0xFFFFu, U), r[1], r[2], r[3], U);
  }
  return k;
}

// Position map of one permutation step: the element at position p after the
// step was at psi(p) before it.
__device__ __forceinline__ int psi(const Step &s, int p) {
  if (s.op == O2OPT) return (p >= s.a && p <= s.b) ? s.a + s.b - p : p;
  if (s.op == OSWAP) return p == s.a ? s.b : (p == s.b ? s.a : p);
  const int i = s.a, q = s.b, L = s.c;
  if (q < i) {
    if (p < q || p >= i + L) return p;
    return p < q + L ? i + (p - q) : p - L;
  }
  if (p < i || p >= q + L) return p;
  return p < q ? p + L : i + (p - q);
}

// position in the current solution of position p after the first m steps
__device__ __forceinline__ int chain(const Step *st, int m, int p) {
  if (m > 2) p = psi(st[2], p);
  if (m > 1) p = psi(st[1], p);
  if (m > 0) p = psi(st[0], p);
  return p;
}

// ------------------------------------------------------------ LNS steps
// The LNS operators (paper, Sec. "Built-in Operator Hierarchy"; ids 5-7 of a
// single-row permutation) destroy L(n) = min(n, 2 + n / 16, 64) entries and
// rebuild them: the segment shuffle permutes the entries from a uniform
// start, the scatter shuffle the entries at L distinct uniform positions
// (Floyd's sampling), the guided rebuild puts the segment's entries in order
// of their heuristic key (the row sums of the heuristic initialisation),
// ascending or, when the top bit of the step's second word is set,
// descending, ties by entry.  Draws beyond the step's three words are word
// i mod 4 of the Philox4x32-10 block with counter (w1, w2, w3, i / 4) and a
// fixed key.  A drawn step becomes a table in LDS: the L positions it touches
// in increasing order and, for each, the index of the position its new entry
// comes from.  Candidates with such a step are rare (their weights stay
// below 2 %); the whole wave computes their objectives from their entries,
// in place of the per-lane delta, and applies them when they win.
// (shfl64: a 64-bit value from lane src)
__device__ __forceinline__ uint64_t shfl64(uint64_t v, uint32_t src) {
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)src, kWave);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)src, kWave);
  return ((uint64_t)hi << 32) | lo;
}
// the value of v on lane q, for a q that is the same on every lane: a register
// read (v_readlane), with none of a shuffle's round trip through the LDS
// crossbar, for the serial loops below whose every pass waits on the last
__device__ __forceinline__ int lane_val(int v, int q) { return __builtin_amdgcn_readlane(v, q); }
__device__ __forceinline__ int64_t lane_val64(int64_t v, int q) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, q);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), q);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ bool is_lns(int op) { return op >= OLNSSEG && op <= OLNSGUIDE; }
__device__ __forceinline__ int lns_len(int n) { return min(min(2 + n / 16, kLnsMax), n); }
__device__ __forceinline__ uint32_t lns_word(const uint32_t *w, int i) {
  uint32_t r[4];
  philox(w[0], w[1], w[2], (uint32_t)(i >> 2), 0x4C4E5331u, 0x4C4E5332u, r);
  return r[i & 3];
}
// the position the entry at p after an LNS step comes from
__device__ __forceinline__ int lns_psi(const LnsTab &T, bool scat, int p) {
  int i;
  if (!scat) {
    i = p - (int)T.pos[0];
    if ((uint32_t)i >= (uint32_t)T.L) return p;
  } else {
    int lo = 0, hi = T.L;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int)T.pos[mid] < p) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= T.L || (int)T.pos[lo] != p) return p;
    i = lo;
  }
  return T.pos[T.src[i]];
}
// chain() with LNS steps read from their tables
__device__ __forceinline__ int lchain(const Step *st, int m, int p, const LnsTab *tabs) {
#pragma unroll
  for (int j = 2; j >= 0; --j)
    if (j < m) p = is_lns(st[j].op) ? lns_psi(tabs[j], st[j].op == OLNSSCAT, p) : psi(st[j], p);
  return p;
}
// the table of LNS step m (op, words w) of a candidate whose earlier steps
// are st[0..m-1] (their tables built), by the whole wave: lane q draws the
// q-th position and holds the q-th words; the serial loops read the
// other lanes' registers.
__device__ __forceinline__ void lns_make(LnsTab &T, int op, const uint32_t *w, int n, const uint16_t *cur,
                                         const Step *st, const LnsTab *tabs, int m, const int64_t *hkey) {
  const int lane = (int)lane_id();
  const int L = n >= 2 ? lns_len(n) : 0;
  if (L < 2) {
    if (lane == 0) T.L = 0;
    wave_sync();
    return;
  }
  // words q and L + q of the step on lane q (Floyd's draws or the segment's
  // shuffle, and the scattered entries' shuffle)
  const uint32_t wa = lns_word(w, lane), wb = op == OLNSSCAT ? lns_word(w, L + lane) : 0u;
  const int a = (int)rmap(w[0], (uint32_t)(n - L + 1));
  if (op == OLNSSCAT) {
    int pos = 0;
    for (int q = 0; q < L; ++q) {   // Floyd's sampling: position q is r, or j when r is taken
      const int j = n - L + q;
      const int r = (int)rmap((uint32_t)lane_val((int)wa, q), (uint32_t)(j + 1));
      const bool have = __ballot(lane < q && pos == r) != 0ull;
      if (lane == q) pos = have ? j : r;
    }
    int rank = 0;   // increasing order
    for (int q = 0; q < L; ++q) rank += lane_val(pos, q) < pos;
    if (lane < L) T.pos[rank] = (uint16_t)pos;
  } else if (lane < L) {
    T.pos[lane] = (uint16_t)(a + lane);
  }
  wave_sync();
  if (op == OLNSGUIDE) {   // sources ordered by (key, entry) of the entries before the step
    const bool desc = (w[1] >> 31) != 0;
    const int e = lane < L ? (int)cur[lchain(st, m, a + lane, tabs)] : 0;
    const int64_t ky = lane < L ? (desc ? -hkey[e] : hkey[e]) : 0;
    int rank = 0;
    for (int q = 0; q < L; ++q) {
      const int eq = lane_val(e, q);
      const int64_t kq = lane_val64(ky, q);
      rank += kq < ky || (kq == ky && eq < e);
    }
    if (lane < L) T.src[rank] = (uint8_t)lane;
  } else {   // Fisher-Yates on the sources, entry i of the step on lane i
    const uint32_t wf = op == OLNSSCAT ? wb : wa;
    int src = lane;
    for (int i = L - 1; i >= 1; --i) {
      const int j = (int)rmap((uint32_t)lane_val((int)wf, L - 1 - i), (uint32_t)(i + 1));
      const int si = lane_val(src, i), sj = lane_val(src, j);
      src = lane == i ? sj : (lane == j ? si : src);
    }
    if (lane < L) T.src[lane] = (uint8_t)src;
  }
  if (lane == 0) T.L = L;
  wave_sync();
}

// One wave's LNS scratch: the step tables, the candidate's entries, and the
// heuristic keys of the entries (in HBM)
struct LnsCtx {
  LnsTab *tabs;
  uint16_t *y;            // the candidate's entries (VRPTW: buffer b at y + b stride)
  const int64_t *hkey;
  int stride;
};

__device__ __forceinline__ bool lns_in(const Step *st, int k) {
  bool h = false;
#pragma unroll
  for (int m = 0; m < 3; ++m) h |= m < k && is_lns(st[m].op);
  return h;
}
// candidate tl of the chunk has an LNS step among its k (op bytes of the tables)
__device__ __forceinline__ bool lns_drawn(const uint8_t *sop, uint32_t tl, int k) {
  bool h = false;
#pragma unroll
  for (int m = 0; m < 3; ++m) h |= m < k && is_lns((int)(sop[3 * tl + m] & 7u));
  return h;
}
// the tables of the LNS steps of candidate t (steps st, k of them) of
// generation g, built by the calling wave
template <bool X3>
__device__ __forceinline__ void lns_tables(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, const Step *st, int k,
                                           int n, const uint16_t *cur, const LnsCtx &lx) {
  for (int m = 0; m < k; ++m) {   // k and the steps are the same on every lane
    if (!is_lns(st[m].op)) continue;
    uint32_t r[4];
    philox(g, sol, (t << 2) | (uint32_t)m, U.key, U.k0, U.k1, r);
    lns_make(lx.tabs[m], st[m].op, r + 1, n, cur, st, lx.tabs, m, lx.hkey);
  }
}
// the hull of the positions a candidate with LNS steps changes
__device__ __forceinline__ void lns_range(const Step *st, int k, const LnsTab *tabs, int &lo, int &hi) {
  lo = 0x7FFFFFFF;
  hi = -1;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    if (m >= k) continue;
    if (is_lns(st[m].op)) {
      if (tabs[m].L) {
        lo = min(lo, (int)tabs[m].pos[0]);
        hi = max(hi, (int)tabs[m].pos[tabs[m].L - 1]);
      }
    } else {
      const bool mv = st[m].op >= OINS;
      lo = min(lo, mv ? min(st[m].a, st[m].b) : st[m].a);
      hi = max(hi, mv ? max(st[m].a, st[m].b) + st[m].c - 1 : st[m].b);
    }
  }
}
// the entries of candidate t of generation g (which holds an LNS step) into
// dst, by the whole wave
template <bool X3>
__device__ __forceinline__ void lns_entries(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, int n,
                                            const uint16_t *cur, const LnsCtx &lx, uint16_t *dst) {
  Step st[3];
  const int k = sample<4, X3>(U, g, sol, t, st);
  lns_tables<X3>(U, g, sol, t, st, k, n, cur, lx);
  for (int p = (int)lane_id(); p < n; p += kWave) dst[p] = cur[lchain(st, k, p, lx.tabs)];
  wave_sync();
}
// its objective: obj of its entries, the same on every lane
template <bool X3, class OBJ>
__device__ __forceinline__ auto lns_eval(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, int n,
                                         const uint16_t *cur, const LnsCtx &lx, const OBJ &obj) {
  lns_entries<X3>(U, g, sol, t, n, cur, lx, lx.y);
  return obj(lx.y);
}
// The LNS candidates of a round (mask mk, candidate index base + lane) of a
// kind whose objective one lane computes alone (VRPTW): the wave writes the
// entries of up to kLnsBatch of them, then lane b computes batch member b's
// value, which moves to the candidate's own lane.  obj(y) runs on one lane.
template <bool X3, class T, class OBJ>
__device__ __forceinline__ void lns_batched(const Uni &U, uint32_t g, uint32_t sol, uint32_t base, unsigned long long mk,
                                            int n, const uint16_t *cur, const LnsCtx &lx, T &mine, const OBJ &obj) {
  const uint32_t lane = lane_id();
  while (mk) {
    unsigned long long bm = 0ull;
    int cnt = 0;
    for (; mk && cnt < kLnsBatch; ++cnt) {
      const uint32_t t = (uint32_t)__builtin_ctzll(mk);
      mk &= mk - 1;
      bm |= 1ull << t;
      lns_entries<X3>(U, g, sol, base + t, n, cur, lx, lx.y + cnt * lx.stride);
    }
    T v{};
    if ((int)lane < cnt) v = obj(lx.y + lane * lx.stride);
    const uint32_t src = (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));   // this lane's member index
    T got;
    const uint64_t *pv = (const uint64_t *)&v;
    uint64_t *pg = (uint64_t *)&got;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i) pg[i] = shfl64(pv[i], src);
    if ((bm >> lane) & 1ull) mine = got;
    wave_sync();   // the buffers are rewritten by the next batch
  }
}
// apply the winning candidate t (steps st, with an LNS step) to cur through
// tmp; returns the changed range.  Every wave of the workgroup calls it.
template <bool X3>
__device__ __forceinline__ void lns_apply(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, const Step *st, int k,
                                          int n, uint16_t *cur, uint16_t *tmp, const LnsCtx &lx, int &lo, int &hi) {
  lns_tables<X3>(U, g, sol, t, st, k, n, cur, lx);
  lns_range(st, k, lx.tabs, lo, hi);
  for (int p = lo + (int)lane_id(); p <= hi; p += kWave) tmp[p] = cur[lchain(st, k, p, lx.tabs)];
  __syncthreads();
  for (int p = lo + (int)lane_id(); p <= hi; p += kWave) cur[p] = tmp[p];
  __syncthreads();
}


// ------------------------------------------------------------ statistics
struct LStats {
  uint32_t u[kOps], v[kOps], uk[3], vk[3];
};

template <int ENC>
__device__ __forceinline__ void credit(LStats &S, const Step *st, int k, bool imp) {
  constexpr int lo = enc_lo<ENC>(), hi = enc_hi<ENC>();
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    if (m < k) {
#pragma unroll
      for (int o = lo; o <= hi; ++o) {
        const uint32_t hit = st[m].op == o;
        S.u[o] += hit;
        S.v[o] += hit & (uint32_t)imp;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint32_t hit = (k == q + 1);
    S.uk[q] += hit;
    S.vk[q] += hit & (uint32_t)imp;
  }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// The delta of a tour candidate t with an LNS step, by the whole wave: its
// entries over the hull [lo, hi] of the positions its steps change and the
// edges that touch the hull, new against old (el: the current edge lengths,
// or null); when the hull leaves fewer than two positions out, the whole new
// tour against f.  Entries outside the hull are the current ones, so the
// value is the full recomputation's.
template <bool X3, class DF>
__device__ __forceinline__ int64_t lns_tour_delta(const Uni &U, uint32_t g, uint32_t sol, uint32_t t, int n,
                                                  const uint16_t *cur, const uint16_t *el, const LnsCtx &lx,
                                                  const DF &D, int64_t f) {
  Step st[3];
  const int k = sample<4, X3>(U, g, sol, t, st);
  lns_tables<X3>(U, g, sol, t, st, k, n, cur, lx);
  int lo, hi;
  lns_range(st, k, lx.tabs, lo, hi);
  if (hi < lo) return 0;   // no step changes a position
  const int lane = (int)lane_id();
  const bool whole = hi - lo + 2 > n;
  if (whole) {
    lo = 0;
    hi = n - 1;
  }
  uint16_t *y = lx.y;
  for (int p = lo + lane; p <= hi; p += kWave) y[p] = cur[lchain(st, k, p, lx.tabs)];
  wave_sync();
  int64_t acc = 0;
  if (whole) {
    for (int p = lane; p < n; p += kWave) acc += D(y[p], y[p + 1 == n ? 0 : p + 1]);
  } else {   // edges (u, u + 1 mod n) for u = lo - 1 .. hi, all distinct
    for (int j = lane; j <= hi - lo + 1; j += kWave) {
      const int u = lo - 1 + j < 0 ? n - 1 : lo - 1 + j, v = u + 1 == n ? 0 : u + 1;
      const int yu = u >= lo && u <= hi ? y[u] : cur[u], yv = v >= lo && v <= hi ? y[v] : cur[v];
      acc += (int64_t)D(yu, yv) - (el ? (int64_t)el[u] : (int64_t)D(cur[u], cur[v]));
    }
  }
  const int64_t s = wave_sum64(acc);
  wave_sync();   // y is rewritten by the next candidate
  return whole ? s - f : s;
}

// Wave-wide minimum of a 32-bit value with DPP moves only (no LDS path):
// pairs, quads, half rows, rows, then row 0 -> 1 and row 2 -> 3 (row_bcast:15)
// and rows 0-1 -> 2-3 (row_bcast:31); lane 63 ends with the minimum.
// The first four patterns give every lane a source lane (no old value
// needed), so each folds into the minimum as its DPP operand.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false));    // quad_perm 1,0,3,2
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false));    // quad_perm 2,3,0,1
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
  v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, false));   // row_mirror
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// wave-wide minimum of a 64-bit key, high word first (result is uniform)
__device__ __forceinline__ unsigned long long wave_min_key(unsigned long long k) {
  const uint32_t hi = wave_min_u32((uint32_t)(k >> 32));
  const uint32_t lo = wave_min_u32((uint32_t)(k >> 32) == hi ? (uint32_t)k : 0xFFFFFFFFu);
  return ((unsigned long long)hi << 32) | lo;
}

// ------------------------------------------------------------ acceptance, cooling
// Alg. 1: accept when delta < 0 or rand() < e^{-delta/T}; delta = 0 is
// accepted.  e^{-delta/T} comes from the integer tables at z = floor(256
// delta / T) (T in Q16), compared with a 31-bit draw.
//
// Threshold for a delta d > 0, or -1 when the move is rejected outright
// (T = 0 or z >= 4096).  z = floor(2^24 d / T) is exact for every d < 2^63:
// z >= 4096 exactly when 2^12 d >= T; otherwise a = 2^12 d < T and
// z = floor(2^12 a / T) < 4096, whose double quotient is within 2^-38 of the
// true one, so its floor is off by at most one and one comparison of the
// 128-bit products each way makes it exact.
__device__ __forceinline__ int64_t accept_threshold(uint64_t d, uint64_t T) {
  if (T == 0 || d >= (1ull << 52)) return -1;
  const uint64_t a = d << 12;
  if (a >= T) return -1;
  uint64_t z = (uint64_t)((double)a * 4096.0 / (double)T);
  const unsigned __int128 num = (unsigned __int128)a << 12;
  if ((unsigned __int128)z * T > num) --z;
  else if (num - (unsigned __int128)z * T >= T) ++z;
  return (int64_t)(((uint64_t)c_exp_hi[z >> 8] * c_exp_lo[z & 255]) >> 31);
}

__device__ __forceinline__ bool accept_worse(int64_t ds, uint64_t T, uint32_t g, uint32_t sol, const Uni &U) {
  const int64_t p = accept_threshold((uint64_t)ds, T);
  if (p < 0) return false;
  uint32_t r[4];
  philox(g, sol, 0xFFFFFFFFu, U.key, U.k0, U.k1, r);
  return (int64_t)(r[0] >> 1) < p;
}

// T <- floor(T * alpha / 2^32) in 64-bit pieces (Alg. 1, T <- alpha T)
__device__ __forceinline__ uint64_t cool(uint64_t t, uint32_t a) {
  return (t >> 32) * a + (((t & 0xFFFFFFFFull) * a) >> 32);
}

// ------------------------------------------------------------ LDS staging
__device__ __forceinline__ uint32_t al16(uint32_t b) { return (b + 15u) & ~15u; }

// copy `bytes` (rounded up to 16; both buffers padded to 16) global -> LDS
__device__ __forceinline__ void stage16(void *dst, const void *src, uint32_t bytes) {
  const uint4 *s = (const uint4 *)src;
  uint4 *d = (uint4 *)dst;
  const uint32_t cnt = al16(bytes) >> 4;
  for (uint32_t i = lane_id(); i < cnt; i += kWave) d[i] = s[i];
}

// exact nearest-integer Euclidean distance for coordinates in [0, 2^14):
// nint(sqrt(s)) = floor(sqrt(s) + 1/2), which equals (isqrt(4 s) + 1) / 2, is
// the k with k(k-1) < s <= k(k+1).  A float estimate that is never above
// sqrt(s) + 1/2 and at most 0.05 below it gives k or k - 1, and one test
// against k(k+1) decides.  |dx|, |dy| < 2^14 fit int16 lanes (s = dx^2 + dy^2
// is one packed subtract and one 2-term dot product for int16 coordinates) and
// k < 2^15, so the test fits the full-rate 24-bit multiplier.
typedef short s16x2 __attribute__((ext_vector_type(2)));
// (the dot product in its three-operand form with an inline zero: the
// intrinsic becomes the two-operand form, which needs the zero copied into
// its destination first)
__device__ __forceinline__ uint32_t sq_norm(short2 p, short2 q) {   // packed difference, 2-term dot
  const s16x2 d = __builtin_bit_cast(s16x2, p) - __builtin_bit_cast(s16x2, q);
  uint32_t r;
  asm("v_dot2_i32_i16 %0, %1, %1, 0" : "=v"(r) : "v"(__builtin_bit_cast(uint32_t, d)));
  return r;
}
__device__ __forceinline__ uint32_t sq_norm(int2 p, int2 q) {
  const int dx = p.x - q.x, dy = p.y - q.y;
  return (uint32_t)(__mul24(dx, dx) + __mul24(dy, dy));
}
template <class V2>
__device__ __forceinline__ int nint_dist(V2 p, V2 q) {
  const uint32_t s = sq_norm(p, q);
  // sqrt(s) (1 - 2^-19) + 1/2 in float: the conversion, root and fused
  // multiply-add err by < 4 * 2^-24 relative, far less than the 2^-19 shrink
  // (k <= 23170, so the shrink stays below 0.05)
  const float y = __builtin_fmaf(__builtin_amdgcn_sqrtf((float)s), 0.99999809265136719f, 0.5f);
  const uint32_t k0 = (uint32_t)y;
  return (int)(k0 + (s > __umul24(k0, k0) + k0));
}

// kEdges: the tour's edge lengths are kept in LDS (distances that are
// computed rather than looked up)
struct DistL16 {
  static constexpr bool kEdges = false;
  const int16_t *d;
  int n;
  __device__ __forceinline__ int operator()(int a, int b) const { return d[a * n + b]; }
};
struct DistXY {   // coordinates as int16 pairs (they lie in [0, 2^14))
  static constexpr bool kEdges = true;
  const short2 *xy;
  __device__ __forceinline__ int operator()(int a, int b) const { return nint_dist(xy[a], xy[b]); }
};
struct DistG16 {
  static constexpr bool kEdges = false;
  const int16_t *__restrict__ d;
  int n;
  __device__ __forceinline__ int operator()(int a, int b) const { return d[a * n + b]; }
};
struct DistG32 {
  static constexpr bool kEdges = false;
  const int32_t *__restrict__ d;
  int n;
  __device__ __forceinline__ int operator()(int a, int b) const { return d[a * n + b]; }
};

// ------------------------------------------------------------ permutation apply
// The positions a composite move changes lie in [lo, hi], the hull of its
// steps' ranges: [a, b] for a reversal or a swap, [min(i, q), max(i, q) + L - 1]
// for a block move (empty when lo > hi).
__device__ __forceinline__ void move_range(const Step *st, int k, int &lo, int &hi) {
  lo = 0x7FFFFFFF;
  hi = -1;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    if (m < k) {
      const bool mv = st[m].op >= OINS;
      lo = min(lo, mv ? min(st[m].a, st[m].b) : st[m].a);
      hi = max(hi, mv ? max(st[m].a, st[m].b) + st[m].c - 1 : st[m].b);
    }
  }
}

// new solution on [lo, hi] into `tmp` (the candidate tables, dead at this
// point, or a second buffer for long permutations), then back into `cur`
__device__ __forceinline__ void perm_apply(uint16_t *cur, uint16_t *tmp, const Step *st, int k, int lo, int hi) {
  for (int p = lo + (int)lane_id(); p <= hi; p += kWave) tmp[p] = cur[chain(st, k, p)];
  __syncthreads();
  for (int p = lo + (int)lane_id(); p <= hi; p += kWave) cur[p] = tmp[p];
  __syncthreads();
}
__device__ __forceinline__ void perm_apply(uint16_t *cur, uint16_t *tmp, const Step *st, int k) {
  int lo, hi;
  move_range(st, k, lo, hi);
  perm_apply(cur, tmp, st, k, lo, hi);
}

__device__ __forceinline__ void perm_store(const uint16_t *cur, int n, int32_t *dst) {
  for (int p = lane_id(); p < n; p += kWave) dst[p] = cur[p];
}

// ------------------------------------------------------------ QAP
// delta = sum_{a in X} sum_b m_b F[a][b] (D[y_a][y_b] - D[x_a][x_b]), X the
// changed positions, y the candidate, m_b = 1 inside X and 2 outside (F, D symmetric)
// ------------------------------------------------------------ VRPTW (giant tour)
// Parts of a VRPTW solution's objective (over: load above the capacity, which
// only the multi-row form can carry; the giant tour's split avoids it)
struct VrpParts {
  int64_t dist, late;
  int routes, longest;
  int64_t over;
};

// Objective of a VRPTW solution: weighted distance, route count and longest
// route (the weighted multi-objective mode; default weights (1, 0, 0)) plus
// the lateness and fleet penalties, and in the multi-row form 100 per unit of
// a row's load above the capacity.
__device__ __forceinline__ int64_t vrp_objective(const DevInst *I, const VrpParts &q) {
  return (int64_t)I->vw_d * q.dist + (int64_t)I->vw_r * q.routes + (int64_t)I->vw_m * q.longest + 100 * q.late +
         10000 * (int64_t)max(0, q.routes - I->vehicles) + 100 * q.over;
}

// Position map of one step (the element at position p after the step was at
// position map(p) before it), as up to three pieces inside [s1, s1 + len):
// p < e1 -> o1, p < e1b -> o2, else -o1 added to p, or to -p for a reversal
// (neg = -1); positions outside the range are fixed.  Only a swap reaches the
// third piece.
//   reversal of [a, b]:  p -> a + b - p;
//   swap of a < b:        a -> b, b -> a;
//   block [i, i+L) moved to start at q: [q, q+L) -> +(i-q) and [q+L, i+L)
//   -> -L when q < i; [i, q) -> +L and [q, q+L) -> +(i-q) when q > i.
struct SMap {
  int s1, len, e1, e1b, neg, o1, o2;
};

__device__ __forceinline__ SMap smap(int op, int a, int b, int L) {
  const bool mv = op >= OINS, sw = op == OSWAP, qlt = b < a;
  SMap M;
  M.s1 = mv ? min(a, b) : a;
  M.len = (mv ? max(a, b) + L : b + 1) - M.s1;
  M.e1 = mv ? (qlt ? b + L : b) : (sw ? a + 1 : b + 1);
  M.e1b = mv ? max(a, b) + L : b;
  M.neg = (mv || sw) ? 0 : -1;
  M.o1 = mv ? (qlt ? a - b : L) : (sw ? b - a : a + b);
  M.o2 = mv ? (qlt ? -L : a - b) : 0;
  return M;
}

__device__ __forceinline__ int sapply(const SMap &M, int p) {
  const int t = (p ^ M.neg) - M.neg;
  const int off = p < M.e1 ? M.o1 : (p < M.e1b ? M.o2 : -M.o1);
  const bool in = (uint32_t)(p - M.s1) < (uint32_t)M.len;
  return in ? t + off : p;
}

struct TspScratch;

// ---- lexicographic mode (paper, Sec. "Multi-Objective Optimization Modes";
// Tab. lexicographic_mode).  A solution's objective vector is (penalty,
// level 1, level 2, level 3): the penalty (lateness and fleet excess, as in
// the weighted mode) compared exactly, then the caller's objectives in
// priority order, two values within a level's tolerance counting as equal so
// that the next level decides.  Unused levels are 0.
struct Vec4 {
  int64_t v[4];
};
struct LexCfg {
  int levels;
  int id[3];        // 1 distance, 2 routes, 3 longest route
  int64_t tol[3];
};

__device__ __forceinline__ LexCfg lex_cfg(const DevInst *I) {
  LexCfg L;
  L.levels = I->lex_levels;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    L.id[i] = I->lex_id[i];
    L.tol[i] = I->lex_tol[i];
  }
  return L;
}

__device__ __forceinline__ Vec4 lex_vector(const VrpParts &q, int vehicles, const LexCfg &L) {
  Vec4 x;
  x.v[0] = 100 * q.late + 10000 * (int64_t)max(0, q.routes - vehicles) + 100 * q.over;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int id = i < L.levels ? L.id[i] : 0;
    x.v[1 + i] = id == 1 ? q.dist : (id == 2 ? (int64_t)q.routes : (id == 3 ? (int64_t)q.longest : 0));
  }
  return x;
}

// a strictly better than b
__device__ __forceinline__ bool lex_better(const Vec4 &a, const Vec4 &b, const LexCfg &L) {
  if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= L.levels) break;
    if (a.v[1 + i] + L.tol[i] < b.v[1 + i]) return true;
    if (b.v[1 + i] + L.tol[i] < a.v[1 + i]) return false;
  }
  return false;
}

// The worsening a winner w brings against the current c (c strictly better
// than w), for the acceptance test: the penalty difference when the
// penalties differ, else the difference at the first level where c is better
// than w by more than the tolerance.
__device__ __forceinline__ int64_t lex_delta(const Vec4 &w, const Vec4 &c, const LexCfg &L) {
  if (w.v[0] != c.v[0]) return w.v[0] - c.v[0];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (i < L.levels && c.v[1 + i] + L.tol[i] < w.v[1 + i]) return w.v[1 + i] - c.v[1 + i];
  return 0;
}

__device__ __forceinline__ Vec4 load_vec(const int64_t *p) {
  Vec4 x;
#pragma unroll
  for (int i = 0; i < 4; ++i) x.v[i] = p[i];
  return x;
}
__device__ __forceinline__ void store_vec(int64_t *p, const Vec4 &x) {
#pragma unroll
  for (int i = 0; i < 4; ++i) p[i] = x.v[i];
}

// The candidate's giant tour is read through its position maps and split in
// one pass; each customer's demand, ready and due times come in one 16-byte
// LDS read, and the three distances a position may need (previous customer
// to this one, previous customer to the depot, depot to this one) are read
// before the route-break test, which then only selects among them.  Two
// waves per solution evaluate one candidate per lane (round by round).
//
// ROWS: the multi-row form (paper, Sec. "Solution Structure"; Tab. operators,
// row level).  The solution's n entries are the rows one after another, each
// closed by a marker (entries >= nc), the final entry a marker; a candidate
// is read through its maps in the same way and each row is a route from the
// depot and back.  Row operator steps are resolved on the candidate as the
// earlier steps left it (resolve_rows) before their maps are built.
template <bool ROWS>
struct VrpK {
  static constexpr int ENC = ROWS ? 3 : 0;
  static constexpr bool kOneLaneObjective = true;   // one lane computes a solution's objective
  uint16_t *cur, *nxt;
  int n, dn, cap, veh, svc, hor;
  const int16_t *D;
  const int4 *attr;   // (demand, ready, due, 0) per node
  const DevInst *I;
  int nc;             // customers (dn - 1)
  __device__ __forceinline__ int64_t eval(const Step *st, int k) const { return vrp_objective(I, parts(st, k)); }
  // Row operator steps of a candidate replaced by the block moves they make
  // on the candidate after its earlier steps (the solution's entry at
  // position p after steps 0..m-1 is cur[chain(st, m, p)]); a step that does
  // nothing becomes an empty block move.  Position n-1 always holds a marker
  // (the permutation steps act on the first n-1 entries, and no row step moves
  // anything past a marker at n-1), which ends every scan below.
  __device__ __forceinline__ void resolve_rows(Step *st, int k) const {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m >= k || st[m].op < OROWSWAP) continue;
      const int op = st[m].op, p = st[m].a;
      int a = 0, b = 0, L = 0;
      if (op == OROWSPLIT) {   // the empty last row's marker moves to p
        if (n >= 2 && p < n - 2 && (int)cur[chain(st, m, n - 2)] >= nc) {
          a = n - 2;
          b = p;
          L = 1;
        }
      } else {
        int e1 = p;            // the marker that closes p's row
        while (e1 < n - 1 && (int)cur[chain(st, m, e1)] < nc) ++e1;
        if (op == OROWMERGE) {   // that marker moves to just before the final one
          if (e1 < n - 2) {
            a = e1;
            b = n - 2;
            L = 1;
          }
        } else if (e1 < n - 1) {   // row swap: the row [s, e1] and the next one [e1 + 1, e2]
          int s0 = p, e2 = e1 + 1;
          while (s0 > 0 && (int)cur[chain(st, m, s0 - 1)] < nc) --s0;
          while (e2 < n - 1 && (int)cur[chain(st, m, e2)] < nc) ++e2;
          a = s0;
          b = s0 + e2 - e1;
          L = e1 - s0 + 1;
        }
      }
      st[m].a = a;
      st[m].b = b;
      st[m].c = L;
    }
  }
  __device__ __forceinline__ VrpParts parts(const Step *st_in, int k) const {
    Step st[3] = {st_in[0], st_in[1], st_in[2]};
    if constexpr (ROWS) resolve_rows(st, k);
    // the candidate's position maps, branch-free (identity past its k steps)
    SMap M[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      M[m] = smap(st[m].op, st[m].a, st[m].b, st[m].c);
      if (m >= k) M[m].len = 0;
    }
    int64_t late = 0;
    // distances, times and route lengths stay below 2^31 (n <= 250, entries < 2^15, times <= 2^19).
    // The entries are taken kB at a time: the LDS reads of a batch (entries,
    // node records, the distances from each entry's predecessor) depend on
    // the sequence alone and are issued together; only the time, load and
    // route arithmetic runs entry after entry.
    constexpr int kB = 8;
    if constexpr (ROWS) {
      int64_t over = 0;
      int dist = 0, t = 0, load = 0, routes = 0, prev = 0, len = 0, longest = 0;
      for (int p0 = 0; p0 < n; p0 += kB) {
        int cc[kB], dd[kB];
        bool mk[kB];
        int4 aa[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int p = min(p0 + u, n - 1);
          const int e = cur[sapply(M[0], sapply(M[1], sapply(M[2], p)))];
          mk[u] = e >= nc;
          cc[u] = mk[u] ? 0 : e + 1;
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          aa[u] = attr[cc[u]];
          dd[u] = D[(u == 0 ? prev : cc[u - 1]) * dn + cc[u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          if (p0 + u < n) {
            // a marker closes its row: back to the depot when the row has customers
            const bool open = prev != 0, close = mk[u] && open;
            const int step = (mk[u] && !open) ? 0 : dd[u];
            dist += step;
            len += step;
            const int ta = t + step, tw = max(ta, aa[u].y);
            late += mk[u] ? (close ? max(0, ta - hor) : 0) : max(0, tw - aa[u].z);
            longest = close ? max(longest, len) : longest;
            over += mk[u] ? max(0, load - cap) : 0;
            routes += close ? 1 : 0;
            t = mk[u] ? 0 : tw + svc;
            len = mk[u] ? 0 : len;
            load = mk[u] ? 0 : load + aa[u].x;
            prev = cc[u];
          }
        }
      }
      return VrpParts{dist, late, routes, longest, over};
    } else {
      int dist = 0, t = 0, load = 0, routes = n > 0 ? 1 : 0, prev = 0, len = 0, longest = 0;
      for (int p0 = 0; p0 < n; p0 += kB) {
        int cc[kB], dpc[kB], dp0[kB], d0c[kB];
        int4 aa[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u)
          cc[u] = cur[sapply(M[0], sapply(M[1], sapply(M[2], min(p0 + u, n - 1))))] + 1;
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int pv = u == 0 ? prev : cc[u - 1];
          aa[u] = attr[cc[u]];
          dpc[u] = D[pv * dn + cc[u]];
          dp0[u] = D[pv * dn];
          d0c[u] = D[cc[u]];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          if (p0 + u < n) {
            // a demand never exceeds the capacity, so the first customer opens no second route
            const bool brk = load + aa[u].x > cap;
            late += brk ? max(0, t + dp0[u] - hor) : 0;
            longest = brk ? max(longest, len + dp0[u]) : longest;
            dist += brk ? dp0[u] : 0;
            routes += brk ? 1 : 0;
            t = brk ? 0 : t;
            len = brk ? 0 : len;
            load = brk ? 0 : load;
            const int d = brk ? d0c[u] : dpc[u];
            dist += d;
            len += d;
            t = max(t + d, aa[u].y);
            late += max(0, t - aa[u].z);
            t += svc;
            load += aa[u].x;
            prev = cc[u];
          }
        }
      }
      if (n > 0) {
        const int back = D[prev * dn];
        dist += back;
        late += max(0, t + back - hor);
        longest = max(longest, len + back);
      }
      return VrpParts{dist, late, routes, longest, 0};
    }
  }
  // the delta of this lane's candidate of the wave's round (k = 0: no candidate)
  template <bool X3>
  __device__ __forceinline__ int64_t delta_round(const TspScratch &W, int tl, int k, int64_t f) const;
  __device__ __forceinline__ void apply(const Step *st_in, int k) {
    Step st[3] = {st_in[0], st_in[1], st_in[2]};
    if constexpr (ROWS) resolve_rows(st, k);   // every lane reads the same solution: the same steps
    perm_apply(cur, nxt, st, k);
  }
  __device__ __forceinline__ void refresh(int, int) {}
  // parts of the solution with entries y (LNS candidates; every lane the same)
  __device__ __forceinline__ VrpParts parts_of(const uint16_t *y) const {
    VrpK k2 = *this;
    k2.cur = (uint16_t *)y;
    const Step none[3] = {};
    return k2.parts(none, 0);
  }
  __device__ __forceinline__ int64_t objective_of(const uint16_t *y) const { return vrp_objective(I, parts_of(y)); }
  __device__ __forceinline__ void store(int32_t *dst) const { perm_store(cur, n, dst); }
};

// ------------------------------------------------------------ 0/1 knapsack
struct KnapK {
  static constexpr int ENC = 1;
  uint8_t *bits;
  const int32_t *w, *v;
  int n;
  int64_t W, V, cap, lam;
  // step m flips the bits [a, a + c); a bit's value before step m is its
  // stored value flipped by every earlier step that covers it
  __device__ __forceinline__ void dwv(const Step *st, int k, int64_t &dW, int64_t &dV) const {
    dW = 0;
    dV = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m < k) {
        for (int i = st[m].a; i < st[m].a + st[m].c; ++i) {
          int b = bits[i];
          if (m > 0 && (uint32_t)(i - st[0].a) < (uint32_t)st[0].c) b ^= 1;
          if (m > 1 && (uint32_t)(i - st[1].a) < (uint32_t)st[1].c) b ^= 1;
          const int sg = b ? -1 : 1;
          dW += sg * w[i];
          dV += sg * v[i];
        }
      }
    }
  }
  __device__ __forceinline__ int64_t fval(int64_t W2, int64_t V2) const {
    const int64_t over = W2 - cap;
    return -V2 + lam * (over > 0 ? over : 0);
  }
  __device__ __forceinline__ int64_t delta(const Step *st, int k, int64_t f) const {
    int64_t dW, dV;
    dwv(st, k, dW, dV);
    return fval(W + dW, V + dV) - f;
  }
  __device__ __forceinline__ void apply(const Step *st, int k) {
    int64_t dW, dV;
    dwv(st, k, dW, dV);
    W += dW;
    V += dV;
    if (lane_id() == 0)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m < k)
          for (int i = st[m].a; i < st[m].a + st[m].c; ++i) bits[i] ^= 1;
    __syncthreads();
  }
  __device__ __forceinline__ void store(int32_t *dst) const {
    for (int p = lane_id(); p < n; p += kWave) dst[p] = bits[p];
  }
};

// ------------------------------------------------------------ integer colouring
struct ColorK {
  static constexpr int ENC = 2;
  int16_t *val;
  const int32_t *off, *adj;
  int n;
  // value of p while step m sets position i: after the earlier steps
  // (each sets [a, a + c) to b) and the positions of step m before i
  __device__ __forceinline__ int vb(const Step *st, int m, int i, int p) const {
    int v = val[p];
    if (m > 0 && (uint32_t)(p - st[0].a) < (uint32_t)st[0].c) v = st[0].b;
    if (m > 1 && (uint32_t)(p - st[1].a) < (uint32_t)st[1].c) v = st[1].b;
    if (p >= st[m].a && p < i) v = st[m].b;
    return v;
  }
  // the positions of every step change one at a time, in order: each change
  // moves the count by the neighbours that match the new value minus those
  // that matched the old one
  __device__ __forceinline__ int64_t delta(const Step *st, int k, int64_t) const {
    int d = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m < k) {
        const int nv = st[m].b;
        for (int i = st[m].a; i < st[m].a + st[m].c; ++i) {
          const int ov = vb(st, m, i, i);
          for (int e = off[i]; e < off[i + 1]; ++e) {
            const int vj = vb(st, m, i, adj[e]);
            d += (nv == vj) - (ov == vj);
          }
        }
      }
    }
    return d;
  }
  __device__ __forceinline__ void apply(const Step *st, int k) {
    if (lane_id() == 0)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        if (m < k)
          for (int i = st[m].a; i < st[m].a + st[m].c; ++i) val[i] = (int16_t)st[m].b;
    __syncthreads();
  }
  __device__ __forceinline__ void store(int32_t *dst) const {
    for (int p = lane_id(); p < n; p += kWave) dst[p] = val[p];
  }
};

// ------------------------------------------------------------ TSP, step-major
// Every TSP operator is one or two "pattern" steps that share one delta
// formula: 2-opt is a reversal, a swap of non-adjacent positions is the
// reversal of [lo, hi] followed by that of [lo+1, hi-1], insert / or-opt is a
// block move.  Per chunk of 128 candidates the wave draws all first steps
// (evaluated on the candidates' own lanes from the drawn registers), then the
// extra steps of the candidates with k >= 2 compacted onto the lanes, builds
// the list of pattern steps grouped by their position in the composite,
// evaluates it with all lanes busy, and sums each candidate's delta with LDS
// atomics.  Draws, moves and deltas are those of the per-candidate
// formulation; only the order of evaluation differs.  (Evaluating each extra
// step's patterns on the lane that drew it, without the grouped list, ran
// slower: swaps and third steps diverge within the wave.)
constexpr int kChunk = 128;
// tables (positions, deltas, pattern list, operator bytes), then for 3-opt
// variants the block lengths of the steps
constexpr uint32_t kTspScratch = kChunk * 3 * 4 + kChunk * 4 + kChunk * 6 * 2 + kChunk * 3;
static_assert(kTspScratch == kTables && kTables + kChunk * 3 * 2 == kTablesX3,
              "lds_bytes_for() reserves the candidate tables");
// The pattern list holds at most 2 x 2 entries per candidate of a chunk
// (steps 2 and 3, two patterns each): 1024 bytes from offset 2048; the rest of
// its 1536 bytes, up to the operator table at 3584, is free on the TSP path
// (a move's rewrite through the tables stays below it).
constexpr uint32_t kTspStatsOff = 2048 + kChunk * 2 * 2 * 2;
static_assert(2 * kOneBufferN <= (int)kTspStatsOff, "tour rewrite below the TSP counters");

// Dynamic LDS of the evolve kernels; the candidate tables sit at fixed offsets
// from its start (so their addresses are compile-time constants).
extern __shared__ __align__(16) char gx_lds[];

struct TspScratch {
  __device__ __forceinline__ uint32_t *sab() const { return (uint32_t *)gx_lds; }         // a | b << 16 at [3t + m]
  __device__ __forceinline__ int32_t *del() const { return (int32_t *)(gx_lds + 1536); }  // delta accumulators
  __device__ __forceinline__ uint16_t *lst() const { return (uint16_t *)(gx_lds + 2048); } // t | m << 8 | sub << 10
  // extra draws t | m << 8; used only before the pattern list is built
  __device__ __forceinline__ uint16_t *dl() const { return (uint16_t *)(gx_lds + 2048); }
  // op - first op of the encoding | L << 3 at [3t + m], k << 6 at m = 0 (L of a 3-opt step in sl)
  __device__ __forceinline__ uint8_t *sop() const { return (uint8_t *)(gx_lds + 3584); }
  __device__ __forceinline__ uint16_t *sl() const { return (uint16_t *)(gx_lds + 3968); }   // block length of a 3-opt step
};

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// number of pattern steps of an operator
__device__ __forceinline__ int n_patterns(int op, int a, int b) { return (op == OSWAP && b - a >= 2) ? 2 : 1; }


template <bool X3>
__device__ __forceinline__ void unpack_step(const TspScratch &W, int t, int m, int &op, int &a, int &b, int &L) {
  const uint32_t ab = W.sab()[3 * t + m];
  const uint32_t ol = W.sop()[3 * t + m];
  a = (int)(ab & 0xFFFFu);
  b = (int)(ab >> 16);
  op = (int)(ol & 7u);
  L = (X3 && op == O3OPT) ? (int)W.sl()[3 * t + m] : (int)((ol >> 3) & 7u);
}

// a step into the tables (the operator relative to its encoding's first id)
template <int ENC, bool X3>
__device__ __forceinline__ void store_step(const TspScratch &W, uint32_t idx, const Step &st, uint32_t kbits) {
  W.sab()[idx] = (uint32_t)(uint16_t)st.a | ((uint32_t)(uint16_t)st.b << 16);
  W.sop()[idx] = (uint8_t)((st.op - enc_lo<ENC>()) | ((st.c & 7) << 3) | kbits);
  if (X3 && enc_perm<ENC>() && st.op == O3OPT) W.sl()[idx] = (uint16_t)st.c;
}

// Draw the composite moves of candidates [c0, c0 + cn): the first step of
// every candidate on its own lane (t = c0 + r*64 + lane), then the extra steps
// of the candidates with k >= 2 and k >= 3 compacted onto consecutive lanes,
// so that the wave computes about as many Philox blocks as there are steps.
// Steps land in the LDS tables; kk[r] receives k of the lane's candidates,
// first[r] (when given) their first steps.  Returns the length of the list of
// extra steps (candidate | step << 8 at dl + 128 rb).
template <int ENC, bool X3, int RN = 2>
__device__ __forceinline__ uint32_t draw_chunk(const TspScratch &W, const Uni &U, uint32_t g, uint32_t sol, uint32_t c0,
                                               uint32_t cn, int kk[RN], uint32_t rb = 0, Step *first = nullptr) {
  // rounds rb .. rb + RN - 1 of the chunk (64 candidates each) on this wave;
  // its extra-step list at dl + 128 rb
  const uint32_t lane = lane_id();
  uint16_t *dl = W.dl() + 128 * rb;
#pragma unroll
  for (int rr = 0; rr < RN; ++rr) {
    const uint32_t tl = (rb + rr) * kWave + lane;
    kk[rr] = 0;
    if (tl < cn) {
      uint32_t w[4];
      philox_lane(g, sol, (c0 + tl) << 2, U.key, U.k0, U.k1, w);
      kk[rr] = pick_k(w[0], U);
      const Step st = make_step<ENC, X3>(pick_op<ENC>(w[0] & 0xFFFFu, U), w[1], w[2], w[3], U);
      store_step<ENC, X3>(W, 3 * tl, st, (uint32_t)kk[rr] << 6);
      if (first) first[rr] = st;
      if constexpr (RN == 2) W.del()[tl] = 0;
    }
  }
  uint32_t nx = 0;
#pragma unroll
  for (int m = 1; m < 3; ++m)
#pragma unroll
    for (int rr = 0; rr < RN; ++rr) {
      const bool need = kk[rr] > m;
      const unsigned long long mk = __ballot(need);
      if (need) dl[nx + lanes_below(mk)] = (uint16_t)(((rb + rr) * kWave + lane) | (m << 8));
      nx += (uint32_t)__popcll(mk);
    }
  __syncthreads();
  for (uint32_t j = lane; j < nx; j += kWave) {
    const uint32_t e = dl[j], tl = e & 0xFFu, m = e >> 8;
    uint32_t w[4];
    philox_lane(g, sol, ((c0 + tl) << 2) | m, U.key, U.k0, U.k1, w);
    const Step st = make_step<ENC, X3>(pick_op<ENC>(w[0] & 0xFFFFu, U), w[1], w[2], w[3], U);
    store_step<ENC, X3>(W, 3 * tl + m, st, 0u);
  }
  __syncthreads();
  return nx;
}

// step m of candidate t from the tables (integer values are stored as int16)
template <int ENC, bool X3>
__device__ __forceinline__ Step load_step(const TspScratch &W, int t, int m) {
  const uint32_t ab = W.sab()[3 * t + m];
  const uint32_t ol = W.sop()[3 * t + m];
  Step st;
  st.a = (int)(ab & 0xFFFFu);
  st.b = ENC == 2 ? (int)(int16_t)(ab >> 16) : (int)(ab >> 16);
  st.op = (int)(ol & 7u) + enc_lo<ENC>();
  st.c = (X3 && enc_perm<ENC>() && st.op == O3OPT) ? (int)W.sl()[3 * t + m] : (int)((ol >> 3) & 7u);
  return st;
}

// delta of pattern step `sub` of operator m of candidate t, on the tour after
// all earlier steps of that candidate (MAPPED: m >= 1, whose read positions
// are mapped back through steps m-1 .. 0)
template <bool ROWS>
template <bool X3>
__device__ __forceinline__ int64_t VrpK<ROWS>::delta_round(const TspScratch &W, int tl, int k, int64_t f) const {
  if (k == 0) return 0;
  Step st[3];
  st[0] = load_step<ENC, X3>(W, tl, 0);
  st[1] = k > 1 ? load_step<ENC, X3>(W, tl, 1) : st[0];
  st[2] = k > 2 ? load_step<ENC, X3>(W, tl, 2) : st[0];
  return eval(st, k) - f;
}

template <bool MAPPED, bool X3, class DF>
__device__ __forceinline__ int pattern_delta(const TspScratch &W, const uint16_t *tour, int n, const DF &D,
                                             int t, int m, int sub) {
  int op, a, b, L;
  unpack_step<X3>(W, t, m, op, a, b, L);
  // Every pattern reads the tour at (X-1, X, r2, r3, Z-1, Z): a block move
  // cuts before X = min(i, q), before B and before Z = max(i, q) + L, with
  // B = i (q < i) or i + L (q > i), so (r2, r3) = (B-1, B); a reversal of
  // [lo, hi] has X = lo, Z = hi + 1 and (r2, r3) = (lo, hi), whose two terms
  // cancel.  Only X-1 and Z can leave [0, n).  A pattern with X = 0 and
  // Z = n (a full reversal or a rotation), or a move of length 0, is zero.
  // The second reversal of a swap (a, b), [a+1, b-1] after [a, b], reads
  // positions b, b-1, b-1, a+1, a+1, a of the tour before the swap.
  const bool mv = op >= OINS;
  const int X = mv ? min(a, b) : a;
  const int Z = mv ? max(a, b) + L : b + 1;
  const int B = a + (b < a ? 0 : L);
  const bool zero = !sub && ((X == 0 && Z == n) || (mv && L == 0));
  int r[6];
  r[0] = sub ? b : (X == 0 ? n : X) - 1;
  r[1] = sub ? b - 1 : X;
  r[2] = sub ? b - 1 : (mv ? B - 1 : X);
  r[3] = sub ? a + 1 : (mv ? B : Z - 1);
  r[4] = sub ? a + 1 : Z - 1;
  r[5] = sub ? a : (Z == n ? 0 : Z);
  if (MAPPED) {
    for (int mm = m - 1; mm >= 0; --mm) {
      int o2, a2, b2, L2;
      unpack_step<X3>(W, t, mm, o2, a2, b2, L2);
      const SMap M = smap(o2, a2, b2, L2);
#pragma unroll
      for (int i = 0; i < 6; ++i) r[i] = sapply(M, r[i]);
    }
  }
  int v[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = tour[r[i]];
  const int d = D(v[0], v[3]) - D(v[0], v[1]) + D(v[4], v[1]) - D(v[2], v[3]) + D(v[2], v[5]) - D(v[4], v[5]);
  return zero ? 0 : d;
}

// Edge lengths of the tour: el[p] = D(tour[p], tour[p + 1 mod n]) for the
// positions p in [lo, hi] taken modulo n (lo may be -1).
template <class DF>
__device__ __forceinline__ void edges_fill(uint16_t *el, const uint16_t *tour, int n, const DF &D, int lo, int hi) {
  for (int p = lo + (int)lane_id(); p <= hi; p += kWave) {
    const int q = p < 0 ? p + n : p;
    el[q] = (uint16_t)D(tour[q], tour[q + 1 == n ? 0 : q + 1]);
  }
}

// Delta of the first step of candidate t, on the current tour, with every
// operator in one form over six tour positions u0..u5: new edges
// (u0,u1), (u1,u2) or (u2,u5), (u3,u4), (u4,u5) and removed edges e0..e3
// (positions e, e + 1), read from the edge lengths when they are kept.
//   swap lo < hi:  u = (lo-1, hi, lo+1, hi-1, lo, hi+1), all four pairs,
//                  removed edges lo-1, lo, hi-1, hi;
//   reversal of [lo, hi]: the same positions, pairs 0 and 3, removed edges
//                  lo-1 and hi (an adjacent swap is the reversal of [lo, hi];
//                  a swap of positions 0 and n-1, neighbours on the cycle,
//                  gives the same cycle as the reversal of [1, n-2]);
//   block move with cuts X, B, Z (see pattern_delta):
//                  u = (X-1, B, B-1, Z-1, X, Z), pairs 0, 1 (as (u2,u5)) and 2,
//                  removed edges X-1, B-1, Z-1.
// Zero patterns as in pattern_delta.
template <class DF>
__device__ __forceinline__ int first_step_delta(const uint16_t *tour, const uint16_t *el, int n, const DF &D, int op,
                                                int a, int b, int L) {
  const bool mv = op >= OINS;
  const bool adj = op == OSWAP && b - a == 1;
  const bool cyc = op == OSWAP && !adj && a == 0 && b == n - 1;
  const bool sw = op == OSWAP && !adj && !cyc;
  const int lo = cyc ? 1 : a, hi = cyc ? n - 2 : b;
  const int P = lo == 0 ? n - 1 : lo - 1, N = hi == n - 1 ? 0 : hi + 1;
  const int X = min(a, b), Z = max(a, b) + L, B = a + (b < a ? 0 : L);
  const int Xm = X == 0 ? n - 1 : X - 1, Zw = Z == n ? 0 : Z;
  const bool zero = mv ? (L == 0 || (X == 0 && Z == n)) : (!sw && lo == 0 && hi == n - 1);
  int u[6], e[4];
  u[0] = mv ? Xm : P;
  u[1] = mv ? B : hi;
  u[2] = mv ? B - 1 : lo + 1;
  u[3] = mv ? Z - 1 : hi - 1;
  u[4] = mv ? X : lo;
  u[5] = mv ? Zw : N;
  e[0] = u[0];
  e[1] = mv ? B - 1 : lo;
  e[2] = mv ? Z - 1 : hi - 1;
  e[3] = hi;
  int c[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) c[i] = tour[u[i]];
  const int d0 = D(c[0], c[1]);
  const int d1 = D(mv ? c[2] : c[1], mv ? c[5] : c[2]);
  const int d2 = D(c[3], c[4]);
  const int d3 = D(c[4], c[5]);
  int o[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if constexpr (DF::kEdges) o[i] = el[e[i]];
    else o[i] = D(tour[e[i]], tour[e[i] + 1 == n ? 0 : e[i] + 1]);
  }
  // pairs used: swap all, reversal 0 and 3, block move 0, 1, 2
  const bool mid = mv || sw, last = !mv;
  int d = d0 - o[0];
  d += mid ? d1 - o[1] + d2 - o[2] : 0;
  d += last ? d3 - o[3] : 0;
  return zero ? 0 : d;
}

// Adds the wave-wide sums of per-lane byte counters (field i at bits 8i) to
// the uniform counts u[i] and v[i]; even and odd bytes are widened to 16-bit
// fields first so that the 64-lane sums cannot carry into a neighbour.
__device__ __forceinline__ void fold_byte_counts(uint32_t *u, uint32_t *v, uint32_t cu, uint32_t cv, int fields) {
  const uint32_t ue = uni(wave_sum(cu & 0x00FF00FFu)), uo = uni(wave_sum((cu >> 8) & 0x00FF00FFu));
  const uint32_t ve = uni(wave_sum(cv & 0x00FF00FFu)), vo = uni(wave_sum((cv >> 8) & 0x00FF00FFu));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (i >= fields) break;
    const int sh = (i >> 1) << 4;
    u[i] += ((i & 1 ? uo : ue) >> sh) & 0xFFFFu;
    v[i] += ((i & 1 ? vo : ve) >> sh) & 0xFFFFu;
  }
}

// The same for 64-bit counters with up to 8 byte fields (operators 4-7 in
// the high word).
__device__ __forceinline__ void fold_op_counts(uint32_t *u, uint32_t *v, uint64_t cu, uint64_t cv, int fields) {
  fold_byte_counts(u, v, (uint32_t)cu, (uint32_t)cv, fields < 4 ? fields : 4);
  if (fields > 4) fold_byte_counts(u + 4, v + 4, (uint32_t)(cu >> 32), (uint32_t)(cv >> 32), fields - 4);
}

// Per-lane operator counters: four byte fields in 32 bits, or with 3-opt (five
// fields) and for the multi-row encoding (eight) in 64 bits.
template <bool W64>
using OpCount = typename std::conditional<W64, uint64_t, uint32_t>::type;
template <bool W64>
__device__ __forceinline__ void fold_ops(uint32_t *u, uint32_t *v, OpCount<W64> cu, OpCount<W64> cv, int fields) {
  if constexpr (W64) fold_op_counts(u, v, cu, cv, fields);
  else fold_byte_counts(u, v, cu, cv, fields < 4 ? fields : 4);
}

template <bool X3, bool LNS, class DF>
__device__ __forceinline__ void tsp_run(uint16_t *cur, uint16_t *nxt, uint16_t *el, int n, const DF &D, const TspScratch &W,
                                        const Uni &U, int32_t *best_row, uint32_t sol, uint32_t g0, uint32_t g1,
                                        uint64_t &T, int64_t &f, int64_t &bf, LStats &S, uint32_t &nacc,
                                        const LnsCtx &lx) {
  const uint32_t lane = lane_id();
  // Per-lane use and improvement counts of the operators and of k = 1..3
  // in byte fields (operator o at bits 8o, k at bits 8(k-1)); a chunk of
  // candidates adds at most 6 to a field of a lane, so the fields are folded
  // into the wave-wide counts of S every 42 chunks and at the end.
  constexpr int kNops = LNS ? 8 : (X3 ? kPermOps : 4);   // the LNS variant: ids 5-7 too
  constexpr int ENC = LNS ? 4 : 0;
  OpCount<X3> cu_op = 0, cv_op = 0;
  uint32_t cu_k = 0, cv_k = 0, since_fold = 0;
  // The wave-wide counts live in the unused tail of the pattern-list table
  // during the run (fewer scalar registers held across the generation loop)
  // and are added into S at the end.  The word after them says whether the
  // current tour is the best-so-far one not yet written to HBM: the best tour
  // is stored lazily, before a move that does not improve on it is applied,
  // or at the end of the launch.
  LStats &SL = *(LStats *)(gx_lds + kTspStatsOff);
  volatile uint32_t *best_is_cur = (volatile uint32_t *)(gx_lds + kTspStatsOff + sizeof(LStats));
  static_assert(sizeof(LStats) % 4 == 0 && sizeof(LStats) / 4 < kWave, "one word per lane");
  static_assert(kTspStatsOff + sizeof(LStats) + 4 <= 3584, "inside the free tail of the pattern list");
  if (lane <= sizeof(LStats) / 4) ((uint32_t *)&SL)[lane] = 0u;
  wave_sync();
  const uint32_t c_last = (U.C - 1) / kChunk * kChunk;
  if constexpr (DF::kEdges) {
    edges_fill(el, cur, n, D, 0, n - 1);
    __syncthreads();
  }
  for (uint32_t g = g0; g < g1; ++g) {
    unsigned long long bk = ~0ull;
    for (uint32_t c0 = 0; c0 < U.C; c0 += kChunk) {
      const uint32_t cn = min((uint32_t)kChunk, U.C - c0);
      int kk[2];
      Step s0[2];
      draw_chunk<ENC, X3>(W, U, g, sol, c0, cn, kk, 0, s0);
      // ---- first steps: one per candidate, on its own lane, from the drawn step
      int d0[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const uint32_t tl = r * kWave + lane;
        d0[r] = (tl < cn && n >= 2) ? first_step_delta(cur, el, n, D, s0[r].op, s0[r].a, s0[r].b, s0[r].c) : 0;
      }
      // ---- later steps of k >= 2 candidates: (candidate, step, pattern)
      // entries, grouped by step, evaluated through the position maps
      uint32_t nq = 0;
#pragma unroll
      for (int m = 1; m < 3; ++m) {
        if (!__ballot(kk[0] > m || kk[1] > m)) break;
#pragma unroll
        for (int sub = 0; sub < 2; ++sub)
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const uint32_t tl = r * kWave + lane;
            bool need = kk[r] > m;
            if (need && sub) {
              int op, a, b, L;
              unpack_step<X3>(W, (int)tl, m, op, a, b, L);
              need = n_patterns(op, a, b) == 2;
            }
            const unsigned long long mk = __ballot(need);
            if (need) W.lst()[nq + lanes_below(mk)] = (uint16_t)(tl | (m << 8) | (sub << 10));
            nq += (uint32_t)__popcll(mk);
          }
      }
      __syncthreads();
      if (n >= 2) {
        for (uint32_t j = lane; j < nq; j += kWave) {
          const uint32_t e = W.lst()[j];
          const int d = pattern_delta<true, X3>(W, cur, n, D, (int)(e & 0xFFu), (int)((e >> 8) & 3u), (int)(e >> 10));
          if (d) atomicAdd(&W.del()[e & 0xFFu], d);
        }
      }
      __syncthreads();
      // ---- candidates with an LNS step (wide variant): their objectives by
      // the whole wave, in place of the per-lane delta
      int64_t lns_d[2] = {0, 0};
      uint32_t lns_c = 0;   // bit r: lane's candidate of round r holds an LNS step
      if constexpr (LNS) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const uint32_t tl = r * kWave + lane;
          const bool has = tl < cn && (is_lns(s0[r].op) || (kk[r] > 1 && lns_drawn(W.sop(), tl, kk[r])));
          for (unsigned long long mk = __ballot(has); mk; mk &= mk - 1) {
            const uint32_t t = (uint32_t)__builtin_ctzll(mk);
            const int64_t dl = lns_tour_delta<X3>(U, g, sol, c0 + r * kWave + t, n, cur, el, lx, D, f);
            if (lane == t) {
              lns_d[r] = dl;
              lns_c |= 1u << r;
            }
          }
        }
      }
      // ---- keys and per-lane statistics (byte counters, folded into S below)
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const uint32_t tl = r * kWave + lane;
        const bool valid = tl < cn;
        int64_t d = valid ? (int64_t)(d0[r] + W.del()[tl]) : 0;
        if constexpr (LNS) d = ((lns_c >> r) & 1u) ? lns_d[r] : d;
        if (U.credit == 0 && valid) {
          const bool imp = d < 0;
#pragma unroll
          for (int m = 0; m < 3; ++m) {   // the first step's operator is in registers
            const uint32_t opm = m == 0 ? (uint32_t)s0[r].op : (W.sop()[3 * tl + m] & 7u);
            const OpCount<X3> inc = kk[r] > m ? (OpCount<X3>)1 << (opm << 3) : (OpCount<X3>)0;
            cu_op += inc;
            cv_op += imp ? inc : (OpCount<X3>)0;
          }
          const uint32_t inck = 1u << ((kk[r] - 1) << 3);
          cu_k += inck;
          cv_k += imp ? inck : 0u;
        }
        if (valid) {
          const unsigned long long key = ((unsigned long long)(d + kDeltaBias) << 16) | (c0 + tl);
          bk = key < bk ? key : bk;
        }
      }
      if (++since_fold == 42) {
        fold_ops<X3>(SL.u, SL.v, cu_op, cv_op, kNops);
        fold_byte_counts(SL.uk, SL.vk, cu_k, cv_k, 3);
        cu_op = cv_op = 0;
        cu_k = cv_k = 0;
        since_fold = 0;
      }
      __syncthreads();
    }
    bk = wave_min_key(bk);
    const uint32_t ts = (uint32_t)(bk & 0xFFFFu);
    const int64_t ds = (int64_t)(bk >> 16) - kDeltaBias;
    bool acc = ds <= 0;
    if (!acc) acc = accept_worse(ds, T, g, sol, U);
    if (acc) {
      // the steps of the winner: from the tables when it was drawn in the
      // last chunk (they still hold that chunk), else drawn again
      Step st[3];
      int k;
      if (ts >= c_last) {
        const int tl = (int)(ts - c_last);
        k = (int)(W.sop()[3 * tl] >> 6);
        st[0] = load_step<ENC, X3>(W, tl, 0);
        st[1] = load_step<ENC, X3>(W, tl, 1);
        st[2] = load_step<ENC, X3>(W, tl, 2);
      } else {
        k = sample<ENC, X3>(U, g, sol, ts, st);
      }
      if (U.credit == 1) {   // wave-uniform counts on this path
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
          for (int o = 0; o < kNops; ++o) {
            const uint32_t hit = m < k && st[m].op == o;
            SL.u[o] += hit;
            SL.v[o] += hit & (uint32_t)(ds < 0);
          }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          SL.uk[q] += (uint32_t)(k == q + 1);
          SL.vk[q] += (uint32_t)(k == q + 1 && ds < 0);
        }
      }
      int lo, hi;
      if constexpr (LNS) {
        if (*best_is_cur && f + ds >= bf) {
          perm_store(cur, n, best_row);
          *best_is_cur = 0u;
        }
        if (lns_in(st, k)) {
          lns_apply<X3>(U, g, sol, ts, st, k, n, cur, nxt, lx, lo, hi);
        } else {
          move_range(st, k, lo, hi);
          perm_apply(cur, nxt, st, k, lo, hi);
        }
      } else {
        move_range(st, k, lo, hi);
        if (*best_is_cur && f + ds >= bf) {
          perm_store(cur, n, best_row);
          *best_is_cur = 0u;
        }
        perm_apply(cur, nxt, st, k, lo, hi);
      }
      if constexpr (DF::kEdges) {
        if (lo <= hi) {
          edges_fill(el, cur, n, D, lo - 1, hi);
          __syncthreads();
        }
      }
      f += ds;
      ++nacc;
      if (f < bf) {
        bf = f;
        *best_is_cur = 1u;
      }
    }
    T = cool(T, U.alpha);
  }
  if (*best_is_cur) perm_store(cur, n, best_row);
  fold_ops<X3>(SL.u, SL.v, cu_op, cv_op, kNops);
  fold_byte_counts(SL.uk, SL.vk, cu_k, cv_k, 3);
  wave_sync();
#pragma unroll
  for (int o = 0; o < kNops; ++o) {
    S.u[o] += SL.u[o];
    S.v[o] += SL.v[o];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    S.uk[q] += SL.uk[q];
    S.vk[q] += SL.vk[q];
  }
}

// ------------------------------------------------------------ generation loop
// ------------------------------------------------------------ QAP
// Positions changed by one step (a superset is enough for the delta below):
// a reversal of [a, b] moves every position but its middle one, a swap two,
// a block move the range [min(i, q), max(i, q) + L).
__device__ __forceinline__ uint64_t range_bits(int lo, int hi) {   // bits lo..hi, empty for lo > hi
  return lo > hi ? 0ull : (2ull << hi) - (1ull << lo);
}
__device__ __forceinline__ uint64_t step_bits(const Step &s) {
  if (s.op == OSWAP) return s.a == s.b ? 0ull : (1ull << s.a) | (1ull << s.b);
  if (s.op < OINS) {
    const uint64_t mid = ((s.a + s.b) & 1) ? 0ull : 1ull << ((s.a + s.b) >> 1);
    return range_bits(s.a, s.b) & ~mid;
  }
  return (s.c == 0 || s.a == s.b) ? 0ull : range_bits(min(s.a, s.b), max(s.a, s.b) + s.c - 1);
}

// A step's position map in 8 bytes (every field of a map over n <= 64 fits a byte).
__device__ __forceinline__ uint2 smap_pack(const SMap &M) {
  const uint32_t lo = (uint32_t)(M.s1 & 255) | (uint32_t)(M.len & 255) << 8 | (uint32_t)(M.e1 & 255) << 16 |
                      (uint32_t)(M.e1b & 255) << 24;
  const uint32_t hi = (uint32_t)(M.neg & 255) | (uint32_t)(M.o1 & 255) << 8 | (uint32_t)(M.o2 & 255) << 16;
  return make_uint2(lo, hi);
}
__device__ __forceinline__ SMap smap_unpack(uint2 v) {
  SMap M;
  M.s1 = (int)(int8_t)(v.x & 255u);
  M.len = (int)(int8_t)((v.x >> 8) & 255u);
  M.e1 = (int)(int8_t)((v.x >> 16) & 255u);
  M.e1b = (int)(int8_t)(v.x >> 24);
  M.neg = (int)(int8_t)(v.y & 255u);
  M.o1 = (int)(int8_t)((v.y >> 8) & 255u);
  M.o2 = (int)(int8_t)((v.y >> 16) & 255u);
  return M;
}

// f(x) = sum_{a,b} F[a][b] D[x_a][x_b] with F and D symmetric.  For a
// candidate y = x o q that agrees with x outside a position set M (any
// superset of the changed positions), splitting the pairs by membership in M
// gives
//   delta = sum_{a in M} ( 2 G_a + sum_{b in M} F[a][b] S_ab ),
//   G_a   = sum_b F[a][b] (D[y_a][x_b] - D[x_a][x_b]) = H[a][y_a] - H[a][x_a],
//   S_ab  = D[y_a][y_b] - D[y_a][x_b] - D[x_a][y_b] + D[x_a][x_b]   (S_ab = S_ba),
// with DX[v][c] = D[v][x_c] and H[a][v] = sum_b F[a][b] DX[v][b] kept for the
// current solution x (a move changes the columns of DX in its range, and H by
// F times the column differences), and D[y_a][y_b] = DX[y_a][q_b].  The pair
// sum runs over unordered pairs.  H entries lie in [0, n max F max D]: 16-bit
// storage when that is below 2^16 (HT = uint16_t), else 32-bit.  When the
// sums can leave int32 (wide entries), H is not kept: G_a is the row product
// <F row a, DX row y_a> minus R_a = <F row a, DX row x_a> in 64-bit arithmetic.
template <class HT>
struct QapK {
  static constexpr int ENC = 0;
  static constexpr bool kOneLaneObjective = false;   // the wave computes a solution's objective
  uint16_t *cur, *nxt;
  int n, np;             // np: n rounded up to 8 (row stride of F and DX)
  const int16_t *F;      // F[a][b] at a * np + b, zero for b >= n
  int16_t *DX;           // D[v][x_c] at v * np + c, zero for c >= n
  HT *H;                 // H[a][v] at a * n + v (int32 sums)
  long long *R;          // R_a (64-bit sums), in the space of H
  const int16_t *Dg;     // D in global memory (n x n)
  // this wave's round: the candidates' maps and deltas, per-window candidate
  // segments (first entry | count << 16), first entry of each rank, and the
  // entry lists (candidate; byte offsets 2a | 2q_a << 8 of position a)
  uint2 *maps;
  long long *dsum;
  uint32_t *seg, *rb;
  uint8_t *tv;
  uint16_t *ent;
  bool sums32;           // 2 n max F max D < 2^31: H, G and the pair sums fit int32

  // <F row a, DX row v> over np columns
  template <class ACC>
  __device__ __forceinline__ ACC row_dot(int a, int v) const {
    const uint4 *fa = (const uint4 *)(F + a * np), *dv = (const uint4 *)(DX + v * np);
    ACC acc = 0;
#pragma unroll 2
    for (int i = 0; i < (np >> 3); ++i) {
      const uint4 f = fa[i], d = dv[i];
      int s = sizeof(ACC) == 4 ? (int)acc : 0;   // 8 products < 2^31 for entries < 2^14
      s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.x), __builtin_bit_cast(s16x2, d.x), s, false);
      s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.y), __builtin_bit_cast(s16x2, d.y), s, false);
      s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.z), __builtin_bit_cast(s16x2, d.z), s, false);
      s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.w), __builtin_bit_cast(s16x2, d.w), s, false);
      if constexpr (sizeof(ACC) == 4) acc = s;
      else acc += s;
    }
    return acc;
  }
  // H (int32 sums) or R (64-bit sums) from F and DX; lane v < n owns column v of H
  __device__ __forceinline__ void build_sums() {
    const int v = (int)lane_id(), wv = (int)(threadIdx.x >> 6);
    if (sums32) {
      if (v < n)
        for (int a = wv; a < n; a += kThreads<KQAP> / kWave) H[a * n + v] = (HT)row_dot<int32_t>(a, v);
    } else if (v < n && wv == 0) {
      R[v] = row_dot<int64_t>(v, cur[v]);
    }
    __syncthreads();
  }
  // F and DX for the current solution, staged through the space of H
  __device__ __forceinline__ void setup(const int16_t *Fg) {
    const int c = (int)lane_id();
    int16_t *tmp = (int16_t *)H;   // holds 2 n^2 bytes (16-padded)
    stage16(tmp, Fg, 2u * n * n);
    __syncthreads();
    if (c < np)
      for (int a = 0; a < n; ++a) ((int16_t *)F)[a * np + c] = c < n ? tmp[a * n + c] : (int16_t)0;
    __syncthreads();
    stage16(tmp, Dg, 2u * n * n);
    __syncthreads();
    if (c < np) {
      const int xc = c < n ? cur[c] : 0;
      for (int v = 0; v < n; ++v) DX[v * np + c] = c < n ? tmp[v * n + xc] : (int16_t)0;
    }
    __syncthreads();
    build_sums();
  }

  template <class ACC>
  __device__ __forceinline__ void entries(uint32_t total) const {
    for (uint32_t e = lane_id(); e < total; e += kWave) {
      const uint32_t t = tv[e], en = ent[e], a = (en & 255u) >> 1, q = en >> 9;
      const uint32_t sg = seg[t], base = sg & 0xFFFFu, cnt = sg >> 16;
      const int ya = cur[q], xa = cur[a];
      const int16_t *Dy = DX + ya * np, *Dx = DX + xa * np, *Fa = F + a * np;
      long long G;
      if constexpr (sizeof(ACC) == 4) G = (long long)((int)H[a * n + ya] - (int)H[a * n + xa]);
      else G = row_dot<int64_t>((int)a, ya) - R[a];
      // diagonal term, then the pairs (e, e + s) for s = 1 .. (cnt - 1) / 2
      // around the candidate's entries, plus the opposite entry once when
      // cnt is even
      ACC c1 = (ACC)Fa[a] * (ACC)(Dy[q] - 2 * Dy[a] + Dx[a]), c2 = 0;
      const uint32_t i = e - base, h = (cnt - 1) >> 1;
      const uint32_t steps = h + ((cnt & 1) == 0 && 2 * i < cnt ? 1u : 0u);
      // four pairs per pass, so that their reads are in flight together; a
      // pass past the last pair reads entries of the candidate and adds nothing
      // (entries hold byte offsets into the int16 rows)
      const char *Fab = (const char *)Fa, *Dyb = (const char *)Dy, *Dxb = (const char *)Dx;
      const uint16_t *ec = ent + base;
      uint32_t jj = i;
      for (uint32_t s = 0; s < steps; s += 4) {
        uint32_t eb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          jj = jj + 1 == cnt ? 0u : jj + 1;
          eb[u] = ec[jj];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {   // loads on every lane, masked sum (no branch around them)
          const uint32_t ob = eb[u] & 255u, oq = eb[u] >> 8;
          const int S = *(const int16_t *)(Dyb + oq) - *(const int16_t *)(Dyb + ob) - *(const int16_t *)(Dxb + oq) +
                        *(const int16_t *)(Dxb + ob);
          c2 += (ACC)((*(const int16_t *)(Fab + ob) * S) & -(int)(s + u < steps));
        }
      }
      atomicAdd((unsigned long long *)&dsum[t], (unsigned long long)(2 * G + (long long)c1 + 2 * (long long)c2));
    }
  }
  // Deltas of the 64 candidates of a round (one per lane, k = 0 for an empty
  // lane), collective over this wave alone (the two waves of the workgroup
  // evaluate one round each, on their own lists): the (candidate, position)
  // entries of all lanes are listed and shared, so the work follows the total
  // number of changed positions rather than the largest one in the wave.
  // Candidates with more changed positions are listed first, so that the
  // entries processed together belong to candidates with similar pair
  // counts; a round with more entries than the list holds is processed in
  // windows of whole candidates.
  template <bool X3>
  __device__ __forceinline__ int64_t delta_round(const TspScratch &W, int tl, int k, int64_t) const {
    const uint32_t l = lane_id();
    uint32_t *tmp = (uint32_t *)dsum;
    const uint32_t cap = kQapListPerN * (uint32_t)n;
    uint64_t mask = 0;
    {
      Step st[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) st[m] = load_step<ENC, X3>(W, tl, m);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        SMap M = smap(st[m].op, st[m].a, st[m].b, st[m].c);
        if (m >= k) M.len = 0;   // identity
        maps[3 * l + m] = smap_pack(M);
        mask |= m < k ? step_bits(st[m]) : 0ull;
      }
    }
    const uint32_t cnt = (uint32_t)__popcll(mask);
    const uint32_t cls = cnt >= 24 ? 0u : (cnt >= 12 ? 1u : (cnt >= 6 ? 2u : (cnt >= 3 ? 3u : 4u)));
    uint32_t rank = 0;
#pragma unroll
    for (uint32_t c = 0; c < 5; ++c) {
      const unsigned long long mc = __ballot(cls == c);
      rank += c < cls ? (uint32_t)__popcll(mc) : (c == cls ? lanes_below(mc) : 0u);
    }
    tmp[rank] = cnt;
    wave_sync();
    const uint32_t cr = tmp[l];   // lanes in rank order from here
    uint32_t incl = cr;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(incl, o, kWave);
      incl += l >= (uint32_t)o ? v : 0u;
    }
    rb[l] = incl - cr;
    wave_sync();
    const uint32_t base = rb[rank];
    dsum[l] = 0;
    for (uint32_t r0 = 0; r0 < (uint32_t)kWave;) {
      // the window: ranks r0 .. r1-1, as many whole candidates as the list holds
      const uint32_t wb = uni(__shfl(incl - cr, r0, kWave));
      const unsigned long long mw = __ballot(l >= r0 && incl - wb <= cap);
      const uint32_t r1 = r0 + (uint32_t)__popcll(mw);
      const uint32_t total = uni(__shfl(incl, r1 - 1, kWave)) - wb;
      const bool mine = rank >= r0 && rank < r1;
      if (mine) {
        seg[l] = (base - wb) | cnt << 16;
        uint64_t mm = mask;
        for (uint32_t j = base - wb; mm; ++j) {
          tv[j] = (uint8_t)l;
          ent[j] = (uint16_t)(2 * __builtin_ctzll(mm));
          mm &= mm - 1;
        }
      }
      wave_sync();
      // q_a of every entry through the candidate's maps
      for (uint32_t e = l; e < total; e += kWave) {
        const uint32_t t = tv[e];
        const int a = ent[e] >> 1;
        const SMap M0 = smap_unpack(maps[3 * t]), M1 = smap_unpack(maps[3 * t + 1]), M2 = smap_unpack(maps[3 * t + 2]);
        const int q = sapply(M0, sapply(M1, sapply(M2, a)));
        ent[e] = (uint16_t)(2 * a | (2 * q) << 8);
      }
      wave_sync();
      if (sums32) entries<int32_t>(total);
      else entries<int64_t>(total);
      wave_sync();
      r0 = r1;
    }
    const int64_t d = dsum[l];
    wave_sync();
    return d;
  }
  // Accepted move: the DX columns of the move's range for the new solution,
  // and H[a][v] changed by sum_b F[a][b] (new - old DX[v][b]).
  __device__ __forceinline__ void apply(const Step *st, int k) {
    int lo, hi;
    move_range(st, k, lo, hi);
    perm_apply(cur, nxt, st, k, lo, hi);
    refresh(lo, hi);
  }
  // DX and H after the solution changed on [lo, hi]
  __device__ __forceinline__ void refresh(int lo, int hi) {
    if (lo > hi) return;
    const int v = (int)lane_id();
    const bool w0 = threadIdx.x < (uint32_t)kWave;
    if (sums32) {
      if (v < n && w0) {
        const int16_t *dcol = Dg + v * n;
        for (int b0 = lo & ~7; b0 <= hi; b0 += 8) {
          int nv[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int b = b0 + i;
            nv[i] = (b >= lo && b <= hi) ? dcol[cur[b]] : 0;
          }
          uint32_t dp[4];
#pragma unroll
          for (int i = 0; i < 8; i += 2) {
            int d2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int b = b0 + i + u;
              d2[u] = 0;
              if (b >= lo && b <= hi) {
                d2[u] = nv[i + u] - DX[v * np + b];
                DX[v * np + b] = (int16_t)nv[i + u];
              }
            }
            dp[i >> 1] = (uint32_t)(d2[0] & 0xFFFF) | (uint32_t)d2[1] << 16;
          }
          for (int a = 0; a < n; ++a) {
            const uint4 f = *(const uint4 *)(F + a * np + b0);
            int s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.x), __builtin_bit_cast(s16x2, dp[0]), 0, false);
            s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.y), __builtin_bit_cast(s16x2, dp[1]), s, false);
            s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.z), __builtin_bit_cast(s16x2, dp[2]), s, false);
            s = __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, f.w), __builtin_bit_cast(s16x2, dp[3]), s, false);
            H[a * n + v] = (HT)((int)H[a * n + v] + s);
          }
        }
      }
      __syncthreads();
    } else {
      if (v < n && w0) {
        const int16_t *dcol = Dg + v * n;
        for (int b = lo; b <= hi; ++b) DX[v * np + b] = dcol[cur[b]];
      }
      __syncthreads();
      build_sums();
    }
  }
  // objective of the solution with entries y (LNS candidates): the wave's sum
  __device__ __forceinline__ int64_t objective_of(const uint16_t *y) const {
    int64_t acc = 0;
    for (int a = (int)lane_id(); a < n; a += kWave) {
      const int16_t *Fa = F + a * np, *Dr = Dg + (int)y[a] * n;
      for (int b = 0; b < n; ++b) acc += (int64_t)Fa[b] * Dr[y[b]];
    }
    return wave_sum64(acc);
  }
  __device__ __forceinline__ void store(int32_t *dst) const { perm_store(cur, n, dst); }
};

// Byte-field counts of one lane: operator o (relative to the encoding's first
// operator) at bits 8o of cu/cv, k at bits 8(k-1) of cuk/cvk.
template <int ENC, bool W64>
__device__ __forceinline__ void credit_bytes(OpCount<W64> &cu, OpCount<W64> &cv, uint32_t &cuk, uint32_t &cvk,
                                             const Step *st, int k, bool imp) {
  constexpr int lo = enc_lo<ENC>();
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const OpCount<W64> inc = m < k ? (OpCount<W64>)1 << ((st[m].op - lo) << 3) : (OpCount<W64>)0;
    cu += inc;
    cv += imp ? inc : (OpCount<W64>)0;
  }
  const uint32_t inck = 1u << ((k - 1) << 3);
  cuk += inck;
  cvk += imp ? inck : 0u;
}

template <bool X3, class KD>
__device__ __forceinline__ void run_gens(KD &kd, const TspScratch &W, const Uni &U, int32_t *best_row, uint32_t sol,
                                         uint32_t g0, uint32_t g1, uint64_t &T, int64_t &f, int64_t &bf, LStats &S,
                                         uint32_t &nacc) {
  constexpr int ENC = KD::ENC;
  constexpr int lo = enc_lo<ENC>();
  constexpr int nf = ENC == 0 ? (X3 ? kPermOps : 4) : 2;
  const uint32_t lane = lane_id();
  // per-lane byte counts (a chunk adds at most 6 to a field of a lane),
  // folded into the wave-uniform counts of S every 42 chunks and at the end
  OpCount<X3> cu = 0, cv = 0;
  uint32_t cuk = 0, cvk = 0, since_fold = 0;
  bool best_is_cur = false;   // the best-so-far solution is the current one, not yet written
  for (uint32_t g = g0; g < g1; ++g) {
    unsigned long long bk = ~0ull;
    for (uint32_t c0 = 0; c0 < U.C; c0 += kChunk) {
      const uint32_t cn = min((uint32_t)kChunk, U.C - c0);
      int kk[2];
      draw_chunk<ENC, X3>(W, U, g, sol, c0, cn, kk);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const uint32_t tl = r * kWave + lane;
        const bool valid = tl < cn;
        if (valid) {
          Step st[3];
          st[0] = load_step<ENC, X3>(W, (int)tl, 0);
          st[1] = kk[r] > 1 ? load_step<ENC, X3>(W, (int)tl, 1) : st[0];
          st[2] = kk[r] > 2 ? load_step<ENC, X3>(W, (int)tl, 2) : st[0];
          const int64_t d = kd.delta(st, kk[r], f);
          if (U.credit == 0) credit_bytes<ENC, X3>(cu, cv, cuk, cvk, st, kk[r], d < 0);
          const unsigned long long key = ((unsigned long long)(d + kDeltaBias) << 16) | (c0 + tl);
          bk = key < bk ? key : bk;
        }
      }
      if (++since_fold == 42) {
        fold_ops<X3>(S.u + lo, S.v + lo, cu, cv, nf);
        fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
        cu = cv = 0;
        cuk = cvk = 0;
        since_fold = 0;
      }
      __syncthreads();
    }
    bk = wave_min_key(bk);
    const uint32_t ts = (uint32_t)(bk & 0xFFFFu);
    const int64_t ds = (int64_t)(bk >> 16) - kDeltaBias;
    bool acc = ds <= 0;
    if (!acc) acc = accept_worse(ds, T, g, sol, U);
    if (acc) {
      Step st[3];
      const int k = sample<ENC, X3>(U, g, sol, ts, st);
      if (U.credit == 1) credit<ENC>(S, st, k, ds < 0);   // the same on every lane
      if (best_is_cur && f + ds >= bf) {
        kd.store(best_row);
        best_is_cur = false;
      }
      kd.apply(st, k);
      f += ds;
      ++nacc;
      if (f < bf) {
        bf = f;
        best_is_cur = true;
      }
    }
    T = cool(T, U.alpha);
  }
  if (best_is_cur) kd.store(best_row);
  fold_ops<X3>(S.u + lo, S.v + lo, cu, cv, nf);
  fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
}

// Generations of a kind evaluated round by round (QAP, VRPTW): the workgroup's two
// waves each draw and evaluate one round of 64 candidates of every chunk,
// then agree on the chunk minimum through LDS; acceptance and the move are
// the same on both (the move's shared state is written by wave 0 or
// identically by both).  Each wave counts its own candidates; the accepted
// count is wave 0's.
template <bool X3, bool LNS, class KD>
__device__ __forceinline__ void round_gens(KD &kd, const TspScratch &W, const Uni &U, int32_t *best_row, uint32_t sol,
                                           uint32_t g0, uint32_t g1, uint64_t &T, int64_t &f, int64_t &bf, LStats &S,
                                           uint32_t &nacc, unsigned long long *xk, const LnsCtx &lx) {
  constexpr int ENC = (KD::ENC == 0 && LNS) ? 4 : KD::ENC;
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  // 3-opt and the eight operators of the multi-row and LNS encodings count in 64 bits
  constexpr bool W64 = X3 || ENC >= 3;
  constexpr int nf = ENC >= 3 ? 8 : (X3 ? kPermOps : 4);
  OpCount<W64> cu = 0, cv = 0;
  uint32_t cuk = 0, cvk = 0, since_fold = 0;
  bool best_is_cur = false;   // the best-so-far solution is the current one, not yet written
  for (uint32_t g = g0; g < g1; ++g) {
    unsigned long long bk = ~0ull;
    for (uint32_t c0 = 0; c0 < U.C; c0 += kChunk) {
      const uint32_t cn = min((uint32_t)kChunk, U.C - c0);
      int kk[1];
      draw_chunk<ENC, X3, 1>(W, U, g, sol, c0, cn, kk, wv);
      const uint32_t tl = wv * kWave + lane;
      const bool valid = tl < cn;
      if (__ballot(valid)) {
        const int k = valid ? kk[0] : 0;
        int64_t d = kd.template delta_round<X3>(W, (int)tl, k, f);
        if constexpr (LNS) {   // candidates with an LNS step: their entries by the whole wave
          const unsigned long long mk = __ballot(valid && lns_drawn(W.sop(), tl, k));
          if constexpr (KD::kOneLaneObjective) {   // the splits of a batch side by side
            int64_t fn = f + d;
            lns_batched<X3>(U, g, sol, c0 + wv * kWave, mk, kd.n, kd.cur, lx, fn,
                            [&](const uint16_t *y) { return kd.objective_of(y); });
            d = fn - f;
          } else {
            for (unsigned long long m = mk; m; m &= m - 1) {
              const uint32_t t = (uint32_t)__builtin_ctzll(m);
              const int64_t fn = lns_eval<X3>(U, g, sol, c0 + wv * kWave + t, kd.n, kd.cur, lx,
                                              [&](const uint16_t *y) { return kd.objective_of(y); });
              if (lane == t) d = fn - f;
            }
          }
        }
        if (valid) {
          if (U.credit == 0) {   // the steps again from the tables: fewer registers live across the round
            Step st[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) st[m].op = (int)(W.sop()[3 * tl + m] & 7u);
            credit_bytes<ENC, W64>(cu, cv, cuk, cvk, st, k, d < 0);
          }
          const unsigned long long key = ((unsigned long long)(d + kDeltaBias) << 16) | (c0 + tl);
          bk = key < bk ? key : bk;
        }
      }
      if (++since_fold == 84) {   // one candidate per lane per chunk: at most 3 per field
        fold_ops<W64>(S.u, S.v, cu, cv, nf);
        fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
        cu = cv = 0;
        cuk = cvk = 0;
        since_fold = 0;
      }
      __syncthreads();
    }
    xk[wv] = wave_min_key(bk);
    __syncthreads();
    bk = xk[0] < xk[1] ? xk[0] : xk[1];
    const uint32_t ts = (uint32_t)(bk & 0xFFFFu);
    const int64_t ds = (int64_t)(bk >> 16) - kDeltaBias;
    bool acc = ds <= 0;
    if (!acc) acc = accept_worse(ds, T, g, sol, U);
    if (acc) {
      Step st[3];
      const int k = sample<ENC, X3>(U, g, sol, ts, st);
      if (U.credit == 1 && wv == 0) credit<ENC>(S, st, k, ds < 0);   // the same on every lane of wave 0
      if (best_is_cur && f + ds >= bf) {   // wave 0 reads the solution before the move's first barrier
        if (wv == 0) kd.store(best_row);
        best_is_cur = false;
      }
      if constexpr (LNS) {
        if (lns_in(st, k)) {
          int lo, hi;
          lns_apply<X3>(U, g, sol, ts, st, k, kd.n, kd.cur, kd.nxt, lx, lo, hi);
          kd.refresh(lo, hi);
        } else {
          kd.apply(st, k);
        }
      } else {
        kd.apply(st, k);
      }
      f += ds;
      nacc += wv == 0;
      if (f < bf) {
        bf = f;
        best_is_cur = true;
      }
    }
    T = cool(T, U.alpha);
  }
  if (best_is_cur && wv == 0) kd.store(best_row);
  fold_ops<W64>(S.u, S.v, cu, cv, nf);
  fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
}

// Generations of a VRPTW solution in the lexicographic mode (Alg. 1 with the
// comparisons of that mode), two waves per solution: each wave draws and
// evaluates one 64-candidate round of every chunk (one candidate per lane)
// and writes the candidates' objective vectors to LDS; then both waves scan
// the chunk's vectors in index order and keep the first candidate that no
// later one is strictly better than (the comparison has tolerances and is not
// transitive, so the scan runs in order; both waves reach the same winner).
// A winner that the current solution does not beat is accepted; a worse one
// passes the exponential test on lex_delta.  A candidate improves when it is
// strictly better than the current solution.  The scalar f reported for a
// solution is its penalty plus its first level.  Counts as in round_gens:
// each wave its own candidates, accepted moves and credit R2 on wave 0.
template <bool X3, bool LNS, class KD>
__device__ __forceinline__ void lex_rounds(KD &kd, const TspScratch &W, const Uni &U, const LexCfg &L,
                                           int32_t *best_row, uint32_t sol, uint32_t g0, uint32_t g1, uint64_t &T,
                                           int64_t &f, int64_t &bf, Vec4 &cv, Vec4 &bsv, LStats &S, uint32_t &nacc,
                                           int64_t *vbuf, const LnsCtx &lx) {
  constexpr int ENC = (KD::ENC == 0 && LNS) ? 4 : KD::ENC;
  constexpr bool W64 = X3 || ENC >= 3;
  constexpr int nf = ENC >= 3 ? 8 : (X3 ? kPermOps : 4);
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  OpCount<W64> cu = 0, cvc = 0;
  uint32_t cuk = 0, cvk = 0, since_fold = 0;
  bool best_is_cur = false;   // the best-so-far solution is the current one, not yet written
  for (uint32_t g = g0; g < g1; ++g) {
    Vec4 bv = {};
    uint32_t bt = 0;
    bool have = false;
    for (uint32_t c0 = 0; c0 < U.C; c0 += kChunk) {
      const uint32_t cn = min((uint32_t)kChunk, U.C - c0);
      int kk[1];
      draw_chunk<ENC, X3, 1>(W, U, g, sol, c0, cn, kk, wv);
      const uint32_t tl = wv * kWave + lane;
      Step st[3];
      Vec4 v = {};
      if (tl < cn) {
        st[0] = load_step<ENC, X3>(W, (int)tl, 0);
        st[1] = kk[0] > 1 ? load_step<ENC, X3>(W, (int)tl, 1) : st[0];
        st[2] = kk[0] > 2 ? load_step<ENC, X3>(W, (int)tl, 2) : st[0];
        v = lex_vector(kd.parts(st, kk[0]), kd.veh, L);
      }
      if constexpr (LNS) {   // candidates with an LNS step: their splits side by side, by batches
        const unsigned long long mk = __ballot(tl < cn && lns_drawn(W.sop(), tl, kk[0]));
        lns_batched<X3>(U, g, sol, c0 + wv * kWave, mk, kd.n, kd.cur, lx, v,
                        [&](const uint16_t *y) { return lex_vector(kd.parts_of(y), kd.veh, L); });
      }
      if (tl < cn) {
        if (U.credit == 0) credit_bytes<ENC, W64>(cu, cvc, cuk, cvk, st, kk[0], lex_better(v, cv, L));
        store_vec(vbuf + 4 * (size_t)tl, v);
      }
      __syncthreads();
      for (uint32_t j = 0; j < cn; ++j) {
        const Vec4 x = load_vec(vbuf + 4 * (size_t)j);
        if (!have || lex_better(x, bv, L)) {
          bv = x;
          bt = c0 + j;
          have = true;
        }
      }
      if (++since_fold == 84) {   // one candidate per lane per chunk: at most 3 per field
        fold_ops<W64>(S.u, S.v, cu, cvc, nf);
        fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
        cu = cvc = 0;
        cuk = cvk = 0;
        since_fold = 0;
      }
      __syncthreads();
    }
    bool acc = !lex_better(cv, bv, L);
    if (!acc) acc = accept_worse(lex_delta(bv, cv, L), T, g, sol, U);
    if (acc) {
      Step st[3];
      const int k = sample<ENC, X3>(U, g, sol, bt, st);
      if (U.credit == 1 && wv == 0) credit<ENC>(S, st, k, lex_better(bv, cv, L));
      const bool new_best = lex_better(bv, bsv, L);
      if (best_is_cur && !new_best) {   // wave 0 reads the solution before the move's first barrier
        if (wv == 0) kd.store(best_row);
        best_is_cur = false;
      }
      if constexpr (LNS) {
        if (lns_in(st, k)) {
          int lo, hi;
          lns_apply<X3>(U, g, sol, bt, st, k, kd.n, kd.cur, kd.nxt, lx, lo, hi);
        } else {
          kd.apply(st, k);
        }
      } else {
        kd.apply(st, k);
      }
      cv = bv;
      f = bv.v[0] + bv.v[1];
      nacc += wv == 0;
      if (new_best) {
        bsv = cv;
        bf = f;
        best_is_cur = true;
      }
    }
    T = cool(T, U.alpha);
  }
  if (best_is_cur && wv == 0) kd.store(best_row);
  fold_ops<W64>(S.u, S.v, cu, cvc, nf);
  fold_byte_counts(S.uk, S.vk, cuk, cvk, 3);
}

// ------------------------------------------------------------ epoch close
// floor(num / den) for den > 0, exact: a double quotient below 2^24 is within
// 2^-27 of num / den, so its floor is off by at most one and one integer
// correction each way fixes it; larger quotients take the integer division.
__device__ __forceinline__ uint64_t udiv_q24(uint64_t num, uint64_t den) {
  const double qd = (double)num / (double)den;
  if (qd >= 16777216.0) return num / den;
  uint64_t q = (uint64_t)qd;
  if (__umul64hi(q, den) != 0 || q * den > num) --q;
  if (num - q * den >= den) ++q;
  return q;
}

// Eq. ema per enabled operator and per K-step, clamp to [floor, 1], normalise;
// stagnation of the instance best resets the K-step weights (Alg. 2).
// caps: the per-sequence weight caps (null for the K-step group); weight i is
// clamped to [min(floor, cap_i), cap_i]
__device__ __forceinline__ void ema_group(uint32_t *w, const unsigned long long *u, const unsigned long long *v, uint32_t mask,
                          int cnt, uint32_t A, uint32_t FL, const uint32_t *caps) {
  uint64_t s = 0;
  for (int i = 0; i < cnt; ++i) {
    if (!(mask & (1u << i))) continue;
    const uint64_t r = udiv_q24((uint64_t)v[i] << 16, u[i] + 1);
    uint64_t nw = ((uint64_t)A * w[i] + (uint64_t)(65536 - A) * (r + FL)) >> 16;
    nw = nw < FL ? FL : (nw > 65536 ? 65536 : nw);
    // [min(floor, cap), cap]: the clamp above, then at most the cap
    if (caps && nw > caps[i]) nw = caps[i];
    w[i] = (uint32_t)nw;
    s += nw;
  }
  for (int i = 0; i < cnt; ++i) {
    if (!(mask & (1u << i))) continue;
    const uint64_t nw = udiv_q24((uint64_t)w[i] << 16, s);
    w[i] = (uint32_t)(nw < 1 ? 1 : nw);
  }
}

// Per-launch counts of one workgroup, added into the accumulator row of its
// solution (row sol mod kShards): slots [0, kOps) uses and [kOps, 2 kOps)
// improvements per operator, the next 3 uses and 3 improvements per k, then
// accepted moves, and the row minimum of the workgroup's best objective in
// slot kCountSlots.  S holds
// per-lane counts (summed here over the wave) or, with UNIFORM, counts that
// are already wave totals.  The atomics need no fence: the epoch kernel reads
// the rows after the kernel boundary.
constexpr int kCountSlots = 2 * kOps + 7;   // uses, improvements per operator and per k, accepted

template <int ENC, bool UNIFORM>
__device__ __forceinline__ void write_counts(DevJob *J, uint32_t sol, const LStats &S, uint32_t nacc, int64_t bf) {
  constexpr int lo = enc_lo<ENC>(), hi = enc_hi<ENC>();
  const uint32_t lane = lane_id();
  uint32_t mine = 0;
#pragma unroll
  for (int o = lo; o <= hi; ++o) {
    const uint32_t u = UNIFORM ? S.u[o] : wave_sum(S.u[o]);
    const uint32_t v = UNIFORM ? S.v[o] : wave_sum(S.v[o]);
    mine = lane == (uint32_t)o ? u : mine;
    mine = lane == (uint32_t)(kOps + o) ? v : mine;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint32_t uk = UNIFORM ? S.uk[q] : wave_sum(S.uk[q]);
    const uint32_t vk = UNIFORM ? S.vk[q] : wave_sum(S.vk[q]);
    mine = lane == (uint32_t)(2 * kOps + q) ? uk : mine;
    mine = lane == (uint32_t)(2 * kOps + 3 + q) ? vk : mine;
  }
  mine = lane == (uint32_t)(2 * kOps + 6) ? nacc : mine;
  unsigned long long *row = J->shard + (size_t)(sol & (kShards - 1)) * kEpochSlots;
  if (lane < (uint32_t)kCountSlots && mine) atomicAdd(&row[lane], (unsigned long long)mine);
  if (lane == (uint32_t)kCountSlots) atomicMin((long long *)&row[kCountSlots], (long long)bf);
}

}  // namespace

// ------------------------------------------------------------ islands
// Island model and elite injection (paper, Sec. "Island Model and Elite
// Injection") at the end of epoch e, by the epoch kernel's workgroup (16 waves
// for jobs that migrate): island i holds solutions [i S, (i+1) S); elites
// (best-so-far solutions) replace the worst current solutions of the
// receiving islands, every source and target chosen before the first copy
// (ring: island i's best to island i+1; top-N: the population's N best to
// every island; hybrid: ring when e / interval is odd, top-N when even); then
// elite injection puts the population's best in place of its worst.  best =
// smallest (best f, index), worst = largest (current f, index).  Sources are
// staged in the job's pool rows (free after the initialisation).  Per-island
// choices are spread over the waves; copies over every thread of the group.
constexpr int kMaxIslands = 64, kMaxMigN = 8, kEpochWide = 1024;

__device__ __forceinline__ bool listed(const int *l, int cnt, int v) {
  bool in = false;
  for (int i = 0; i < cnt; ++i) in |= l[i] == v;
  return in;
}

// Pick keys: smaller (value key, index key) is preferred; MIN: smallest
// (v, s), else largest (v, s).
// The values are read eight strides at a time (independent loads in flight
// together: the scan is bound by memory latency, not bandwidth).
template <bool MIN>
__device__ __forceinline__ void pick_scan(const int64_t *v, int lo, int hi, const int *ex, int nex, int first,
                                          int stride, unsigned long long &bk, uint32_t &bs) {
  constexpr unsigned long long kSign = 1ull << 63;
  constexpr int kB = 8;
  bk = ~0ull;
  bs = 0xFFFFFFFFu;
  for (int s0 = lo + first; s0 < hi; s0 += kB * stride) {
    int64_t x[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) x[u] = s0 + u * stride < hi ? v[s0 + u * stride] : 0;
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int s = s0 + u * stride;
      if (s >= hi || listed(ex, nex, s)) continue;
      const unsigned long long k = MIN ? ((unsigned long long)x[u] ^ kSign) : ~((unsigned long long)x[u] ^ kSign);
      const uint32_t ks = MIN ? (uint32_t)s : ~(uint32_t)s;
      if (k < bk || (k == bk && ks < bs)) {
        bk = k;
        bs = ks;
      }
    }
  }
}

// dst[e] = src(e) for e in [0, total), over every thread of the workgroup,
// four elements per thread in flight (loads first, then stores)
template <class SRC, class DST>
__device__ __forceinline__ void group_copy(int total, const SRC &src, const DST &dst) {
  const int st = (int)blockDim.x;
  for (int e0 = (int)threadIdx.x; e0 < total; e0 += 4 * st) {
    int32_t x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = e0 + u * st < total ? src(e0 + u * st) : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + u * st < total) dst(e0 + u * st, x[u]);
  }
}

// wave-wide lexicographic minimum of (bk, bs); uniform
__device__ __forceinline__ void wave_min_pair(unsigned long long &bk, uint32_t &bs) {
  const unsigned long long m = wave_min_key(bk);
  bs = wave_min_u32(bk == m ? bs : 0xFFFFFFFFu);
  bk = m;
}

// smallest (v[s], s) over [lo, hi) \ ex (MIN) or largest (MIN = false), by one wave
template <bool MIN>
__device__ int wave_pick(const int64_t *v, int lo, int hi, const int *ex, int nex) {
  unsigned long long bk;
  uint32_t bs;
  pick_scan<MIN>(v, lo, hi, ex, nex, (int)lane_id(), kWave, bk, bs);
  wave_min_pair(bk, bs);
  return (int)(MIN ? bs : ~bs);
}

// the same by the whole workgroup (every thread calls it; result uniform)
template <bool MIN>
__device__ int block_pick(const int64_t *v, int lo, int hi, const int *ex, int nex) {
  __shared__ unsigned long long s_k[kEpochWide / kWave];
  __shared__ uint32_t s_s[kEpochWide / kWave];
  const int nw = (int)(blockDim.x / kWave), w = (int)(threadIdx.x / kWave);
  unsigned long long bk;
  uint32_t bs;
  pick_scan<MIN>(v, lo, hi, ex, nex, (int)threadIdx.x, (int)blockDim.x, bk, bs);
  wave_min_pair(bk, bs);
  if (lane_id() == 0) {
    s_k[w] = bk;
    s_s[w] = bs;
  }
  __syncthreads();
  bk = ~0ull;
  bs = 0xFFFFFFFFu;
  for (int i = 0; i < nw; ++i)
    if (s_k[i] < bk || (s_k[i] == bk && s_s[i] < bs)) {
      bk = s_k[i];
      bs = s_s[i];
    }
  __syncthreads();   // s_k, s_s free for the next call
  return (int)(MIN ? bs : ~bs);
}

// Scratch of the migration in the epoch kernel's dynamic LDS (launches that
// may migrate only): per (target, source) pair its target, source vector,
// objective and whether it improves the target's best; per source its solution.
struct MigLds {
  int tgt[kMaxIslands * kMaxMigN];
  int better[kMaxIslands * kMaxMigN];
  long long f[kMaxIslands * kMaxMigN];
  const int32_t *row[kMaxIslands * kMaxMigN];
  int src[kMaxIslands];
  Vec4 v[kMaxIslands * kMaxMigN];   // the source's best vector (lexicographic mode)
};

// Lexicographic mode: the best (best vectors; a later solution replaces the
// one kept when strictly better) or the worst (current vectors; a later one
// replaces the one kept when the kept one is not strictly better than it) of
// [lo, hi) outside ex[0..nex), by an ordered scan; the scalar rules with
// "smaller" replaced by the mode's relation.  Uniform over the calling lanes.
template <bool BEST>
__device__ int lex_pick(const DevJob *J, const LexCfg &L, int lo, int hi, const int *ex, int nex) {
  const int64_t *V = BEST ? J->best_v : J->cur_v;
  int k = -1;
  Vec4 kv = {};
  for (int s = lo; s < hi; ++s) {
    if (listed(ex, nex, s)) continue;
    const Vec4 x = load_vec(V + 4 * (size_t)s);
    const bool take = k < 0 || (BEST ? lex_better(x, kv, L) : !lex_better(x, kv, L));
    if (take) {
      k = s;
      kv = x;
    }
  }
  return k;
}

// Copies for `npairs` (target, source row) pairs in M: target t takes the
// n-vector row as its current solution and objective f, and as its best when
// f is below its best objective (decided for every pair before any copy).
// Targets are distinct and no source row is a target's row.  All threads of
// the workgroup take part.
__device__ void mig_copy(DevJob *J, int n, int npairs, MigLds &M) {
  const bool lex = J->lex_levels != 0;
  for (int q = (int)threadIdx.x; q < npairs; q += (int)blockDim.x)
    M.better[q] = lex ? lex_better(M.v[q], load_vec(J->best_v + 4 * (size_t)M.tgt[q]), lex_cfg(J->inst))
                      : M.f[q] < J->best_f[M.tgt[q]];
  __syncthreads();
  group_copy(
      npairs * n, [&](int e) { return M.row[e / n][e % n]; },
      [&](int e, int32_t x) {
        const int q = e / n, p = e - q * n;
        const size_t o = (size_t)M.tgt[q] * n + p;
        J->cur[o] = x;
        if (M.better[q]) J->best[o] = x;
      });
  for (int q = (int)threadIdx.x; q < npairs; q += (int)blockDim.x) {
    J->cur_f[M.tgt[q]] = M.f[q];
    if (M.better[q]) J->best_f[M.tgt[q]] = M.f[q];
    if (lex) {
      store_vec(J->cur_v + 4 * (size_t)M.tgt[q], M.v[q]);
      if (M.better[q]) store_vec(J->best_v + 4 * (size_t)M.tgt[q], M.v[q]);
    }
  }
  // vectors and objectives visible to the next choice: the workgroup's
  // waves share one CU, so the barrier's workgroup-scope ordering suffices (a
  // device-scope fence here would write the whole L2 back each time)
  __syncthreads();
}

__device__ void migrate_block(DevJob *J, uint32_t e, MigLds &M) {
  const int P = (int)J->P, n = J->inst->n, I = (int)J->islands, S = P / I;
  const int nw = (int)(blockDim.x / kWave), w = (int)(threadIdx.x / kWave);
  const bool lex = J->lex_levels != 0;
  const LexCfg L = lex_cfg(J->inst);
  if (J->mig_epochs && e % J->mig_epochs == 0 && I >= 2) {
    int mode = (int)J->mig_mode;
    if (mode == 2) mode = ((e / J->mig_epochs) & 1) ? 0 : 1;
    const int N = mode == 0 ? 1 : (int)J->mig_n, n_src = mode == 0 ? I : N;
    int chosen[kMaxMigN];
    if (mode == 0) {   // island i's best and island i+1's worst, islands spread over the waves
      for (int i = w; i < I; i += nw) {
        const int j = i + 1 == I ? 0 : i + 1;
        const int src = lex ? lex_pick<true>(J, L, i * S, (i + 1) * S, chosen, 0)
                            : wave_pick<true>(J->best_f, i * S, (i + 1) * S, chosen, 0);
        const int tgt = lex ? lex_pick<false>(J, L, j * S, (j + 1) * S, chosen, 0)
                            : wave_pick<false>(J->cur_f, j * S, (j + 1) * S, chosen, 0);
        if (lane_id() == 0) {
          M.src[i] = src;
          M.tgt[i] = tgt;
        }
      }
    } else {           // the population's N best, then each island's N worst
      for (int k = 0; k < N; ++k) {
        chosen[k] = lex ? lex_pick<true>(J, L, 0, P, chosen, k) : block_pick<true>(J->best_f, 0, P, chosen, k);
        if (threadIdx.x == 0) M.src[k] = chosen[k];
      }
      for (int i = w; i < I; i += nw)
        for (int k = 0; k < N; ++k) {
          chosen[k] = lex ? lex_pick<false>(J, L, i * S, (i + 1) * S, chosen, k)
                          : wave_pick<false>(J->cur_f, i * S, (i + 1) * S, chosen, k);
          if (lane_id() == 0) M.tgt[i * N + k] = chosen[k];
        }
    }
    __syncthreads();
    // sources staged first (pool row k holds source k), then every pair's
    // row and objective: ring pair i takes island i's best, top-N pair i N + k
    // the k-th best
    group_copy(
        n_src * n, [&](int x) { return J->best[(size_t)M.src[x / n] * n + x % n]; },
        [&](int x, int32_t y) { J->pool[x] = y; });
    const int npairs = I * N;
    for (int q = (int)threadIdx.x; q < npairs; q += (int)blockDim.x) {
      const int k = mode == 0 ? q : q % N;
      M.row[q] = J->pool + (size_t)k * n;
      M.f[q] = J->best_f[M.src[k]];
      if (lex) M.v[q] = load_vec(J->best_v + 4 * (size_t)M.src[k]);
    }
    __syncthreads();
    mig_copy(J, n, npairs, M);
  }
  if (J->elite_epochs && e % J->elite_epochs == 0) {
    int none[1];
    const int b = lex ? lex_pick<true>(J, L, 0, P, none, 0) : block_pick<true>(J->best_f, 0, P, none, 0);
    const int wst = lex ? lex_pick<false>(J, L, 0, P, none, 0) : block_pick<false>(J->cur_f, 0, P, none, 0);
    if (wst != b) {
      if (threadIdx.x == 0) {
        M.tgt[0] = wst;
        M.row[0] = J->best + (size_t)b * n;
        M.f[0] = J->best_f[b];
        if (lex) M.v[0] = load_vec(J->best_v + 4 * (size_t)b);
      }
      __syncthreads();
      mig_copy(J, n, 1, M);
    }
  }
}

// Lexicographic mode: the population's best by the ordered scan over the
// solutions' best vectors (index order; a later solution replaces the one
// kept only when strictly better).  Every lane that calls it returns the same
// index.  The vectors are read eight solutions at a time.
__device__ __forceinline__ uint32_t lex_scan_best(const DevJob *J, const LexCfg &L) {
  const uint32_t P = J->P;
  const int64_t *bv = J->best_v;
  Vec4 keep = load_vec(bv);
  uint32_t b = 0;
  constexpr uint32_t kB = 8;
  for (uint32_t s0 = 1; s0 < P; s0 += kB) {
    Vec4 x[kB];
#pragma unroll
    for (uint32_t u = 0; u < kB; ++u) x[u] = s0 + u < P ? load_vec(bv + 4 * (size_t)(s0 + u)) : keep;
#pragma unroll
    for (uint32_t u = 0; u < kB; ++u)
      if (s0 + u < P && lex_better(x[u], keep, L)) {
        keep = x[u];
        b = s0 + u;
      }
  }
  return b;
}

// After each evolve launch: fold the accumulator rows of every job into its
// epoch statistics, the instance best and the temperature, and at an epoch
// boundary apply the AOS update (the kernel boundary orders it after every
// evolve workgroup).  Wave 0 of the job's workgroup, its lanes sharing the
// work as described at epoch_fold.  The launch covered generations [g0, g1).
static_assert(kShards == kWave && kCountSlots < kWave, "one accumulator row and one slot per lane");
// Lanes share the work: lane l sums slot l over the 64 rows (column l) and
// clears it; lane o < kOps then owns operator o and lane 2 kOps + q owns
// k = q + 1 (their statistics, run totals and weights: loads, the Eq. ema
// update with its clamp, the normalisation through a wave sum, stores); the
// scalars are uniform and lane 0 stores them.
// pre (lexicographic mode, launches that migrate): the instance best's vector
// and objective taken before the exchange, which may change best vectors
__device__ __forceinline__ void epoch_fold(DevJob *J, uint32_t g0, uint32_t E, uint32_t g1,
                                           const long long *pre = nullptr) {
  const uint32_t l = threadIdx.x;
  constexpr uint32_t kMinSlot = kCountSlots, kAccSlot = 2 * kOps + 6;
  const bool op_lane = l < (uint32_t)kOps, k_lane = l >= 2u * kOps && l < 2u * kOps + 3;
  const uint32_t q = l - 2 * kOps;   // k lanes
  // this lane's own state first (one batch of loads, no store between)
  uint64_t u = 0, v = 0, tu = 0, tv = 0;
  uint32_t w = 0, cap = 65536;
  if (op_lane) {
    u = J->u_op[l];
    v = J->v_op[l];
    tu = J->tot_u_op[l];
    tv = J->tot_v_op[l];
    w = J->w_op[l];
    cap = J->w_cap[l];
  } else if (k_lane) {
    u = J->u_k[q];
    v = J->v_k[q];
    tu = J->tot_u_k[q];
    tv = J->tot_v_k[q];
    w = J->w_k[q];
  }
  const uint32_t alpha = J->alpha, op_mask = J->op_mask, aos_A = J->aos_A;
  const uint32_t w_floor = J->w_floor, stag_limit = J->stag_limit;
  // per-solution weights: the evolve workgroups update them; the instance
  // statistics and weights stay as initialised
  const bool inst_scope = J->aos_scope == 0;
  const bool lex = J->lex_levels != 0;
  uint32_t stag = J->stag;
  uint64_t T = J->T;
  int64_t inst_best = J->inst_best, epoch_ref = J->epoch_ref;
  const unsigned long long accepted = J->accepted;
  // column l of the accumulator rows, then cleared for the next launch
  unsigned long long *col = J->shard + l;
  unsigned long long c = l == kMinSlot ? (unsigned long long)LLONG_MAX : 0ull;
  if (l <= kMinSlot) {
    constexpr int kB = kShards / 2;   // rows per batch of loads in flight
#pragma unroll
    for (int r0 = 0; r0 < kShards; r0 += kB) {
      unsigned long long x[kB];
#pragma unroll
      for (int r = 0; r < kB; ++r) x[r] = col[(r0 + r) * kEpochSlots];
#pragma unroll
      for (int r = 0; r < kB; ++r)
        col[(r0 + r) * kEpochSlots] = l == kMinSlot ? (unsigned long long)LLONG_MAX : 0ull;
#pragma unroll
      for (int r = 0; r < kB; ++r)
        c = l == kMinSlot ? (unsigned long long)min((long long)c, (long long)x[r]) : c + x[r];
    }
  }
  // the launch's counts where their owners need them
  const uint64_t add_u = c;                                                 // slot l: uses of op l / of k (lane 2 kOps + q)
  const uint64_t add_v = shfl64(c, op_lane ? l + kOps : (k_lane ? l + 3 : l));   // improvements
  const unsigned long long add_acc = shfl64(c, kAccSlot);
  const long long mn = (long long)shfl64(c, kMinSlot);
  if (op_lane || k_lane) {
    if (inst_scope) {
      u += add_u;
      v += add_v;
    }
    tu += add_u;
    tv += add_v;
  }
  if (mn < inst_best) inst_best = mn;
  for (uint32_t g = g0; g < g1; ++g) T = cool(T, alpha);
  if (g1 % E == 0 && inst_scope) {
    // Eq. ema on every enabled operator and on the k weights, clamp, then normalisation per group
    const bool upd = (op_lane && ((op_mask >> l) & 1u)) || k_lane;
    uint64_t nw = 0;
    if (upd) {   // clamped to [min(floor, cap), cap] (an operator's cap; 1.0 for the k weights)
      const uint64_t r = udiv_q24(v << 16, u + 1);
      nw = ((uint64_t)aos_A * w + (uint64_t)(65536 - aos_A) * (r + w_floor)) >> 16;
      const uint64_t lo = min(w_floor, cap);
      nw = nw < lo ? lo : (nw > cap ? cap : nw);
    }
    const uint32_t s_op = wave_sum(op_lane ? (uint32_t)nw : 0u), s_k = wave_sum(k_lane ? (uint32_t)nw : 0u);
    if (upd) {
      const uint64_t z = udiv_q24(nw << 16, op_lane ? s_op : s_k);
      w = (uint32_t)(z < 1 ? 1 : z);
    }
    bool improved = inst_best < epoch_ref;
    int64_t ref_now = inst_best;
    if (lex) {   // the instance best by the ordered scan; improved when strictly better than the last one
      const LexCfg L = lex_cfg(J->inst);
      Vec4 now;
      if (pre) {
        now = load_vec((const int64_t *)pre);
        ref_now = pre[4];
      } else {
        const uint32_t b = lex_scan_best(J, L);
        now = load_vec(J->best_v + 4 * (size_t)b);
        ref_now = J->best_f[b];
      }
      improved = lex_better(now, load_vec(J->ref_v), L);
      if (l == 0) store_vec(J->ref_v, now);
    }
    if (improved) stag = 0;
    else stag += 1;
    epoch_ref = ref_now;
    if (stag >= stag_limit) {
      if (k_lane) w = q == 0 ? 52429u : (q == 1 ? 9830u : 3277u);
      stag = 0;
    }
    u = v = 0;
  }
  if (op_lane) {
    J->u_op[l] = u;
    J->v_op[l] = v;
    J->tot_u_op[l] = tu;
    J->tot_v_op[l] = tv;
    J->w_op[l] = w;
  } else if (k_lane) {
    J->u_k[q] = u;
    J->v_k[q] = v;
    J->tot_u_k[q] = tu;
    J->tot_v_k[q] = tv;
    J->w_k[q] = w;
  }
  if (l == 0) {
    J->accepted = accepted + add_acc;
    J->inst_best = inst_best;
    J->epoch_ref = epoch_ref;
    J->stag = stag;
    J->T = T;
    J->g = g1;
  }
}

__global__ __launch_bounds__(64) void k_epoch(DevJob *jobs, const uint32_t *idx, uint32_t *next, uint32_t n_next) {
  if (blockIdx.x == 0 && threadIdx.x < n_next) next[threadIdx.x] = 0;   // work-item counters of the launch
  DevJob *J = jobs + (idx ? idx[blockIdx.x] : blockIdx.x);
  const uint32_t g0 = J->g, gstop = J->g_stop;
  if (g0 >= gstop) return;
  const uint32_t E = J->E;
  epoch_fold(J, g0, E, min(gstop, (g0 / E + 1) * E));
}

// The epoch kernel of launches in which a job may migrate or inject its elite
// (kEpochWide threads per job, MigLds in dynamic LDS).  The exchange at an
// epoch end comes before the fold; the two touch disjoint state.
__global__ __launch_bounds__(kEpochWide) void k_epoch_mig(DevJob *jobs, const uint32_t *idx, uint32_t *next,
                                                          uint32_t n_next) {
  if (blockIdx.x == 0 && threadIdx.x < n_next) next[threadIdx.x] = 0;
  DevJob *J = jobs + (idx ? idx[blockIdx.x] : blockIdx.x);
  const uint32_t g0 = J->g, gstop = J->g_stop, E = J->E;
  __syncthreads();   // every wave has read g before wave 0 advances it
  if (g0 >= gstop) return;
  const uint32_t g1 = min(gstop, (g0 / E + 1) * E);
  // the lexicographic instance best is taken on the state before the exchange
  __shared__ long long pre[5];
  const bool lex_pre = J->lex_levels != 0 && J->aos_scope == 0 && g1 % E == 0;
  if (lex_pre && threadIdx.x < kWave) {
    const uint32_t b = lex_scan_best(J, lex_cfg(J->inst));
    if (threadIdx.x == 0) {
      store_vec((int64_t *)pre, load_vec(J->best_v + 4 * (size_t)b));
      pre[4] = J->best_f[b];
    }
  }
  __syncthreads();
  if (g1 % E == 0 && (J->mig_epochs | J->elite_epochs)) migrate_block(J, g1 / E, *(MigLds *)gx_lds);
  if (threadIdx.x >= kWave) return;
  epoch_fold(J, g0, E, g1, lex_pre ? pre : nullptr);
}

namespace {

// Weights per solution (aos_scope 1): the workgroup adds its launch's counts
// to its solution's record and, at an epoch end, applies the Eq. ema update,
// clamp, normalisation and stagnation check of Alg. 2 to the solution's own
// weights, with its own best objective in place of the instance best.  S
// holds this wave's totals; two waves add theirs through LDS first.
template <int NT>
__device__ __forceinline__ void solution_aos_close(DevJob *J, uint32_t sol, LStats S, int64_t bf, uint32_t g1,
                                                   uint32_t E) {
  constexpr int NW = (int)(sizeof(LStats) / 4);
  uint32_t *sw = (uint32_t *)&S;
  if constexpr (NT > kWave) {
    __syncthreads();   // the candidate tables are dead: wave 1's counts go there
    uint32_t *X = (uint32_t *)gx_lds;
    if (threadIdx.x == kWave)
#pragma unroll
      for (int i = 0; i < NW; ++i) X[i] = sw[i];
    __syncthreads();
    if (threadIdx.x < kWave)
#pragma unroll
      for (int i = 0; i < NW; ++i) sw[i] += X[i];
    __syncthreads();
  }
  if (threadIdx.x >= kWave) return;
  SolAos *A = J->saos + sol;
  unsigned long long u[kOps], v[kOps], uk[3], vk[3];
  uint32_t w[kOps], wk[3];
#pragma unroll
  for (int o = 0; o < kOps; ++o) {
    u[o] = A->u_op[o] + S.u[o];
    v[o] = A->v_op[o] + S.v[o];
    w[o] = A->w_op[o];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    uk[q] = A->u_k[q] + S.uk[q];
    vk[q] = A->v_k[q] + S.vk[q];
    wk[q] = A->w_k[q];
  }
  uint32_t stag = A->stag;
  int64_t ref = A->epoch_ref;
  if (g1 % E == 0) {
    ema_group(w, u, v, J->op_mask, kOps, J->aos_A, J->w_floor, J->w_cap);
    ema_group(wk, uk, vk, 7u, 3, J->aos_A, J->w_floor, nullptr);
    stag = bf < ref ? 0u : stag + 1;
    ref = bf;
    if (stag >= J->stag_limit) {
      wk[0] = 52429; wk[1] = 9830; wk[2] = 3277;
      stag = 0;
    }
#pragma unroll
    for (int o = 0; o < kOps; ++o) u[o] = v[o] = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) uk[q] = vk[q] = 0;
  }
  if (lane_id() != 0) return;
#pragma unroll
  for (int o = 0; o < kOps; ++o) {
    A->u_op[o] = (uint32_t)u[o];
    A->v_op[o] = (uint32_t)v[o];
    A->w_op[o] = w[o];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    A->u_k[q] = (uint32_t)uk[q];
    A->v_k[q] = (uint32_t)vk[q];
    A->w_k[q] = wk[q];
  }
  A->stag = stag;
  A->epoch_ref = ref;
}

// ------------------------------------------------------------ one workgroup
template <int KIND, int VAR>
__device__ __forceinline__ void evolve_wg(DevJob *J, uint32_t sol, char *lds) {
  constexpr int STAGE = VAR & 7;
  constexpr bool x3 = (VAR & kVarX3) != 0;   // 3-opt in the operator set
  const uint32_t g0 = uni(J->g), gstop = uni(J->g_stop);
  if (g0 >= gstop) return;
  const uint32_t E = J->E;
  const uint32_t g1 = min(gstop, (g0 / E + 1) * E);
  const DevInst *I = J->inst;
  const int n = I->n;
  constexpr bool rows = (VAR & kVarRows) != 0;   // multi-row VRPTW
  Uni U;
  U.n = (uint32_t)(rows ? n - 1 : n);   // the multi-row form keeps its final marker in place
  U.C = J->C;
  U.key = J->key;
  U.k0 = (uint32_t)J->seed;
  U.k1 = (uint32_t)(J->seed >> 32);
  U.credit = J->credit;
  U.alpha = J->alpha;
  U.lb = I->lb;
  U.ub = I->ub;
  // the operator and K-step weights of the instance, or of this solution
  const bool sol_scope = J->aos_scope != 0;
  const uint32_t *wsrc = sol_scope ? J->saos[sol].w_op : J->w_op;
  const uint32_t *wksrc = sol_scope ? J->saos[sol].w_k : J->w_k;
  // cumulative weights of the encoding's operators (the others weigh 0): one
  // bound per operator but the last, which only adds to the total
  constexpr bool lnsv = (VAR & kVarLns) != 0;   // LNS operators in the operator set
  constexpr int ENC = KIND == KKNAP ? 1 : (KIND == KCOLOR ? 2 : (rows ? 3 : (lnsv ? 4 : 0)));
  constexpr int lo = enc_lo<ENC>(), span = enc_hi<ENC>() - lo;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < span; ++i) {
    c += wsrc[lo + i];
    U.cw[i] = c;
  }
  U.sw = c + wsrc[enc_hi<ENC>()];
  U.ck[0] = wksrc[0];
  U.ck[1] = wksrc[0] + wksrc[1];
  U.swk = U.ck[1] + wksrc[2];

  // LNS scratch of this wave (wide variants of single-row permutations)
  LnsCtx lx{nullptr, nullptr, nullptr, 0};
  if constexpr (lnsv) {
    char *lb = lds + lds_core_bytes(KIND, n, VAR, I->rows) + (threadIdx.x >> 6) * lns_wave_bytes(KIND, n);
    lx.hkey = J->sums;
    lx.tabs = (LnsTab *)lb;
    lx.y = (uint16_t *)(lb + 3 * sizeof(LnsTab));
    lx.stride = (int)(((2u * n + 15u) & ~15u) / 2u);
  }
  uint64_t T = J->T;
  int64_t f = J->cur_f[sol], bf = J->best_f[sol];
  LStats S = {};
  uint32_t nacc = 0;
  const uint32_t lane = lane_id();
  int32_t *cur_g = J->cur + (size_t)sol * n;
  int32_t *best_row = J->best + (size_t)sol * n;
  // LDS: candidate tables first, then the solution and the instance data
  const TspScratch W;
  char *const base = lds + (x3 ? kTablesX3 : kTables);

  if constexpr (KIND == KTSP || KIND == KQAP || KIND == KVRP) {
    // one tour buffer; the move application writes through the candidate
    // tables (kOneBufferN entries) or, for longer tours, a second buffer
    uint16_t *t0 = (uint16_t *)base;
    uint16_t *t1 = n <= kOneBufferN ? (uint16_t *)lds : (uint16_t *)(base + al16(2 * n));
    char *rest = base + (n <= kOneBufferN ? 1 : 2) * al16(2 * n);
    for (int p = lane; p < n; p += kWave) t0[p] = (uint16_t)cur_g[p];
    if constexpr (KIND == KTSP) {
      if constexpr (STAGE == SLDS16) {
        stage16(rest, I->d16, 2u * n * n);
        __syncthreads();
        if constexpr (x3) tsp_run<true, lnsv>(t0, t1, nullptr, n, DistL16{(const int16_t *)rest, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
        else tsp_run<false, false>(t0, t1, nullptr, n, DistL16{(const int16_t *)rest, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
      } else if constexpr (STAGE == SLDSXY) {
        short2 *xy = (short2 *)rest;
        uint16_t *el = (uint16_t *)(rest + al16(4 * n));
        for (int p = lane; p < n; p += kWave) xy[p] = make_short2((short)I->xy[2 * p], (short)I->xy[2 * p + 1]);
        __syncthreads();
        if constexpr (x3) tsp_run<true, lnsv>(t0, t1, el, n, DistXY{xy}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
        else tsp_run<false, false>(t0, t1, el, n, DistXY{xy}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
      } else if constexpr (STAGE == SGLB16) {
        __syncthreads();
        if constexpr (x3) tsp_run<true, lnsv>(t0, t1, nullptr, n, DistG16{I->d16, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
        else tsp_run<false, false>(t0, t1, nullptr, n, DistG16{I->d16, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
      } else {
        __syncthreads();
        if constexpr (x3) tsp_run<true, lnsv>(t0, t1, nullptr, n, DistG32{I->d32, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
        else tsp_run<false, false>(t0, t1, nullptr, n, DistG32{I->d32, n}, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, lx);
      }
      perm_store(t0, n, cur_g);
    } else if constexpr (KIND == KQAP) {
      // F and DX rows padded to 8, then H (2 or 4 n^2 bytes: 16-bit entries
      // for STAGE 1), the chunk minima of the two waves, wave 1's maps, and
      // per wave: deltas, window segments, first entry of each rank, entry
      // lists.  Wave 0's maps sit in the candidate tables (free during rounds).
      using HT = typename std::conditional<STAGE == 1, uint16_t, int32_t>::type;
      const int np = (n + 7) & ~7;
      const uint32_t wv = threadIdx.x >> 6;
      int16_t *F = (int16_t *)rest;
      int16_t *DX = (int16_t *)(rest + al16(2 * n * np));
      char *sums = rest + 2 * al16(2 * n * np);
      unsigned long long *xk = (unsigned long long *)(sums + al16((uint32_t)sizeof(HT) * n * n));
      uint2 *maps1 = (uint2 *)(xk + 2);
      const uint32_t per_wave = 8 * kWave + 8 * kWave + al16(kQapListPerN * n) + al16(2 * kQapListPerN * n);
      char *mine = (char *)(maps1 + 3 * kWave) + wv * per_wave;
      long long *dsum = (long long *)mine;
      uint32_t *seg = (uint32_t *)(mine + 8 * kWave);
      uint32_t *rbk = seg + kWave;
      uint8_t *tv = (uint8_t *)(rbk + kWave);
      uint16_t *ent = (uint16_t *)((char *)tv + al16(kQapListPerN * n));
      uint2 *maps = wv == 0 ? (uint2 *)(lds + 2048) : maps1;
      QapK<HT> kd{t0, t1, n, np, F, DX, (HT *)sums, (long long *)sums, I->qd, maps, dsum, seg, rbk, tv, ent,
                  I->qap_sums32 != 0};
      __syncthreads();
      kd.setup(I->qf);
      if constexpr (x3) round_gens<true, lnsv>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, xk, lx);
      else round_gens<false, false>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, xk, lx);
      if (wv == 0) perm_store(kd.cur, n, cur_g);
    } else {
      // int16 distances, the per-node (demand, ready, due) records, the two
      // waves' chunk minima, and in the lexicographic mode the chunk's
      // candidate vectors
      const int dn = I->dn;   // depot and customers
      int16_t *D = (int16_t *)rest;
      int4 *attr = (int4 *)(rest + al16(2 * dn * dn));
      unsigned long long *xk = (unsigned long long *)(attr + dn);
      stage16(D, I->d16, 2u * dn * dn);
      for (int c = (int)threadIdx.x; c < dn; c += kThreads<KIND, VAR>)
        attr[c] = make_int4(I->dem[c], I->rdy[c], I->due[c], 0);
      __syncthreads();
      VrpK<rows> kd{t0, t1, n, dn, I->capacity, I->vehicles, I->service, I->horizon, D, attr, I, dn - 1};
      if constexpr ((VAR & kVarLex) != 0) {
        const LexCfg L = lex_cfg(I);
        Vec4 cv = load_vec(J->cur_v + 4 * (size_t)sol), bsv = load_vec(J->best_v + 4 * (size_t)sol);
        lex_rounds<x3, lnsv>(kd, W, U, L, best_row, sol, g0, g1, T, f, bf, cv, bsv, S, nacc, (int64_t *)(xk + 2), lx);
        if (threadIdx.x == 0) {
          store_vec(J->cur_v + 4 * (size_t)sol, cv);
          store_vec(J->best_v + 4 * (size_t)sol, bsv);
        }
      } else if constexpr (x3) {
        round_gens<true, lnsv>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, xk, lx);
      } else {
        round_gens<false, false>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc, xk, lx);
      }
      if (threadIdx.x < kWave) perm_store(kd.cur, n, cur_g);
    }
  } else if constexpr (KIND == KKNAP) {
    uint8_t *bits = (uint8_t *)base;
    int32_t *w = (int32_t *)(base + al16(n));
    int32_t *v = w + al16(4 * n) / 4;
    int64_t pw = 0, pv = 0;
    for (int p = lane; p < n; p += kWave) {
      const int b = cur_g[p];
      bits[p] = (uint8_t)b;
      pw += b ? I->kw[p] : 0;
      pv += b ? I->kv[p] : 0;
    }
    stage16(w, I->kw, 4u * n);
    stage16(v, I->kv, 4u * n);
    const int64_t Wsum = wave_sum64(pw), Vsum = wave_sum64(pv);
    __syncthreads();
    KnapK kd{bits, w, v, n, (int64_t)uni64((uint64_t)Wsum), (int64_t)uni64((uint64_t)Vsum), I->capacity, I->lambda};
    run_gens<false>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc);
    kd.store(cur_g);
  } else {
    int16_t *val = (int16_t *)base;
    int32_t *off = (int32_t *)(base + al16(2 * n));
    int32_t *adj = off + al16(4 * (n + 1)) / 4;
    for (int p = lane; p < n; p += kWave) val[p] = (int16_t)cur_g[p];
    stage16(off, I->adj_off, 4u * (n + 1));
    stage16(adj, I->adj, 8u * I->n_edges);
    __syncthreads();
    ColorK kd{val, off, adj, n};
    run_gens<false>(kd, W, U, best_row, sol, g0, g1, T, f, bf, S, nacc);
    kd.store(cur_g);
  }
  if (threadIdx.x == 0) {
    J->cur_f[sol] = f;
    J->best_f[sol] = bf;
  }
  if (sol_scope) solution_aos_close<kThreads<KIND, VAR>>(J, sol, S, bf, g1, E);
  write_counts<ENC, true>(J, sol, S, nacc, bf);   // every wave adds the counts of its own candidates
}

}  // namespace

// ------------------------------------------------------------ evolve kernels
// The TSP kernels are held to 96 VGPRs (5 waves per SIMD): their scalar state
// exceeds the SGPR file and part of it lives in VGPR lanes; the compiler's
// own choice (about 100 VGPRs, 4 waves) runs slower.  The LNS variant takes
// 128 (4 waves): at 96 it spills most of its wave-wide evaluation path.
template <int KIND, int VAR>
__global__ __launch_bounds__((kThreads<KIND, VAR>)) __attribute__((amdgpu_waves_per_eu(KIND == KTSP ? ((VAR & kVarLns) ? 4 : 5) : 1))) void k_evolve(
    DevJob *job) {
  evolve_wg<KIND, VAR>(job, blockIdx.x, gx_lds);
}

// Persistent walk over the (job, solution) work items of one (kind, staging)
// group of many jobs: each workgroup takes the next item from the group's
// counter until the list is done, so workgroups that finish early take more.
// The epoch kernel clears the counter after the launch.
template <int KIND, int VAR>
__global__ __launch_bounds__((kThreads<KIND, VAR>)) __attribute__((amdgpu_waves_per_eu(3))) void k_evolve_group(DevJob *jobs, const uint2 *items, uint32_t n_items,
                                                                 uint32_t *next) {
  for (;;) {
    uint32_t it = 0;
    if (threadIdx.x == 0) it = atomicAdd(next, 1u);
    if constexpr (kThreads<KIND, VAR> > kWave) {   // to every wave of the workgroup (LDS is dead between items)
      if (threadIdx.x == 0) *(volatile uint32_t *)gx_lds = it;
      __syncthreads();
      it = *(volatile uint32_t *)gx_lds;
      __syncthreads();
    }
    it = uni(it);
    if (it >= n_items) break;
    const uint2 w = items[it];
    evolve_wg<KIND, VAR>(jobs + w.x, w.y, gx_lds);
    __syncthreads();
  }
}

// ------------------------------------------------------------ initialisation
namespace {

__device__ __forceinline__ int glb_tsp_dist(const DevInst *I, int a, int b) {
  const int n = I->n;
  if (I->d16) return I->d16[a * n + b];
  if (I->d32) return I->d32[a * n + b];
  const int2 *xy = (const int2 *)I->xy;
  return nint_dist(xy[a], xy[b]);
}

__device__ VrpParts vrp_parts_of(const DevInst *I, const int32_t *x);

// full objective of one solution, by its definition (initial pool only)
__device__ int64_t full_objective(const DevInst *I, const int32_t *x) {
  const int n = I->n;
  if (I->kind == KTSP) {
    int64_t f = 0;
    for (int i = 0; i < n; ++i) f += glb_tsp_dist(I, x[i], x[i + 1 == n ? 0 : i + 1]);
    return f;
  }
  if (I->kind == KQAP) {
    int64_t f = 0;
    for (int i = 0; i < n; ++i) {
      const int16_t *Fi = I->qf + i * n, *Dr = I->qd + x[i] * n;
      for (int j = 0; j < n; ++j) f += (int64_t)Fi[j] * Dr[x[j]];
    }
    return f;
  }
  if (I->kind == KKNAP) {
    int64_t W = 0, V = 0;
    for (int i = 0; i < n; ++i)
      if (x[i]) {
        W += I->kw[i];
        V += I->kv[i];
      }
    const int64_t over = W - I->capacity;
    return -V + I->lambda * (over > 0 ? over : 0);
  }
  if (I->kind == KVRP) return vrp_objective(I, vrp_parts_of(I, x));
  int64_t f = 0;
  for (int e = 0; e < I->n_edges; ++e) f += x[I->edges[2 * e]] == x[I->edges[2 * e + 1]];
  return f;
}

// parts of a VRPTW solution's objective, from the instance's global arrays
__device__ VrpParts vrp_parts_of(const DevInst *I, const int32_t *x) {
  const int n = I->n;
  if (I->rows) {   // rows closed by markers, each a route from the depot and back
    const int dn = I->dn, nc = dn - 1;
    int64_t dist = 0, late = 0, over = 0;
    int t = 0, load = 0, routes = 0, prev = 0, len = 0, longest = 0;
    for (int p = 0; p < n; ++p) {
      const int e = x[p];
      if (e < nc) {
        const int c = e + 1, dd = I->d16[prev * dn + c];
        dist += dd;
        len += dd;
        t = max(t + dd, I->rdy[c]);
        late += max(0, t - I->due[c]);
        t += I->service;
        load += I->dem[c];
        prev = c;
        continue;
      }
      if (prev != 0) {
        const int back = I->d16[prev * dn];
        dist += back;
        late += max(0, t + back - I->horizon);
        longest = max(longest, len + back);
        over += max(0, load - I->capacity);
        ++routes;
      }
      t = load = len = prev = 0;
    }
    return VrpParts{dist, late, routes, longest, over};
  }
  {
    const int dn = I->dn;
    int64_t dist = 0, late = 0;
    int t = 0, load = 0, routes = 0, prev = 0, len = 0, longest = 0;
    for (int p = 0; p < n; ++p) {
      const int c = x[p] + 1;
      if (routes == 0 || load + I->dem[c] > I->capacity) {
        if (routes > 0) {
          const int back = I->d16[prev * dn];
          dist += back;
          t += back;
          late += max(0, t - I->horizon);
          longest = max(longest, len + back);
        }
        ++routes;
        load = 0;
        t = 0;
        prev = 0;
        len = 0;
      }
      const int dd = I->d16[prev * dn + c];
      dist += dd;
      len += dd;
      t = max(t + dd, I->rdy[c]);
      late += max(0, t - I->due[c]);
      t += I->service;
      load += I->dem[c];
      prev = c;
    }
    if (routes > 0) {
      const int back = I->d16[prev * dn];
      dist += back;
      t += back;
      late += max(0, t - I->horizon);
      longest = max(longest, len + back);
    }
    return VrpParts{dist, late, routes, longest, 0};
  }
}

__device__ __forceinline__ int heur_mats(int kind) {
  return kind == KQAP ? 2 : ((kind == KTSP || kind == KVRP) ? 1 : 0);
}
// pool slots the heuristic solutions take: four per data matrix, or the one
// sweep solution of the multi-row form
__device__ __forceinline__ uint32_t heur_slots(const DevInst *I) {
  return I->rows ? 1u : 4u * (uint32_t)heur_mats(I->kind);
}

// sweep order of customer nodes a and b about the depot: polar angle
// counter-clockwise from the positive x axis (the half-plane dy > 0 or
// (dy = 0, dx >= 0) first, then the sign of the cross product), then squared
// distance, then index -- all exact in integers
__device__ __forceinline__ bool sweep_before(const int2 *xy, int a, int b) {
  const int64_t ax = xy[a].x - xy[0].x, ay = xy[a].y - xy[0].y, bx = xy[b].x - xy[0].x, by = xy[b].y - xy[0].y;
  const int ha = (ay < 0 || (ay == 0 && ax < 0)), hb = (by < 0 || (by == 0 && bx < 0));
  if (ha != hb) return ha < hb;
  const int64_t cr = ax * by - ay * bx;
  if (cr != 0) return cr > 0;
  const int64_t da = ax * ax + ay * ay, db = bx * bx + by * by;
  if (da != db) return da < db;
  return a < b;
}
// window order within a row: due time, then ready time, then index
__device__ __forceinline__ bool window_before(const DevInst *I, int a, int b) {
  if (I->due[a] != I->due[b]) return I->due[a] < I->due[b];
  if (I->rdy[a] != I->rdy[b]) return I->rdy[a] < I->rdy[b];
  return a < b;
}

// Initial solution of the multi-row form (Sec. "Partition Encoding Heuristic
// Initialization": customers grouped by place, routes ordered by time
// window), read as a sweep: customers in sweep order fill the rows in turn, a
// row closing when the next demand would take its load above the capacity
// (the last row takes the rest); each row is ordered by window_before and
// closed by its marker nc + r.  One workgroup per job; the job's heuristic-sum
// scratch holds the sweep order, each customer's row and the row offsets.
__device__ void sweep_rows(DevJob *J, const DevInst *I, int32_t *out) {
  const int nc = I->dn - 1, R = I->rows;
  const int2 *xy = (const int2 *)I->xy;
  int32_t *ord = (int32_t *)J->sums, *row = ord + nc, *off = row + nc + 1;
  for (int c = 1 + (int)threadIdx.x; c <= nc; c += blockDim.x) {
    int rank = 0;
    for (int b = 1; b <= nc; ++b) rank += sweep_before(xy, b, c);
    ord[rank] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int r = 0, load = 0, cnt = 0;
    for (int i = 0; i < nc; ++i) {
      const int c = ord[i];
      if (load + I->dem[c] > I->capacity && r < R - 1) {
        off[r++] = cnt;
        cnt = 0;
        load = 0;
      }
      row[c] = r;
      load += I->dem[c];
      ++cnt;
    }
    off[r] = cnt;
    for (int q = r + 1; q < R; ++q) off[q] = 0;
    // counts -> first entry of each row (customers of the earlier rows plus their markers)
    int at = 0;
    for (int q = 0; q < R; ++q) {
      const int k = off[q];
      off[q] = at;
      at += k + 1;
      out[at - 1] = nc + q;
    }
  }
  __syncthreads();
  for (int c = 1 + (int)threadIdx.x; c <= nc; c += blockDim.x) {
    const int r = row[c];
    int rank = 0;
    for (int b = 1; b <= nc; ++b) rank += (row[b] == r) && window_before(I, b, c);
    out[off[r] + rank] = c - 1;
  }
}

// entry (i, j) of heuristic data matrix `mat` (Sec. heuristic init: any n x n data matrix)
__device__ __forceinline__ int64_t heur_entry(const DevInst *I, int mat, int i, int j) {
  if (I->kind == KTSP) return glb_tsp_dist(I, i, j);
  if (I->kind == KQAP) return mat == 0 ? I->qf[i * I->n + j] : I->qd[i * I->n + j];
  return I->d16[(i + 1) * I->dn + (j + 1)];
}

}  // namespace

// row / column sums of each data matrix, sorted ascending and descending
// (ties by index) -> four permutations per matrix in pool slots 4*mat ..
__global__ __launch_bounds__(256) void k_init_heur(DevJob *jobs) {
  DevJob *J = jobs + blockIdx.x;
  const DevInst *I = J->inst;
  const int mat = blockIdx.y;
  if (I->rows) {
    if (mat == 0 && J->Q > 0) sweep_rows(J, I, J->pool);
    return;
  }
  if (mat >= heur_mats(I->kind)) return;
  const int base = 4 * mat;
  if ((uint32_t)base >= J->Q) return;
  const int n = I->n;
  int64_t *rs = J->sums + (size_t)mat * 2 * n, *cs = rs + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    int64_t r = 0, c = 0;
    for (int j = 0; j < n; ++j) {
      r += heur_entry(I, mat, i, j);
      c += heur_entry(I, mat, j, i);
    }
    rs[i] = r;
    cs[i] = c;
  }
  __syncthreads();
  for (int h = 0; h < 4; ++h) {
    if ((uint32_t)(base + h) >= J->Q) break;
    const int64_t *s = h < 2 ? rs : cs;
    const int64_t sg = (h & 1) ? -1 : 1;
    int32_t *row = J->pool + (size_t)(base + h) * n;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const int64_t ki = sg * s[i];
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const int64_t kj = sg * s[j];
        rank += (kj < ki) || (kj == ki && j < i);
      }
      row[rank] = i;
    }
  }
}

// random members of the pool: Fisher-Yates from the identity (multi-row
// form: over the entries before the final marker), random bits, or uniform
// integers; draw i comes from word (i mod 4) of the block with counter
// (0xFFFFFFFF, pool index, i / 4, instance key)
__global__ __launch_bounds__(64) void k_init_random(DevJob *jobs) {
  DevJob *J = jobs + blockIdx.y;
  const DevInst *I = J->inst;
  const uint32_t q = blockIdx.x * 64 + threadIdx.x;
  const uint32_t H = min(heur_slots(I), J->Q);
  if (q < H || q >= J->Q) return;
  const int n = I->n;
  int32_t *x = J->pool + (size_t)q * n;
  const uint32_t k0 = (uint32_t)J->seed, k1 = (uint32_t)(J->seed >> 32);
  uint32_t r[4];
  if (I->kind == KKNAP || I->kind == KCOLOR) {
    for (int i = 0; i < n; ++i) {
      if ((i & 3) == 0) philox(0xFFFFFFFFu, q, (uint32_t)(i >> 2), J->key, k0, k1, r);
      const uint32_t w = r[i & 3];
      x[i] = I->kind == KKNAP ? (int32_t)(w >> 31) : I->lb + (int32_t)rmap(w, (uint32_t)(I->ub - I->lb + 1));
    }
  } else {
    // the multi-row form shuffles the entries before its final marker
    const int m = I->rows ? n - 1 : n;
    for (int i = 0; i < n; ++i) x[i] = i;
    for (int i = m - 1; i >= 1; --i) {
      if (i == m - 1 || (i & 3) == 3) philox(0xFFFFFFFFu, q, (uint32_t)(i >> 2), J->key, k0, k1, r);
      const uint32_t j = rmap(r[i & 3], (uint32_t)(i + 1));
      const int32_t t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
}

__global__ __launch_bounds__(64) void k_init_eval(DevJob *jobs) {
  DevJob *J = jobs + blockIdx.y;
  const uint32_t q = blockIdx.x * 64 + threadIdx.x;
  if (q >= J->Q) return;
  const int32_t *x = J->pool + (size_t)q * J->inst->n;
  if (J->lex_levels) {   // the vector, and as the scalar its penalty plus its first level
    const Vec4 v = lex_vector(vrp_parts_of(J->inst, x), J->inst->vehicles, lex_cfg(J->inst));
    store_vec(J->pool_v + 4 * (size_t)q, v);
    J->pool_f[q] = v.v[0] + v.v[1];
    return;
  }
  J->pool_f[q] = full_objective(J->inst, x);
}

// vector a before vector b, level by level without tolerances (a total order)
__device__ __forceinline__ int vec_cmp(const Vec4 &a, const Vec4 &b) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (a.v[i] != b.v[i]) return a.v[i] < b.v[i] ? -1 : 1;
  return 0;
}

// keep the P best of the pool, ordered by (f, pool index), or in the
// lexicographic mode by (vector, pool index)
__global__ __launch_bounds__(64) void k_init_select(DevJob *jobs) {
  DevJob *J = jobs + blockIdx.y;
  const uint32_t q = blockIdx.x * 64 + threadIdx.x;
  if (q >= J->Q) return;
  const int64_t fq = J->pool_f[q];
  uint32_t rank = 0;
  if (J->lex_levels) {
    const Vec4 vq = load_vec(J->pool_v + 4 * (size_t)q);
    for (uint32_t o = 0; o < J->Q; ++o) {
      const int c = vec_cmp(load_vec(J->pool_v + 4 * (size_t)o), vq);
      rank += c < 0 || (c == 0 && o < q);
    }
  } else {
    for (uint32_t o = 0; o < J->Q; ++o) {
      const int64_t fo = J->pool_f[o];
      rank += (fo < fq) || (fo == fq && o < q);
    }
  }
  if (rank >= J->P) return;
  if (J->lex_levels) {
    const Vec4 vq = load_vec(J->pool_v + 4 * (size_t)q);
    store_vec(J->cur_v + 4 * (size_t)rank, vq);
    store_vec(J->best_v + 4 * (size_t)rank, vq);
  }
  const int n = J->inst->n;
  const int32_t *src = J->pool + (size_t)q * n;
  int32_t *c = J->cur + (size_t)rank * n, *b = J->best + (size_t)rank * n;
  for (int i = 0; i < n; ++i) {
    c[i] = src[i];
    b[i] = src[i];
  }
  J->cur_f[rank] = fq;
  J->best_f[rank] = fq;
}

// initial temperature, weights (Tab. weight_preset) and counters
__global__ void k_init_final(DevJob *jobs, int count) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  DevJob *J = jobs + j;
  const int n = J->inst->n;
  const int64_t f0 = J->cur_f[0];
  if (J->t0_param) J->T = J->t0_param;
  else {
    const uint64_t a = (uint64_t)(f0 < 0 ? -f0 : f0);
    J->T = ((a << 16) / (uint64_t)n) >> 2;
  }
  uint64_t raw[kOps], s = 0;
  for (int i = 0; i < kOps; ++i) {
    raw[i] = 0;
    if (!(J->op_mask & (1u << i))) continue;
    raw[i] = 65536;
    if (i == OOROPT) raw[i] = n <= 100 ? 52429 : (n <= 250 ? 45875 : 19661);
    if (i == O3OPT) raw[i] = n <= 100 ? 32768 : (n <= 250 ? 19661 : 3277);
    if (J->lns_cap && ((kLnsMask >> i) & 1u)) raw[i] = n <= 100 ? 393 : (n <= 250 ? 262 : 66);
    if (J->init_w[i]) raw[i] = J->init_w[i];
    s += raw[i];
  }
  for (int i = 0; i < kOps; ++i) {
    if (!raw[i]) {
      J->w_op[i] = 0;
      continue;
    }
    const uint64_t v = (raw[i] << 16) / s;
    J->w_op[i] = (uint32_t)(v < 1 ? 1 : v);
  }
  J->w_k[0] = 52429; J->w_k[1] = 9830; J->w_k[2] = 3277;
  for (int r = 0; r < kShards; ++r) {
    for (int i = 0; i < kCountSlots; ++i) J->shard[r * kEpochSlots + i] = 0;
    J->shard[r * kEpochSlots + kCountSlots] = (unsigned long long)LLONG_MAX;
  }
  for (int i = 0; i < kOps; ++i) J->u_op[i] = J->v_op[i] = 0;
  for (int i = 0; i < 3; ++i) J->u_k[i] = J->v_k[i] = 0;
  for (int i = 0; i < kOps; ++i) J->tot_u_op[i] = J->tot_v_op[i] = 0;
  for (int i = 0; i < 3; ++i) J->tot_u_k[i] = J->tot_v_k[i] = 0;
  if (J->aos_scope)   // every solution starts from the instance's initial weights and its own objective
    for (uint32_t sol = 0; sol < J->P; ++sol) {
      SolAos *A = J->saos + sol;
      for (int i = 0; i < kOps; ++i) A->w_op[i] = J->w_op[i], A->u_op[i] = A->v_op[i] = 0;
      for (int i = 0; i < 3; ++i) A->w_k[i] = J->w_k[i], A->u_k[i] = A->v_k[i] = 0;
      A->stag = 0;
      A->epoch_ref = J->best_f[sol];
    }
  J->g = 0;
  J->g_stop = 0;
  J->stag = 0;
  J->done = 0;
  J->accepted = 0;
  J->epoch_ref = f0;
  J->inst_best = f0;
  if (J->lex_levels)
    for (int i = 0; i < 4; ++i) J->ref_v[i] = J->cur_v[i];
}

__global__ void k_set_stop(DevJob *jobs, int count, uint32_t add, int use_total) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  DevJob *J = jobs + j;
  J->g_stop = use_total ? J->G : J->g_stop + add;
}

// best solution of each job: min of (best_f, index), or in the
// lexicographic mode the ordered scan over the best vectors
__global__ __launch_bounds__(64) void k_best(DevJob *jobs) {
  DevJob *J = jobs + blockIdx.x;
  const uint32_t lane = threadIdx.x;
  int64_t bf = INT64_MAX;
  uint32_t bi = 0xFFFFFFFFu;
  if (J->lex_levels) {
    bi = lex_scan_best(J, lex_cfg(J->inst));
    bf = J->best_f[bi];
  } else {
    for (uint32_t s = lane; s < J->P; s += 64) {
      const int64_t f = J->best_f[s];
      if (f < bf) {
        bf = f;
        bi = s;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t of = __shfl_xor(bf, o, 64);
      const uint32_t oi = __shfl_xor(bi, o, 64);
      if (of < bf || (of == bf && oi < bi)) {
        bf = of;
        bi = oi;
      }
    }
  }
  const int n = J->inst->n;
  const int32_t *src = J->best + (size_t)bi * n;
  for (int p = lane; p < n; p += 64) J->best_out[p] = src[p];
  if (lane == 0) {
    J->best_out_f = bf;
    J->best_idx = (int32_t)bi;
  }
}

__global__ void k_build_d16(const int32_t *xy, int n, int16_t *d16) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int2 *p = (const int2 *)xy;
  d16[idx] = (int16_t)nint_dist(p[i], p[j]);
}

__global__ void k_build_d32(const int32_t *xy, int n, int32_t *d32) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx % n);
  const int2 *p = (const int2 *)xy;
  d32[idx] = nint_dist(p[i], p[j]);
}

// Device arithmetic on given inputs, for comparison with independent
// implementations: what 1 = both Philox forms (the per-lane one with a
// uniform key, and the general one), 2 = nearest-integer distance (int16 and
// int32 coordinate paths), 3 = acceptance threshold.
__global__ __launch_bounds__(64) void k_check(int what, uint64_t key, const uint64_t *in, uint64_t *out,
                                              int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= count) return;
  if (what == 1) {
    const uint64_t a = in[2 * i], b = in[2 * i + 1];
    const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    uint32_t r[4], s[4];
    philox_lane((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32), k0, k1, r);
    philox((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32), k0, k1, s);
    out[4 * i] = r[0] | (uint64_t)r[1] << 32;
    out[4 * i + 1] = r[2] | (uint64_t)r[3] << 32;
    out[4 * i + 2] = s[0] | (uint64_t)s[1] << 32;
    out[4 * i + 3] = s[2] | (uint64_t)s[3] << 32;
  } else if (what == 2) {
    const uint64_t v = in[i];
    const int x1 = (int)(v & 0xFFFF), y1 = (int)((v >> 16) & 0xFFFF), x2 = (int)((v >> 32) & 0xFFFF),
              y2 = (int)(v >> 48);
    out[2 * i] = (uint64_t)nint_dist(make_short2((short)x1, (short)y1), make_short2((short)x2, (short)y2));
    out[2 * i + 1] = (uint64_t)nint_dist(make_int2(x1, y1), make_int2(x2, y2));
  } else {
    out[i] = (uint64_t)accept_threshold(in[2 * i], in[2 * i + 1]);
  }
}

// a job record written from the kernel argument (no host copy)
__global__ void k_write_job(DevJob *dst, DevJob src) { *dst = src; }
__global__ void k_copy_i64(int64_t *dst, const int64_t *src) { *dst = *src; }

// ------------------------------------------------------------ launch wrappers
namespace gxk {

hipError_t write_job(DevJob *dst, const DevJob &src, hipStream_t s) {
  hipLaunchKernelGGL(k_write_job, dim3(1), dim3(1), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t copy_i64(int64_t *dst, const int64_t *src, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t device_check(int what, uint64_t key, const uint64_t *in, uint64_t *out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, s, what, key, in, out, count);
  return hipGetLastError();
}

hipError_t set_exp_tables(const uint32_t *hi, const uint32_t *lo) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_exp_hi), hi, 16 * sizeof(uint32_t));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_exp_lo), lo, 256 * sizeof(uint32_t));
}

hipError_t build_tsp_d16_from_xy(const int32_t *xy, int n, int16_t *d16, hipStream_t s) {
  const int64_t tot = (int64_t)n * n;
  hipLaunchKernelGGL(k_build_d16, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xy, n, d16);
  return hipGetLastError();
}

hipError_t build_d32_from_xy(const int32_t *xy, int n, int32_t *d32, hipStream_t s) {
  const int64_t tot = (int64_t)n * n;
  hipLaunchKernelGGL(k_build_d32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xy, n, d32);
  return hipGetLastError();
}

hipError_t init_jobs(DevJob *jobs, int count, uint32_t max_q, int, int max_heur_mats, hipStream_t s) {
  if (max_heur_mats > 0)
    hipLaunchKernelGGL(k_init_heur, dim3(count, max_heur_mats), dim3(256), 0, s, jobs);
  const dim3 g((max_q + 63) / 64, count);
  hipLaunchKernelGGL(k_init_random, g, dim3(64), 0, s, jobs);
  hipLaunchKernelGGL(k_init_eval, g, dim3(64), 0, s, jobs);
  hipLaunchKernelGGL(k_init_select, g, dim3(64), 0, s, jobs);
  hipLaunchKernelGGL(k_init_final, dim3((count + 63) / 64), dim3(64), 0, s, jobs, count);
  return hipGetLastError();
}

hipError_t set_stop(DevJob *jobs, int count, uint32_t add, int use_total, hipStream_t s) {
  hipLaunchKernelGGL(k_set_stop, dim3((count + 63) / 64), dim3(64), 0, s, jobs, count, add, use_total);
  return hipGetLastError();
}

// the kernel of a (kind, variant): variant = staging | kVarX3 (3-opt) | kVarLex (VRPTW lexicographic)
// | kVarRows (VRPTW multi-row) | kVarLns (LNS operators; always with kVarX3)
#define GX_KERNEL_OF(KERNEL)                                                                 \
  static const void *KERNEL##_of(int kind, int var) {                                      \
    const bool x3 = (var & kVarX3) != 0;                                                     \
    if (var & kVarLns) switch (kind) {                                                       \
        case KTSP:                                                                           \
          switch (var & 7) {                                                                 \
            case SLDS16: return (const void *)KERNEL<KTSP, SLDS16 | kVarX3 | kVarLns>;       \
            case SLDSXY: return (const void *)KERNEL<KTSP, SLDSXY | kVarX3 | kVarLns>;       \
            case SGLB16: return (const void *)KERNEL<KTSP, SGLB16 | kVarX3 | kVarLns>;       \
            default: return (const void *)KERNEL<KTSP, SGLB32 | kVarX3 | kVarLns>;           \
          }                                                                                  \
        case KQAP:                                                                           \
          if ((var & 7) == 1) return (const void *)KERNEL<KQAP, 1 | kVarX3 | kVarLns>;       \
          return (const void *)KERNEL<KQAP, kVarX3 | kVarLns>;                               \
        default:                                                                             \
          if (var & kVarLex) return (const void *)KERNEL<KVRP, kVarLex | kVarX3 | kVarLns>;  \
          return (const void *)KERNEL<KVRP, kVarX3 | kVarLns>;                               \
      }                                                                                      \
    switch (kind) {                                                                          \
      case KTSP:                                                                             \
        switch (var & 7) {                                                                   \
          case SLDS16: return x3 ? (const void *)KERNEL<KTSP, SLDS16 | kVarX3> : (const void *)KERNEL<KTSP, SLDS16>; \
          case SLDSXY: return x3 ? (const void *)KERNEL<KTSP, SLDSXY | kVarX3> : (const void *)KERNEL<KTSP, SLDSXY>; \
          case SGLB16: return x3 ? (const void *)KERNEL<KTSP, SGLB16 | kVarX3> : (const void *)KERNEL<KTSP, SGLB16>; \
          default: return x3 ? (const void *)KERNEL<KTSP, SGLB32 | kVarX3> : (const void *)KERNEL<KTSP, SGLB32>;    \
        }                                                                                    \
      case KQAP:                                                                             \
        if ((var & 7) == 1) return x3 ? (const void *)KERNEL<KQAP, 1 | kVarX3> : (const void *)KERNEL<KQAP, 1>;    \
        return x3 ? (const void *)KERNEL<KQAP, kVarX3> : (const void *)KERNEL<KQAP, 0>;   \
      case KKNAP: return (const void *)KERNEL<KKNAP, 0>;                                     \
      case KVRP:                                                                             \
        if (var & kVarRows) {                                                                \
          if (var & kVarLex)                                                                 \
            return x3 ? (const void *)KERNEL<KVRP, kVarRows | kVarLex | kVarX3>              \
                      : (const void *)KERNEL<KVRP, kVarRows | kVarLex>;                      \
          return x3 ? (const void *)KERNEL<KVRP, kVarRows | kVarX3> : (const void *)KERNEL<KVRP, kVarRows>; \
        }                                                                                    \
        if (var & kVarLex) return x3 ? (const void *)KERNEL<KVRP, kVarLex | kVarX3> : (const void *)KERNEL<KVRP, kVarLex>; \
        return x3 ? (const void *)KERNEL<KVRP, kVarX3> : (const void *)KERNEL<KVRP, 0>;   \
      default: return (const void *)KERNEL<KCOLOR, 0>;                                      \
    }                                                                                        \
  }
GX_KERNEL_OF(k_evolve)
GX_KERNEL_OF(k_evolve_group)
#undef GX_KERNEL_OF

static const void *plain_kernel(int kind, int var) { return k_evolve_of(kind, var); }
static const void *group_kernel(int kind, int var) { return k_evolve_group_of(kind, var); }

hipError_t prepare_kernel_attrs(uint32_t max_lds) {
  const int kinds[][2] = {{KTSP, SLDS16},          {KTSP, SLDSXY},          {KTSP, SGLB16},
                          {KTSP, SGLB32},          {KQAP, 0},               {KQAP, 1},
                          {KKNAP, 0},              {KVRP, 0},               {KCOLOR, 0},
                          {KTSP, SLDS16 | kVarX3}, {KTSP, SLDSXY | kVarX3}, {KTSP, SGLB16 | kVarX3},
                          {KTSP, SGLB32 | kVarX3}, {KQAP, kVarX3},          {KQAP, 1 | kVarX3},
                          {KVRP, kVarX3},          {KVRP, kVarLex},         {KVRP, kVarLex | kVarX3},
                          {KVRP, kVarRows},        {KVRP, kVarRows | kVarX3},
                          {KVRP, kVarRows | kVarLex}, {KVRP, kVarRows | kVarLex | kVarX3},
                          {KTSP, SLDS16 | kVarX3 | kVarLns}, {KTSP, SLDSXY | kVarX3 | kVarLns},
                          {KTSP, SGLB16 | kVarX3 | kVarLns}, {KTSP, SGLB32 | kVarX3 | kVarLns},
                          {KQAP, kVarX3 | kVarLns}, {KQAP, 1 | kVarX3 | kVarLns},
                          {KVRP, kVarX3 | kVarLns}, {KVRP, kVarLex | kVarX3 | kVarLns}};
  for (auto &k : kinds) {
    hipError_t e = hipFuncSetAttribute(plain_kernel(k[0], k[1]), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)max_lds);
    if (e != hipSuccess) return e;
  }
  for (auto &k : kinds) {
    hipError_t e = hipFuncSetAttribute(group_kernel(k[0], k[1]), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)max_lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int threads_of(int kind, int) { return (kind == KQAP || kind == KVRP) ? 2 * kWave : kWave; }

hipError_t evolve_plain(DevJob *job, int kind, int stage, uint32_t P, uint32_t lds, hipStream_t s) {
  void *args[] = {&job};
  return hipLaunchKernel(plain_kernel(kind, stage), dim3(P), dim3(threads_of(kind, stage)), args, lds, s);
}

hipError_t evolve_group(int kind, int stage, DevJob *jobs, const uint2 *items, uint32_t n_items, uint32_t *next,
                        uint32_t grid, uint32_t lds, hipStream_t s) {
  void *args[] = {&jobs, &items, &n_items, &next};
  return hipLaunchKernel(group_kernel(kind, stage), dim3(grid), dim3(threads_of(kind, stage)), args, lds, s);
}

hipError_t epoch(DevJob *jobs, const uint32_t *idx, uint32_t count, uint32_t *next, uint32_t n_next, bool mig,
                 hipStream_t s) {
  if (mig)
    hipLaunchKernelGGL(k_epoch_mig, dim3(count), dim3(kEpochWide), sizeof(MigLds), s, jobs, idx, next, n_next);
  else
    hipLaunchKernelGGL(k_epoch, dim3(count), dim3(64), 0, s, jobs, idx, next, n_next);
  return hipGetLastError();
}

hipError_t fetch_best(DevJob *jobs, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_best, dim3(count), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

hipError_t occupancy_group(int kind, int stage, uint32_t lds, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, group_kernel(kind, stage), threads_of(kind, stage), lds);
}

hipError_t occupancy_plain(int kind, int stage, uint32_t lds, int *blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, plain_kernel(kind, stage), threads_of(kind, stage), lds);
}

}  // namespace gxk
