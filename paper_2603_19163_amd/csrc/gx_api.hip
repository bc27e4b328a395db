// gx_api.hip -- host runtime behind the C interface in include/gx.h:
// device checks, instance staging, job allocation, launch planning (one
// evolve launch per AOS epoch chunk, replayed from a captured HIP graph),
// results and snapshots.
#include "../../include/gx.h"
#include "gx_internal.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace gx;

// Side streams for the concurrent launches of one epoch's work-item groups:
// the groups fork from the main stream through one event and join back
// through one event each (also inside a captured graph).
// Work items are grouped by (kind, staging, LDS class): a launch reserves the
// LDS of its largest item for every workgroup, so small instances of a kind
// get a launch of their own with more workgroups per CU.
constexpr int kLdsClasses = 4;
constexpr int kMaxGroups = 16;
inline int lds_class(uint32_t lds) { return lds <= 8192 ? 0 : (lds <= 16384 ? 1 : (lds <= 32768 ? 2 : 3)); }
struct Fan {
  hipStream_t side[kMaxGroups - 1] = {};
  hipEvent_t fork = nullptr, join[kMaxGroups - 1] = {};
  bool ready = false;
};

struct gx_ctx {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Fan fan;
  std::string err;
  gx_device_info info{};
  uint32_t max_lds = 0;
  std::vector<gx_instance *> insts;
  std::vector<gx_job *> jobs;
};

struct gx_instance {
  DevInst h{};
  DevInst *d = nullptr;
  std::vector<void *> bufs;
  int max_d = 0;
  uint32_t key = 0;
};

struct gx_batch;

struct gx_job {
  gx_ctx *ctx = nullptr;
  gx_instance *inst = nullptr;
  DevJob h{};
  DevJob *d = nullptr;
  std::vector<void *> bufs;
  gx_batch *batch = nullptr;   // jobs of one gx_solve_batch share their storage
  uint32_t g_host = 0, launches = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  float evolve_ms = 0.f;
  hipGraphExec_t gexec = nullptr;
  uint32_t gchunk = 0;
};

struct gx_batch {
  int refs = 0;
  DevJob *jobs_d = nullptr;
  void *arena = nullptr;
  uint2 *items = nullptr;
  uint32_t *next = nullptr;   // work-item counters, one per group
};

namespace {

gx_status fail(gx_ctx *c, gx_status s, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIPCHK(ctx, call)                                                                       \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail((ctx), GX_E_DEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t pad16(size_t b) { return (b + 15) & ~size_t(15); }

// Exponential tables of the acceptance test, round-half-even of 2^31 e^-x,
// evaluated in x87 extended precision.
void make_exp_tables(uint32_t hi[16], uint32_t lo[256]) {
  for (int i = 0; i < 16; ++i) hi[i] = (uint32_t)nearbyintl(ldexpl(expl(-(long double)i), 31));
  for (int j = 0; j < 256; ++j) lo[j] = (uint32_t)nearbyintl(ldexpl(expl(-(long double)j / 256.0L), 31));
}

template <class T>
gx_status dalloc(gx_ctx *c, std::vector<void *> &owner, T **p, size_t bytes) {
  void *q = nullptr;
  const hipError_t e = hipMalloc(&q, pad16(bytes) + 16);
  if (e != hipSuccess) return fail(c, GX_E_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  owner.push_back(q);
  *p = (T *)q;
  return GX_OK;
}

gx_status to_host(gx_ctx *c, const gx_instance_desc *d, const int32_t *src, size_t count, std::vector<int32_t> &out) {
  out.resize(count);
  if (count == 0) return GX_OK;
  if (!src) return fail(c, GX_E_INVALID, "missing array of %zu elements", count);
  if (d->is_device_ptr) HIPCHK(c, hipMemcpy(out.data(), src, count * 4, hipMemcpyDeviceToHost));
  else memcpy(out.data(), src, count * 4);
  return GX_OK;
}

// the operators a job on this instance takes when op_mask is 0
uint32_t encoding_ops(const DevInst &h) {
  if (h.kind == KKNAP) return (1u << OFLIP) | (1u << OSFLIP);
  if (h.kind == KCOLOR) return (1u << ORESET) | (1u << OSRESET);
  const uint32_t perm = (1u << O2OPT) | (1u << OSWAP) | (1u << OINS) | (1u << OOROPT) | (1u << O3OPT);
  if (h.rows) return perm | (1u << OROWSWAP) | (1u << OROWSPLIT) | (1u << OROWMERGE);
  return perm;
}
// the operators op_mask may name: single-row permutations add the LNS
// operators, which are taken only when named
uint32_t allowed_ops(const DevInst &h) {
  const bool single = !h.rows && (h.kind == KTSP || h.kind == KQAP || h.kind == KVRP);
  return encoding_ops(h) | (single ? kLnsMask : 0u);
}
// Tab. weight_preset, LNS cap (Q16) by scale; 0 where ids 5-7 are not LNS operators
uint32_t lns_cap_of(const DevInst &h) {
  if (h.rows || !(h.kind == KTSP || h.kind == KQAP || h.kind == KVRP)) return 0;
  return h.n <= 100 ? 1311u : (h.n <= 250 ? 655u : 328u);
}

void free_bufs(std::vector<void *> &b) {
  for (void *p : b) (void)hipFree(p);
  b.clear();
}


// ------------------------------------------------------------ instance staging
// prepare_instance validates a description and builds the host-side arrays
// (int16 conversions, CSR); place_instance lays them out in one device block,
// builds derived distance matrices with a kernel and writes the DevInst record
// at the end of the block.
enum Field { F_XY, F_D16, F_D32, F_QF, F_QD, F_KW, F_KV, F_DEM, F_RDY, F_DUE, F_ADJOFF, F_ADJ, F_EDGES };

struct HostArr {
  int field;
  size_t bytes;
  std::vector<char> data;   // empty: built on the device
};

struct Prepared {
  DevInst h{};
  std::vector<HostArr> arrs;
  int build_d16_side = 0;   // > 0: d16 (side x side) from the coordinates
  int max_d = 0;
  uint32_t key = 0;
  size_t dev_bytes() const {
    size_t b = 0;
    for (const auto &a : arrs) b += pad16(a.bytes) + 16;
    return b + pad16(sizeof(DevInst)) + 16;
  }
};

template <class T>
void add_arr(Prepared &pr, int field, const std::vector<T> &v) {
  HostArr a{field, v.size() * sizeof(T), {}};
  a.data.resize(a.bytes);
  if (a.bytes) memcpy(a.data.data(), v.data(), a.bytes);
  pr.arrs.push_back(std::move(a));
}

void add_built(Prepared &pr, int field, size_t bytes) { pr.arrs.push_back(HostArr{field, bytes, {}}); }

gx_status prepare_instance(gx_ctx *c, const gx_instance_desc *d, Prepared &pr, bool tsp_d16) {
  const int n = d->n;
  if (n < 1) return fail(c, GX_E_INVALID, "n must be >= 1 (got %d)", n);
  DevInst &h = pr.h;
  // the multi-row VRPTW runs the VRPTW kernels with its rows (and markers) in the solution
  const bool rows = d->kind == GX_VRPTW_ROWS;
  h.kind = rows ? KVRP : d->kind;
  h.n = n;
  h.lb = d->lb;
  h.ub = d->ub;
  h.capacity = d->capacity;
  h.vehicles = d->vehicles;
  h.service = d->service_time;
  h.horizon = d->horizon;
  h.n_edges = d->n_edges;
  pr.key = d->instance_key;
  if (h.kind != KVRP && (d->obj_weights[0] | d->obj_weights[1] | d->obj_weights[2]))
    return fail(c, GX_E_INVALID, "objective weights apply to VRPTW only");
  if (h.kind != KVRP && (d->lex_order[0] | d->lex_order[1] | d->lex_order[2]))
    return fail(c, GX_E_INVALID, "the lexicographic mode applies to VRPTW only");
  std::vector<int32_t> A, B;
  gx_status st = GX_OK;
  double fbound = 0;
  if (d->kind == KTSP) {
    if (n > 65535) return fail(c, GX_E_UNSUPPORTED, "TSP n <= 65535");
    if (d->a_is_coords) {
      if ((st = to_host(c, d, d->a, (size_t)2 * n, A))) return st;
      for (int32_t v : A)
        if (v < 0 || v >= kMaxCoord) return fail(c, GX_E_INVALID, "coordinates must lie in [0, 16384)");
      add_arr(pr, F_XY, A);
      h.has_xy = 1;
      if (tsp_d16 && n <= 4096) {
        add_built(pr, F_D16, (size_t)2 * n * n);
        pr.build_d16_side = n;
      }
      pr.max_d = 23171;
    } else {
      if ((st = to_host(c, d, d->a, (size_t)n * n, A))) return st;
      int mx = 0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const int32_t v = A[(size_t)i * n + j];
          if (v < 0 || v >= (1 << 24) || v != A[(size_t)j * n + i] || (i == j && v != 0))
            return fail(c, GX_E_INVALID, "TSP matrix must be symmetric, zero-diagonal, in [0, 2^24)");
          mx = std::max(mx, v);
        }
      pr.max_d = mx;
      add_arr(pr, F_D32, A);
      if (mx < 32768) add_arr(pr, F_D16, std::vector<int16_t>(A.begin(), A.end()));
    }
    fbound = 6.0 * n * (double)std::max(pr.max_d, 1);
  } else if (d->kind == KQAP) {
    if (n > kMaxQapN) return fail(c, GX_E_UNSUPPORTED, "QAP n <= %d", kMaxQapN);
    if ((st = to_host(c, d, d->a, (size_t)n * n, A)) || (st = to_host(c, d, d->b, (size_t)n * n, B))) return st;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
        if (A[ij] < 0 || A[ij] >= 16384 || B[ij] < 0 || B[ij] >= 16384 || A[ij] != A[ji] || B[ij] != B[ji])
          return fail(c, GX_E_INVALID, "QAP matrices must be symmetric with entries in [0, 16384)");
      }
    const int64_t mf = *std::max_element(A.begin(), A.end()), md = *std::max_element(B.begin(), B.end());
    h.qap_sums32 = 2 * (int64_t)n * mf * md < (int64_t(1) << 31);
    h.qap_h16 = (int64_t)n * mf * md < (int64_t(1) << 16);
    add_arr(pr, F_QF, std::vector<int16_t>(A.begin(), A.end()));
    add_arr(pr, F_QD, std::vector<int16_t>(B.begin(), B.end()));
    fbound = 4.0 * n * n * 16384.0 * 16384.0;
  } else if (d->kind == KKNAP) {
    if (n > 16384) return fail(c, GX_E_UNSUPPORTED, "knapsack n <= 16384");
    if ((st = to_host(c, d, d->a, (size_t)n, A)) || (st = to_host(c, d, d->b, (size_t)n, B))) return st;
    int64_t mv = 0, sw = 0, sv = 0;
    for (int i = 0; i < n; ++i) {
      if (A[i] < 0 || A[i] > (1 << 20) || B[i] < 0 || B[i] > (1 << 20))
        return fail(c, GX_E_INVALID, "knapsack weights and values must lie in [0, 2^20]");
      mv = std::max<int64_t>(mv, B[i]);
      sw += A[i];
      sv += B[i];
    }
    if (d->capacity < 0) return fail(c, GX_E_INVALID, "capacity must be >= 0");
    h.lambda = mv + 1;
    add_arr(pr, F_KW, A);
    add_arr(pr, F_KV, B);
    fbound = 4.0 * ((double)sv + (double)h.lambda * (double)sw);
  } else if (h.kind == KVRP) {
    if (n > kMaxVrpN) return fail(c, GX_E_UNSUPPORTED, "VRPTW n <= %d", kMaxVrpN);
    if (rows && (d->vehicles < 1 || d->vehicles > kMaxVrpN))
      return fail(c, GX_E_UNSUPPORTED, "multi-row VRPTW takes 1 to %d rows (vehicles)", kMaxVrpN);
    if (rows && d->capacity > (1 << 22)) return fail(c, GX_E_UNSUPPORTED, "multi-row VRPTW capacity <= 2^22");
    const int m = n + 1;
    if ((st = to_host(c, d, d->a, (size_t)2 * m, A)) || (st = to_host(c, d, d->b, (size_t)3 * m, B))) return st;
    for (int32_t v : A)
      if (v < 0 || v >= kMaxCoord) return fail(c, GX_E_INVALID, "coordinates must lie in [0, 16384)");
    if (d->capacity < 1 || d->vehicles < 1 || d->service_time < 0 || d->service_time > (1 << 16) ||
        d->horizon < 0 || d->horizon > (1 << 19))
      return fail(c, GX_E_INVALID, "VRPTW capacity, vehicles >= 1; service <= 2^16; horizon in [0, 2^19]");
    for (int i = 0; i < m; ++i) {
      const int32_t q = B[i], r = B[m + i], u = B[2 * m + i];
      if (q < 0 || q > d->capacity || r < 0 || u < 0 || r > (1 << 19) || u > (1 << 19))
        return fail(c, GX_E_INVALID, "VRPTW demand in [0, capacity], times in [0, 2^19]");
    }
    const int32_t *w = d->obj_weights;
    for (int i = 0; i < 3; ++i)
      if (w[i] < 0 || w[i] > (1 << 20)) return fail(c, GX_E_INVALID, "VRPTW objective weights must lie in [0, 2^20]");
    const bool dflt = w[0] == 0 && w[1] == 0 && w[2] == 0;
    h.vw_d = dflt ? 1 : w[0];
    h.vw_r = dflt ? 0 : w[1];
    h.vw_m = dflt ? 0 : w[2];
    // lexicographic mode: levels up to the first 0, distinct objectives 1..3
    int levels = 0;
    while (levels < 3 && d->lex_order[levels] != 0) ++levels;
    for (int i = 0; i < 3; ++i) {
      const int id = d->lex_order[i], tol = d->lex_tol[i];
      if (i >= levels ? (id != 0 || tol != 0) : (id < 1 || id > 3 || tol < 0 || tol > (1 << 30)))
        return fail(c, GX_E_INVALID, "lex_order entries in 1..3 ended by 0 (tolerances in [0, 2^30], 0 past the end)");
      for (int k = 0; k < i && i < levels; ++k)
        if (d->lex_order[k] == id) return fail(c, GX_E_INVALID, "lex_order repeats an objective");
    }
    if (levels && !dflt) return fail(c, GX_E_INVALID, "obj_weights must be zero in the lexicographic mode");
    h.lex_levels = levels;
    for (int i = 0; i < 3; ++i) {
      h.lex_id[i] = i < levels ? d->lex_order[i] : 0;
      h.lex_tol[i] = i < levels ? d->lex_tol[i] : 0;
    }
    h.dn = m;
    add_arr(pr, F_XY, A);
    h.has_xy = 1;
    add_built(pr, F_D16, (size_t)2 * m * m);
    pr.build_d16_side = m;
    add_arr(pr, F_DEM, std::vector<int32_t>(B.begin(), B.begin() + m));
    add_arr(pr, F_RDY, std::vector<int32_t>(B.begin() + m, B.begin() + 2 * m));
    add_arr(pr, F_DUE, std::vector<int32_t>(B.begin() + 2 * m, B.end()));
    fbound = 4.0 * ((h.vw_d + h.vw_m) * m * 23171.0 + (double)h.vw_r * m +
                    100.0 * m * (m * 23171.0 + (1 << 19) + (double)m * (1 << 16)) + 10000.0 * m);
    if (rows) {   // the solution's entries: customers and one marker per row; loads above capacity
      h.rows = d->vehicles;
      h.n = n + d->vehicles;
      fbound += 4.0 * 100.0 * m * (double)d->capacity;
    }
  } else if (d->kind == KCOLOR) {
    if (n > 32767) return fail(c, GX_E_UNSUPPORTED, "colouring n <= 32767");
    if (d->lb > d->ub || d->lb < -32768 || d->ub > 32767)
      return fail(c, GX_E_INVALID, "colouring needs -32768 <= lb <= ub <= 32767");
    if (d->n_edges < 0 || d->n_edges > (1 << 20)) return fail(c, GX_E_INVALID, "n_edges in [0, 2^20]");
    if ((st = to_host(c, d, d->a, (size_t)2 * d->n_edges, A))) return st;
    std::vector<int32_t> off(n + 1, 0), adj((size_t)2 * d->n_edges);
    for (int e = 0; e < d->n_edges; ++e) {
      const int u = A[2 * e], v = A[2 * e + 1];
      if (u < 0 || v < 0 || u >= n || v >= n || u == v)
        return fail(c, GX_E_INVALID, "edge %d out of range or a self loop", e);
      off[u + 1]++;
      off[v + 1]++;
    }
    for (int i = 0; i < n; ++i) off[i + 1] += off[i];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int e = 0; e < d->n_edges; ++e) {
      const int u = A[2 * e], v = A[2 * e + 1];
      adj[fill[u]++] = v;
      adj[fill[v]++] = u;
    }
    add_arr(pr, F_ADJOFF, off);
    add_arr(pr, F_ADJ, adj);
    add_arr(pr, F_EDGES, A);
    fbound = 4.0 * d->n_edges + 4;
  } else {
    return fail(c, GX_E_INVALID, "unknown problem kind %d", d->kind);
  }
  if (fbound >= std::ldexp(1.0, 45)) return fail(c, GX_E_UNSUPPORTED, "objective range exceeds 2^45");
  return GX_OK;
}

// Copies the instance arrays and its record into the device block at `base`;
// with `stage` (pinned host memory of staging_bytes(pr)) the copies go through
// it, so that they are asynchronous.
size_t staging_bytes(const Prepared &pr) {
  size_t b = pad16(sizeof(DevInst));
  for (const auto &a : pr.arrs) b += pad16(a.bytes);
  return b;
}

gx_status place_instance(gx_ctx *c, Prepared &pr, char *base, hipStream_t s, DevInst *out_h, DevInst **out_d,
                         char *stage = nullptr) {
  DevInst h = pr.h;
  char *q = base;
  char *sp = stage ? stage + pad16(sizeof(DevInst)) : nullptr;
  for (const auto &a : pr.arrs) {
    char *dst = q;
    q += pad16(a.bytes) + 16;
    if (!a.data.empty()) {
      const void *src = a.data.data();
      if (sp) {
        memcpy(sp, src, a.bytes);
        src = sp;
        sp += pad16(a.bytes);
      }
      HIPCHK(c, hipMemcpyAsync(dst, src, a.bytes, hipMemcpyHostToDevice, s));
    }
    switch (a.field) {
      case F_XY: h.xy = (const int32_t *)dst; break;
      case F_D16: h.d16 = (const int16_t *)dst; break;
      case F_D32: h.d32 = (const int32_t *)dst; break;
      case F_QF: h.qf = (const int16_t *)dst; break;
      case F_QD: h.qd = (const int16_t *)dst; break;
      case F_KW: h.kw = (const int32_t *)dst; break;
      case F_KV: h.kv = (const int32_t *)dst; break;
      case F_DEM: h.dem = (const int32_t *)dst; break;
      case F_RDY: h.rdy = (const int32_t *)dst; break;
      case F_DUE: h.due = (const int32_t *)dst; break;
      case F_ADJOFF: h.adj_off = (const int32_t *)dst; break;
      case F_ADJ: h.adj = (const int32_t *)dst; break;
      default: h.edges = (const int32_t *)dst; break;
    }
  }
  if (pr.build_d16_side > 0) HIPCHK(c, gxk::build_tsp_d16_from_xy(h.xy, pr.build_d16_side, (int16_t *)h.d16, s));
  DevInst *dd = (DevInst *)q;
  *out_h = h;
  // the record is copied from pr.h's twin kept alive by the caller until the stream syncs
  pr.h = h;
  const void *rec = &pr.h;
  if (stage) {
    memcpy(stage, &pr.h, sizeof(DevInst));
    rec = stage;
  }
  HIPCHK(c, hipMemcpyAsync(dd, rec, sizeof(DevInst), hipMemcpyHostToDevice, s));
  *out_d = dd;
  return GX_OK;
}

}  // namespace

// ------------------------------------------------------------ static workspace
// gx_solve_static keeps a whole solve's device state in this file-scope array
// (each device holds its own copy for the life of the process).  Host code
// never passes the array's name to a kernel or a copy: gx_create looks up the
// array's device address once per device, with that device current, and the
// entry point uses that address.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices];

static hipError_t static_scratch_setup(int dev) {   // the device is current
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = (char *)ptr;
  return hipSuccess;
}

extern "C" {

gx_status gx_exp_tables(uint32_t hi[16], uint32_t lo[256]) {
  if (!hi || !lo) return GX_E_INVALID;
  make_exp_tables(hi, lo);
  return GX_OK;
}

gx_status gx_device_check(gx_ctx *c, int32_t what, uint64_t key, const uint64_t *in, uint64_t *out,
                          int64_t count) {
  if (!c || (count > 0 && (!in || !out))) return fail(c, GX_E_INVALID, "null argument");
  if (what < GX_CHECK_PHILOX || what > GX_CHECK_ACCEPT) return fail(c, GX_E_INVALID, "unknown check %d", what);
  if (count < 0 || count > (int64_t(1) << 26)) return fail(c, GX_E_INVALID, "count in [0, 2^26]");
  if (count == 0) return GX_OK;
  const size_t in_w = what == GX_CHECK_DIST ? 1 : 2, out_w = what == GX_CHECK_PHILOX ? 4 : (what == GX_CHECK_DIST ? 2 : 1);
  if (what == GX_CHECK_DIST)
    for (int64_t i = 0; i < count; ++i)
      for (int s = 0; s < 64; s += 16)
        if (((in[i] >> s) & 0xFFFF) >= (uint64_t)kMaxCoord)
          return fail(c, GX_E_INVALID, "coordinates must lie in [0, 16384)");
  HIPCHK(c, hipSetDevice(c->dev));
  std::vector<void *> bufs;
  uint64_t *din = nullptr, *dout = nullptr;
  gx_status st;
  if ((st = dalloc(c, bufs, &din, 8 * in_w * count)) || (st = dalloc(c, bufs, &dout, 8 * out_w * count))) {
    free_bufs(bufs);
    return st;
  }
  hipError_t e = hipMemcpyAsync(din, in, 8 * in_w * count, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = gxk::device_check(what, key, din, dout, count, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, 8 * out_w * count, hipMemcpyDeviceToHost, c->stream);
  const hipError_t es = hipStreamSynchronize(c->stream);   // before the buffers are freed
  if (e == hipSuccess) e = es;
  free_bufs(bufs);
  if (e != hipSuccess) return fail(c, GX_E_DEVICE, "device check: %s", hipGetErrorString(e));
  return GX_OK;
}

gx_status gx_create(int device_ordinal, void *hip_stream, gx_ctx **out) {
  if (!out) return GX_E_INVALID;
  *out = nullptr;
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt == 0) return GX_E_DEVICE;
  if (device_ordinal < 0 || device_ordinal >= cnt) return GX_E_INVALID;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device_ordinal) != hipSuccess) return GX_E_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GX_E_DEVICE;
  gx_ctx *c = new gx_ctx();
  c->dev = device_ordinal;
  if (hipSetDevice(device_ordinal) != hipSuccess) {
    delete c;
    return GX_E_DEVICE;
  }
  if (hip_stream) c->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return GX_E_DEVICE;
    }
    c->own_stream = true;
  }
  c->info.cus = prop.multiProcessorCount;
  c->info.lds_per_block = (int32_t)prop.sharedMemPerBlock;
  c->info.wave_size = prop.warpSize;
  c->info.l2_bytes = prop.l2CacheSize;
  snprintf(c->info.arch, sizeof c->info.arch, "%s", prop.gcnArchName);
  c->max_lds = (uint32_t)prop.sharedMemPerBlock;
  uint32_t hi[16], lo[256];
  make_exp_tables(hi, lo);
  if (gxk::set_exp_tables(hi, lo) != hipSuccess || gxk::prepare_kernel_attrs(c->max_lds) != hipSuccess ||
      prop.warpSize != kWave || static_scratch_setup(device_ordinal) != hipSuccess) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return GX_E_DEVICE;
  }
  *out = c;
  return GX_OK;
}

const char *gx_last_error(const gx_ctx *c) { return c ? c->err.c_str() : "null context"; }

gx_status gx_measure_peaks(gx_ctx *c, gx_peaks *out) {
  if (!c || !out) return fail(c, GX_E_INVALID, "null argument");
  memset(out, 0, sizeof *out);
  HIPCHK(c, hipSetDevice(c->dev));
  HIPCHK(c, gxk::measure_peaks(c->info.cus, c->stream, out));
  return GX_OK;
}

gx_status gx_get_device_info(gx_ctx *c, gx_device_info *out) {
  if (!c || !out) return GX_E_INVALID;
  *out = c->info;
  return GX_OK;
}

gx_status gx_instance_free(gx_ctx *c, gx_instance *in) {
  if (!c || !in) return GX_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  free_bufs(in->bufs);
  c->insts.erase(std::remove(c->insts.begin(), c->insts.end(), in), c->insts.end());
  delete in;
  return GX_OK;
}

gx_status gx_instance_upload(gx_ctx *c, const gx_instance_desc *d, gx_instance **out) {
  if (!c || !d || !out) return fail(c, GX_E_INVALID, "null argument");
  *out = nullptr;
  HIPCHK(c, hipSetDevice(c->dev));
  Prepared pr;
  gx_status st = prepare_instance(c, d, pr, true);
  if (st) return st;
  gx_instance *in = new gx_instance();
  char *base = nullptr;
  if ((st = dalloc(c, in->bufs, &base, pr.dev_bytes()))) {
    delete in;
    return st;
  }
  DevInst *dd = nullptr;
  if ((st = place_instance(c, pr, base, c->stream, &in->h, &dd)) ||
      (st = hipStreamSynchronize(c->stream) == hipSuccess ? GX_OK : fail(c, GX_E_DEVICE, "instance staging failed"))) {
    free_bufs(in->bufs);
    delete in;
    return st;
  }
  in->d = dd;
  in->key = pr.key;
  in->max_d = pr.max_d;
  c->insts.push_back(in);
  *out = in;
  return GX_OK;
}

}  // extern "C"

namespace {

// What job setup needs to know about an instance (uploaded or prepared).
struct InstInfo {
  DevInst h;            // host copy (device pointers may be null before placement)
  DevInst *d;           // device record (null before placement)
  bool has_d16, has_d32, has_xy;
  uint32_t key;
};

InstInfo info_of(const gx_instance *in) {
  return InstInfo{in->h, in->d, in->h.d16 != nullptr, in->h.d32 != nullptr, in->h.has_xy != 0, in->key};
}

uint32_t resolve_stage(const InstInfo &ii, uint32_t req) {
  if (ii.h.kind == KQAP) return ii.h.qap_h16 ? 1u : 0u;   // 16-bit row sums when they fit
  if (ii.h.kind != KTSP) return 0;
  if (req != SAUTO) return req;
  // Coordinates in LDS keep the footprint at 6n + 2n bytes, so a CU holds
  // as many workgroups as its registers allow; an int16 matrix in LDS
  // (2n^2 bytes) cuts that to a few per CU at n ~ 100, which costs more than
  // the exact distance recomputation saves.
  const int n = ii.h.n;
  if (ii.has_xy) return SLDSXY;
  if (n <= 128 && ii.has_d16) return SLDS16;
  if (ii.has_d16) return SGLB16;
  return SGLB32;
}

uint32_t job_lds(const InstInfo &ii, uint32_t stage, uint32_t op_mask) {
  uint32_t b = lds_bytes_for(ii.h.kind, ii.h.n, evolve_variant(ii.h.kind, stage, op_mask, ii.h.lex_levels, ii.h.rows),
                             ii.h.rows);
  if (ii.h.kind == KCOLOR) b += (uint32_t)pad16((size_t)8 * ii.h.n_edges);
  return std::max<uint32_t>(b, 16);
}

// Validate parameters and fill the constant part of a DevJob.
gx_status fill_job(gx_ctx *c, const InstInfo &ii, const gx_solve_params *p, DevJob &h, uint32_t P_auto,
                   uint32_t lds_limit) {
  if (!p) return fail(c, GX_E_INVALID, "null parameters");
  const uint32_t mask = p->op_mask ? (p->op_mask & allowed_ops(ii.h)) : encoding_ops(ii.h);
  if (!mask) return fail(c, GX_E_INVALID, "op_mask enables no operator of this encoding");
  if (p->alpha_q32 == 0) return fail(c, GX_E_INVALID, "alpha_q32 is required");
  const uint32_t C = p->candidates ? p->candidates : 128;
  if (C > 65536) return fail(c, GX_E_INVALID, "candidates <= 65536");
  const uint32_t E = p->aos_epoch ? p->aos_epoch : 10;
  const uint32_t A = p->aos_alpha_q16 ? p->aos_alpha_q16 : 49152;
  if (A >= 65536) return fail(c, GX_E_INVALID, "aos_alpha_q16 < 65536");
  const uint32_t FL = p->w_floor_q16 ? p->w_floor_q16 : 1024;
  if (FL > 65536) return fail(c, GX_E_INVALID, "w_floor_q16 <= 65536");
  if (p->aos_credit > 1) return fail(c, GX_E_INVALID, "aos_credit is 0 or 1");
  if (p->generations > 0xFFFFFFFEu) return fail(c, GX_E_INVALID, "generations <= 2^32 - 2");
  const uint32_t P = p->population ? p->population : P_auto;
  if (P < 1 || P > (1u << 20)) return fail(c, GX_E_INVALID, "population in [1, 2^20]");
  const uint32_t K = p->oversample_k ? p->oversample_k : 4;
  if ((uint64_t)K * P > (1u << 22)) return fail(c, GX_E_UNSUPPORTED, "oversample pool <= 2^22");
  if (p->staging > SGLB32) return fail(c, GX_E_INVALID, "unknown staging %u", p->staging);
  const uint32_t isl = p->islands > 1 ? p->islands : 1;
  if (isl > 1 && (isl > 64 || P % isl != 0 || P / isl < 2))
    return fail(c, GX_E_INVALID, "islands <= 64 dividing the population into islands of >= 2 (P = %u)", P);
  if (p->migrate_mode > 2) return fail(c, GX_E_INVALID, "migrate_mode is 0 (ring), 1 (top-N) or 2 (hybrid)");
  const uint32_t mig_n = p->migrate_n ? p->migrate_n : 1;
  if (mig_n > 8 || (isl > 1 && mig_n >= P / isl)) return fail(c, GX_E_INVALID, "migrate_n <= 8 and below the island size");
  const uint32_t stage = resolve_stage(ii, p->staging);
  if (ii.h.kind == KTSP) {
    if ((stage == SLDS16 || stage == SGLB16) && !ii.has_d16)
      return fail(c, GX_E_UNSUPPORTED, "no int16 distance matrix for this instance");
    if (stage == SLDSXY && !ii.has_xy) return fail(c, GX_E_UNSUPPORTED, "coordinates-in-LDS needs coordinates");
  }
  if (p->aos_scope > 1) return fail(c, GX_E_INVALID, "aos_scope is 0 (instance) or 1 (solution)");
  if (p->aos_scope == 1 && (uint64_t)E * C > (1u << 30))
    return fail(c, GX_E_INVALID, "per-solution weights need aos_epoch * candidates <= 2^30");
  for (int i = 0; i < kOps; ++i)
    if (p->init_weight_q16[i] > (1u << 24)) return fail(c, GX_E_INVALID, "init_weight_q16 entries <= 2^24");
  for (int i = 0; i < kOps; ++i)
    if (p->weight_cap_q16[i] > 65536u) return fail(c, GX_E_INVALID, "weight_cap_q16 entries <= 2^16");
  if (ii.h.lex_levels && p->aos_scope)
    return fail(c, GX_E_UNSUPPORTED, "the lexicographic mode takes aos_scope 0");
  const uint32_t lds = job_lds(ii, stage, mask);
  if (lds > lds_limit)
    return fail(c, GX_E_UNSUPPORTED, "instance needs %u bytes of LDS per workgroup (limit %u)", lds, lds_limit);
  memset(&h, 0, sizeof h);
  h.inst = ii.d;
  h.seed = p->seed;
  h.t0_param = p->t0_q16;
  h.P = P;
  h.C = C;
  h.G = p->generations;
  h.E = E;
  h.op_mask = mask;
  h.credit = p->aos_credit;
  h.aos_A = A;
  h.w_floor = FL;
  h.stag_limit = p->stagnation_epochs ? p->stagnation_epochs : 5;
  h.key = ii.key;
  h.alpha = p->alpha_q32;
  h.Q = K * P;
  h.stage = stage;
  h.lds_bytes = lds;
  h.islands = isl;
  h.mig_epochs = p->migrate_epochs;
  h.mig_mode = p->migrate_mode;
  h.mig_n = mig_n;
  h.elite_epochs = p->elite_epochs;
  h.aos_scope = p->aos_scope;
  for (int i = 0; i < kOps; ++i) h.init_w[i] = p->init_weight_q16[i];
  h.lex_levels = (uint32_t)ii.h.lex_levels;
  h.rows = (uint32_t)ii.h.rows;
  h.lns_cap = lns_cap_of(ii.h);
  for (int i = 0; i < kOps; ++i)   // the caller's caps, else the LNS cap or 1.0
    h.w_cap[i] = p->weight_cap_q16[i] ? p->weight_cap_q16[i]
                                      : ((h.lns_cap && ((kLnsMask >> i) & 1u)) ? h.lns_cap : 65536u);
  return GX_OK;
}

// whether a job's epoch ends can exchange solutions (island migration or
// elite injection): its epoch kernel then runs the wide variant
bool migrates(const DevJob &h) { return (h.mig_epochs && h.islands >= 2) || h.elite_epochs; }

int heur_mats_of(int kind) { return kind == KQAP ? 2 : ((kind == KTSP || kind == KVRP) ? 1 : 0); }

// bytes of the per-job device arrays, laid out by carve_job (lex: the
// objective vectors of the lexicographic mode)
size_t job_array_bytes(size_t n, size_t P, size_t Q, bool lex) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return 2 * al(4 * n * P) + 2 * al(8 * P) + al(4 * n * Q) + al(8 * Q) + al(32 * n) + al(4 * n) +
         al(8 * kShards * kEpochSlots) + al(sizeof(SolAos) * P) + (lex ? 2 * al(32 * P) + al(32 * Q) : 0);
}

void carve_job(DevJob &h, char *q, size_t n) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  auto take = [&](size_t bytes) {
    char *r = q;
    q += al(bytes);
    return r;
  };
  h.cur = (int32_t *)take(4 * n * h.P);
  h.best = (int32_t *)take(4 * n * h.P);
  h.cur_f = (int64_t *)take(8 * (size_t)h.P);
  h.best_f = (int64_t *)take(8 * (size_t)h.P);
  h.pool = (int32_t *)take(4 * n * h.Q);
  h.pool_f = (int64_t *)take(8 * (size_t)h.Q);
  h.sums = (int64_t *)take(32 * n);
  h.best_out = (int32_t *)take(4 * n);
  h.shard = (unsigned long long *)take(8 * kShards * kEpochSlots);
  h.saos = (SolAos *)take(sizeof(SolAos) * h.P);
  if (h.lex_levels) {
    h.cur_v = (int64_t *)take(32 * (size_t)h.P);
    h.best_v = (int64_t *)take(32 * (size_t)h.P);
    h.pool_v = (int64_t *)take(32 * (size_t)h.Q);
  }
}

// every device array the kernels dereference for this job is in place
bool job_arrays_placed(const DevJob &h) {
  const bool base = h.cur && h.best && h.cur_f && h.best_f && h.pool && h.pool_f && h.sums && h.best_out && h.shard &&
                    h.saos;
  return base && (!h.lex_levels || (h.cur_v && h.best_v && h.pool_v));
}

gx_status ensure_d32(gx_ctx *c, gx_instance *in) {
  if (in->h.d32) return GX_OK;
  int32_t *d32;
  gx_status st;
  const int n = in->h.n;
  if ((st = dalloc(c, in->bufs, &d32, (size_t)4 * n * n))) return st;
  HIPCHK(c, gxk::build_d32_from_xy(in->h.xy, n, d32, c->stream));
  in->h.d32 = d32;
  HIPCHK(c, hipMemcpy(in->d, &in->h, sizeof(DevInst), hipMemcpyHostToDevice));
  return GX_OK;
}

uint32_t chunks_between(uint32_t g, uint32_t target, uint32_t E) {
  uint32_t k = 0;
  while (g < target) {
    const uint64_t nb = ((uint64_t)g / E + 1) * E;
    g = (uint32_t)std::min<uint64_t>(target, nb);
    ++k;
  }
  return k;
}

bool graphs_disabled() {
  const char *e = getenv("GX_DISABLE_GRAPH");
  return e && *e && *e != '0';
}

bool fan_disabled() {
  const char *e = getenv("GX_SERIAL_GROUPS");
  return e && *e && *e != '0';
}

hipError_t fan_init(Fan &f) {
  if (f.ready) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming);
  for (int g = 0; e == hipSuccess && g < kMaxGroups - 1; ++g) {
    e = hipStreamCreateWithFlags(&f.side[g], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f.join[g], hipEventDisableTiming);
  }
  f.ready = e == hipSuccess;
  return e;
}

void fan_free(Fan &f) {
  for (int g = 0; g < kMaxGroups - 1; ++g) {
    if (f.side[g]) (void)hipStreamDestroy(f.side[g]);
    if (f.join[g]) (void)hipEventDestroy(f.join[g]);
    f.side[g] = nullptr;
    f.join[g] = nullptr;
  }
  if (f.fork) (void)hipEventDestroy(f.fork);
  f.fork = nullptr;
  f.ready = false;
}

// The work items of one epoch launch, grouped by (kind, staging): every group
// is one launch of that group's kernel (its own registers and LDS), items
// heaviest first within the group.
struct Group {
  int kind, stage;
  uint32_t off, count, lds, grid;
  double cost;   // summed cost estimate of the group's items
};
struct ItemRec {
  int kind, stage;
  uint32_t lds;
  double cost;
  uint2 item;
};

gx_status make_groups(gx_ctx *c, std::vector<ItemRec> &recs, uint2 *items, std::vector<Group> &gs) {
  std::stable_sort(recs.begin(), recs.end(), [](const ItemRec &x, const ItemRec &y) {
    if (x.kind != y.kind) return x.kind < y.kind;
    if (x.stage != y.stage) return x.stage < y.stage;
    const int cx = lds_class(x.lds), cy = lds_class(y.lds);
    if (cx != cy) return cx < cy;
    return x.cost > y.cost;
  });
  gs.clear();
  for (size_t k = 0; k < recs.size(); ++k) {
    const ItemRec &r = recs[k];
    items[k] = r.item;
    if (gs.empty() || gs.back().kind != r.kind || gs.back().stage != r.stage ||
        lds_class(gs.back().lds) != lds_class(r.lds)) {
      if ((int)gs.size() == kMaxGroups) return fail(c, GX_E_UNSUPPORTED, "more than %d work-item groups", kMaxGroups);
      gs.push_back(Group{r.kind, r.stage, (uint32_t)k, 0, std::max<uint32_t>(16, r.lds), 0, 0.0});
    }
    gs.back().count++;
    gs.back().cost += r.cost;
    gs.back().lds = std::max(gs.back().lds, r.lds);
  }
  for (Group &g : gs) {
    int occ = 0;
    HIPCHK(c, gxk::occupancy_group(g.kind, g.stage, g.lds, &occ));
    g.grid = (uint32_t)std::min<size_t>(g.count, (size_t)c->info.cus * (size_t)std::max(1, occ));
  }
  // the heaviest group is launched first, so that the epoch's critical path
  // takes the CUs first and the lighter groups fill in beside it
  std::stable_sort(gs.begin(), gs.end(), [](const Group &x, const Group &y) { return x.cost > y.cost; });
  return GX_OK;
}

// One epoch chunk of every group: concurrent launches on the side streams
// (or one after the other on s), then the epoch kernel, which also clears the
// groups' work-item counters.
hipError_t launch_groups(const Fan &f, const std::vector<Group> &gs, DevJob *jobs, const uint2 *items,
                         uint32_t *next, const uint32_t *idx, uint32_t njobs, bool mig, hipStream_t s) {
  const bool fan = gs.size() > 1 && f.ready && !fan_disabled();
  hipError_t e = fan ? hipEventRecord(f.fork, s) : hipSuccess;
  for (size_t g = 0; e == hipSuccess && g < gs.size(); ++g) {
    hipStream_t sg = (fan && g > 0) ? f.side[g - 1] : s;
    if (fan && g > 0) e = hipStreamWaitEvent(sg, f.fork, 0);
    if (e == hipSuccess)
      e = gxk::evolve_group(gs[g].kind, gs[g].stage, jobs, items + gs[g].off, gs[g].count, next + g, gs[g].grid,
                            gs[g].lds, sg);
    if (e == hipSuccess && fan && g > 0) e = hipEventRecord(f.join[g - 1], sg);
  }
  for (size_t g = 1; e == hipSuccess && fan && g < gs.size(); ++g) e = hipStreamWaitEvent(s, f.join[g - 1], 0);
  return e != hipSuccess ? e : gxk::epoch(jobs, idx, njobs, next, (uint32_t)gs.size(), mig, s);
}

// Enqueue L identical evolve launches; a run of 64 is captured once into a
// graph and replayed (every launch reads its generation window from the job).
template <class Launch>
gx_status enqueue_launches(gx_ctx *c, gx_job *j, uint32_t L, Launch launch) {
  const uint32_t chunk = 64;
  uint32_t done = 0;
  if (L >= chunk && !graphs_disabled()) {
    if (!j->gexec) {
      hipGraph_t g;
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      for (uint32_t i = 0; i < chunk; ++i) {
        const hipError_t e = launch();
        if (e != hipSuccess) {
          hipGraph_t dummy;
          (void)hipStreamEndCapture(c->stream, &dummy);
          return fail(c, GX_E_DEVICE, "evolve launch during capture: %s", hipGetErrorString(e));
        }
      }
      HIPCHK(c, hipStreamEndCapture(c->stream, &g));
      const hipError_t e = hipGraphInstantiate(&j->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(c, GX_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      j->gchunk = chunk;
    }
    for (; done + chunk <= L; done += chunk) HIPCHK(c, hipGraphLaunch(j->gexec, c->stream));
  }
  for (; done < L; ++done) HIPCHK(c, launch());
  return GX_OK;
}

}  // namespace

extern "C" {

gx_status gx_autosize_population(gx_ctx *c, const gx_instance *in, const gx_solve_params *p, uint32_t *out) {
  if (!c || !in || !out) return fail(c, GX_E_INVALID, "null argument");
  const InstInfo ii = info_of(in);
  const uint32_t stage = resolve_stage(ii, p ? p->staging : 0);
  const uint32_t mask = p && p->op_mask ? (p->op_mask & allowed_ops(in->h)) : encoding_ops(in->h);
  const uint32_t lds = job_lds(ii, stage, mask);
  int occ = 0;
  HIPCHK(c, gxk::occupancy_plain(in->h.kind, evolve_variant(in->h.kind, stage, mask, in->h.lex_levels, in->h.rows), lds, &occ));
  // every CU filled to the residency the kernel's registers and LDS allow
  occ = std::max(1, std::min(occ, 32));
  *out = (uint32_t)(c->info.cus * occ);
  return GX_OK;
}

gx_status gx_job_create(gx_ctx *c, const gx_instance *cin, const gx_solve_params *p, gx_job **out) {
  if (!c || !cin || !p || !out) return fail(c, GX_E_INVALID, "null argument");
  *out = nullptr;
  gx_instance *in = const_cast<gx_instance *>(cin);
  HIPCHK(c, hipSetDevice(c->dev));
  uint32_t P_auto = 0;
  gx_status st;
  if (!p->population && (st = gx_autosize_population(c, in, p, &P_auto))) return st;
  gx_job *j = new gx_job();
  j->ctx = c;
  j->inst = in;
  DevJob &h = j->h;
  auto bail = [&](gx_status s) {
    free_bufs(j->bufs);
    delete j;
    return s;
  };
  if ((st = fill_job(c, info_of(in), p, h, P_auto, c->max_lds))) return bail(st);
  if (h.stage == SGLB32 && (st = ensure_d32(c, in))) return bail(st);
  const size_t n = (size_t)in->h.n;
  if ((st = dalloc(c, j->bufs, &h.cur, 4 * n * h.P)) || (st = dalloc(c, j->bufs, &h.best, 4 * n * h.P)) ||
      (st = dalloc(c, j->bufs, &h.cur_f, (size_t)8 * h.P)) || (st = dalloc(c, j->bufs, &h.best_f, (size_t)8 * h.P)) ||
      (st = dalloc(c, j->bufs, &h.pool, 4 * n * h.Q)) || (st = dalloc(c, j->bufs, &h.pool_f, (size_t)8 * h.Q)) ||
      (st = dalloc(c, j->bufs, &h.sums, 32 * n)) || (st = dalloc(c, j->bufs, &h.best_out, 4 * n)) ||
      (st = dalloc(c, j->bufs, &h.shard, (size_t)8 * kShards * kEpochSlots)) ||
      (st = dalloc(c, j->bufs, &h.saos, sizeof(SolAos) * h.P)) ||
      (st = dalloc(c, j->bufs, &j->d, sizeof(DevJob))))
    return bail(st);
  if (h.lex_levels &&
      ((st = dalloc(c, j->bufs, &h.cur_v, (size_t)32 * h.P)) || (st = dalloc(c, j->bufs, &h.best_v, (size_t)32 * h.P)) ||
       (st = dalloc(c, j->bufs, &h.pool_v, (size_t)32 * h.Q))))
    return bail(st);
  if (!job_arrays_placed(h)) return bail(fail(c, GX_E_DEVICE, "job arrays incomplete"));
  if (hipMemcpy(j->d, &h, sizeof(DevJob), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(c, GX_E_DEVICE, "job upload failed"));
  const int mats = heur_mats_of(in->h.kind);
  hipError_t e = gxk::init_jobs(j->d, 1, h.Q, (int)n, mats, c->stream);
  if (e != hipSuccess) return bail(fail(c, GX_E_DEVICE, "init launch: %s", hipGetErrorString(e)));
  if (hipEventCreate(&j->ev0) != hipSuccess || hipEventCreate(&j->ev1) != hipSuccess)
    return bail(fail(c, GX_E_DEVICE, "hipEventCreate failed"));
  c->jobs.push_back(j);
  *out = j;
  return GX_OK;
}

gx_status gx_job_advance(gx_ctx *c, gx_job *j, uint32_t ng) {
  if (!c || !j) return fail(c, GX_E_INVALID, "null argument");
  if (j->batch) return fail(c, GX_E_INVALID, "batched jobs run to completion in gx_solve_batch");
  if (ng == 0) return GX_OK;
  const uint64_t target = (uint64_t)j->g_host + ng;
  if (target > 0xFFFFFFFEull) return fail(c, GX_E_INVALID, "generation counter would exceed 2^32 - 2");
  HIPCHK(c, hipSetDevice(c->dev));
  const uint32_t L = chunks_between(j->g_host, (uint32_t)target, j->h.E);
  HIPCHK(c, gxk::set_stop(j->d, 1, ng, 0, c->stream));
  HIPCHK(c, hipEventRecord(j->ev0, c->stream));
  DevJob *dj = j->d;
  const int kind = j->inst->h.kind, stage = evolve_variant(kind, j->h.stage, j->h.op_mask, j->h.lex_levels, j->h.rows);
  const uint32_t P = j->h.P, lds = j->h.lds_bytes;
  const bool mig = migrates(j->h);
  hipStream_t s = c->stream;
  gx_status st = enqueue_launches(c, j, L, [=]() {
    const hipError_t e = gxk::evolve_plain(dj, kind, stage, P, lds, s);
    return e != hipSuccess ? e : gxk::epoch(dj, nullptr, 1, nullptr, 0, mig, s);
  });
  if (st) return st;
  HIPCHK(c, hipEventRecord(j->ev1, c->stream));
  j->timed = true;
  j->g_host = (uint32_t)target;
  j->launches += L;
  return GX_OK;
}

gx_status gx_solve(gx_ctx *c, const gx_instance *in, const gx_solve_params *p, gx_job **out) {
  if (!p || p->generations == 0) return fail(c, GX_E_INVALID, "generations must be >= 1");
  gx_status st = gx_job_create(c, in, p, out);
  if (st) return st;
  st = gx_job_advance(c, *out, p->generations);
  if (st) {
    gx_job_free(c, *out);
    *out = nullptr;
  }
  return st;
}

gx_status gx_solve_static(gx_ctx *c, const gx_instance *in, const gx_solve_params *p, int32_t *best_solution,
                          int64_t *best_objective) {
  if (!c || !in || !p || !best_solution || !best_objective) return fail(c, GX_E_INVALID, "null argument");
  if (p->generations == 0) return fail(c, GX_E_INVALID, "generations must be >= 1");
  char *ws = (c->dev >= 0 && c->dev < kMaxDevices) ? g_scratch_ptr[c->dev] : nullptr;
  if (!ws) return fail(c, GX_E_DEVICE, "static workspace address unknown on device %d", c->dev);
  HIPCHK(c, hipSetDevice(c->dev));
  uint32_t P_auto = 0;
  gx_status st;
  if (!p->population && (st = gx_autosize_population(c, in, p, &P_auto))) return st;
  DevJob h;
  if ((st = fill_job(c, info_of(in), p, h, P_auto, c->max_lds))) return st;
  if (h.stage == SGLB32 && !in->h.d32)
    return fail(c, GX_E_UNSUPPORTED, "int32 distances of coordinates would need an allocation: choose another staging");
  const size_t n = (size_t)in->h.n;
  const size_t rec = (sizeof(DevJob) + 255) & ~size_t(255);
  const size_t need = rec + job_array_bytes(n, h.P, h.Q, h.lex_levels != 0);
  if (need > kStaticScratchBytes)
    return fail(c, GX_E_UNSUPPORTED, "solve needs %zu bytes of workspace; the static workspace holds %zu", need,
                kStaticScratchBytes);
  DevJob *dj = (DevJob *)ws;
  carve_job(h, ws + rec, n);
  h.best_out = best_solution;
  hipStream_t s = c->stream;
  const bool mig = migrates(h);
  const int kind = in->h.kind, stage = evolve_variant(kind, h.stage, h.op_mask, h.lex_levels, h.rows);
  HIPCHK(c, gxk::write_job(dj, h, s));
  HIPCHK(c, gxk::init_jobs(dj, 1, h.Q, (int)n, heur_mats_of(kind), s));
  HIPCHK(c, gxk::set_stop(dj, 1, 0, 1, s));
  const uint32_t L = chunks_between(0, h.G, h.E);
  for (uint32_t i = 0; i < L; ++i) {
    HIPCHK(c, gxk::evolve_plain(dj, kind, stage, h.P, h.lds_bytes, s));
    HIPCHK(c, gxk::epoch(dj, nullptr, 1, nullptr, 0, mig, s));
  }
  HIPCHK(c, gxk::fetch_best(dj, 1, s));
  HIPCHK(c, gxk::copy_i64(best_objective, (const int64_t *)((char *)dj + offsetof(DevJob, best_out_f)), s));
  return GX_OK;
}

gx_status gx_wait(gx_ctx *c, gx_job *j) {
  if (!c) return GX_E_INVALID;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (j && j->timed) {
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, j->ev0, j->ev1));
    j->evolve_ms = ms;
  }
  return GX_OK;
}

gx_status gx_poll(gx_ctx *c, gx_job *j) {
  if (!c) return GX_E_INVALID;
  const hipError_t e = j && j->timed ? hipEventQuery(j->ev1) : hipStreamQuery(c->stream);
  if (e == hipSuccess) return GX_OK;
  if (e == hipErrorNotReady) return GX_E_NOT_READY;
  return fail(c, GX_E_DEVICE, "poll: %s", hipGetErrorString(e));
}

gx_status gx_fetch_best(gx_ctx *c, gx_job *j, int32_t *sol, int32_t cap, int64_t *obj) {
  if (!c || !j) return fail(c, GX_E_INVALID, "null argument");
  const int n = j->inst->h.n;
  if (sol && cap < n) return fail(c, GX_E_INVALID, "solution buffer holds %d < n = %d", cap, n);
  HIPCHK(c, gxk::fetch_best(j->d, 1, c->stream));
  if (sol) HIPCHK(c, hipMemcpyAsync(sol, j->h.best_out, (size_t)4 * n, hipMemcpyDeviceToHost, c->stream));
  int64_t f = 0;
  HIPCHK(c, hipMemcpyAsync(&f, (char *)j->d + offsetof(DevJob, best_out_f), 8, hipMemcpyDeviceToHost, c->stream));
  gx_status st = gx_wait(c, j);
  if (st) return st;
  if (obj) *obj = f;
  return GX_OK;
}

// a strictly better than b in the lexicographic mode of instance h (the
// penalty exactly, then each level within its tolerance)
static bool lex_better_host(const int64_t a[4], const int64_t b[4], const DevInst &h) {
  if (a[0] != b[0]) return a[0] < b[0];
  for (int i = 0; i < h.lex_levels; ++i) {
    if (a[1 + i] + h.lex_tol[i] < b[1 + i]) return true;
    if (b[1 + i] + h.lex_tol[i] < a[1 + i]) return false;
  }
  return false;
}

gx_status gx_portfolio_best(gx_ctx *c, gx_job *const *jobs, int32_t count, int32_t *sol, int32_t cap, int64_t *obj,
                            int32_t *index) {
  if (!c || !jobs || count < 1 || !obj || !index) return fail(c, GX_E_INVALID, "bad portfolio arguments");
  for (int i = 0; i < count; ++i)
    if (!jobs[i] || jobs[i]->inst != jobs[0]->inst) return fail(c, GX_E_INVALID, "portfolio jobs must share one instance");
  const DevInst &ih = jobs[0]->inst->h;
  int best = 0;
  int64_t fb = 0, vb[4] = {0, 0, 0, 0};
  for (int i = 0; i < count; ++i) {
    int64_t f = 0;
    gx_status st = gx_fetch_best(c, jobs[i], nullptr, 0, &f);
    if (st) return st;
    bool take = i == 0 || f < fb;
    if (ih.lex_levels) {   // the job's reported best vector, compared in job order
      int32_t bi = 0;
      int64_t v[4];
      HIPCHK(c, hipMemcpy(&bi, (char *)jobs[i]->d + offsetof(DevJob, best_idx), 4, hipMemcpyDeviceToHost));
      HIPCHK(c, hipMemcpy(v, jobs[i]->h.best_v + 4 * (size_t)bi, 32, hipMemcpyDeviceToHost));
      take = i == 0 || lex_better_host(v, vb, ih);
      if (take) memcpy(vb, v, sizeof vb);
    }
    if (take) {
      fb = f;
      best = i;
    }
  }
  if (sol) {
    gx_status st = gx_fetch_best(c, jobs[best], sol, cap, &fb);
    if (st) return st;
  }
  *obj = fb;
  *index = best;
  return GX_OK;
}

gx_status gx_job_info_get(gx_ctx *c, gx_job *j, gx_job_info *out) {
  if (!c || !j || !out) return fail(c, GX_E_INVALID, "null argument");
  gx_status st = gx_wait(c, j);
  if (st) return st;
  DevJob h;
  HIPCHK(c, hipMemcpy(&h, j->d, sizeof h, hipMemcpyDeviceToHost));
  out->population = j->h.P;
  out->candidates = j->h.C;
  out->generations_done = h.g;
  out->staging = j->h.stage;
  out->move_evals = (uint64_t)j->h.P * j->h.C * h.g;
  out->accepted = h.accepted;
  out->evolve_launches = j->launches;
  out->evolve_ms = j->evolve_ms;
  const bool every = j->h.credit == 0;   // the totals count evaluated steps only when every candidate credits
  for (int i = 0; i < kOps; ++i) out->op_steps[i] = every ? h.tot_u_op[i] : 0;
  for (int i = 0; i < 3; ++i) out->k_count[i] = every ? h.tot_u_k[i] : 0;
  return GX_OK;
}

gx_status gx_job_stats(gx_ctx *c, gx_job *j, gx_run_stats *out) {
  if (!c || !j || !out) return fail(c, GX_E_INVALID, "null argument");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  DevJob h;
  HIPCHK(c, hipMemcpy(&h, j->d, sizeof h, hipMemcpyDeviceToHost));
  memset(out, 0, sizeof *out);
  out->move_evals = (uint64_t)j->h.P * j->h.C * h.g;
  out->accepted = h.accepted;
  for (int i = 0; i < kOps; ++i) {
    out->u_op[i] = h.tot_u_op[i];
    out->v_op[i] = h.tot_v_op[i];
  }
  for (int i = 0; i < 3; ++i) {
    out->u_k[i] = h.tot_u_k[i];
    out->v_k[i] = h.tot_v_k[i];
  }
  out->generations_done = h.g;
  out->population = j->h.P;
  return GX_OK;
}

gx_status gx_job_population(gx_ctx *c, gx_job *j, uint32_t *out) {
  if (!c || !j || !out) return fail(c, GX_E_INVALID, "null argument");
  *out = j->h.P;
  return GX_OK;
}

gx_status gx_snapshot_aos(gx_ctx *c, gx_job *j, gx_sol_aos *out) {
  if (!c || !j || !out) return fail(c, GX_E_INVALID, "null argument");
  static_assert(sizeof(gx_sol_aos) == sizeof(SolAos), "per-solution record layout");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(out, j->h.saos, sizeof(SolAos) * j->h.P, hipMemcpyDeviceToHost));
  return GX_OK;
}

gx_status gx_snapshot_lex(gx_ctx *c, gx_job *j, int64_t *cur_v, int64_t *best_v, int64_t *ref_v) {
  if (!c || !j) return fail(c, GX_E_INVALID, "null argument");
  if (!j->h.lex_levels) return fail(c, GX_E_INVALID, "the job is not in the lexicographic mode");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const size_t P = j->h.P;
  if (cur_v) HIPCHK(c, hipMemcpy(cur_v, j->h.cur_v, 32 * P, hipMemcpyDeviceToHost));
  if (best_v) HIPCHK(c, hipMemcpy(best_v, j->h.best_v, 32 * P, hipMemcpyDeviceToHost));
  if (ref_v) HIPCHK(c, hipMemcpy(ref_v, (char *)j->d + offsetof(DevJob, ref_v), 32, hipMemcpyDeviceToHost));
  return GX_OK;
}

gx_status gx_snapshot(gx_ctx *c, gx_job *j, gx_state_scalars *sc, int32_t *cur, int64_t *cur_f, int32_t *best,
                      int64_t *best_f) {
  if (!c || !j) return fail(c, GX_E_INVALID, "null argument");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  DevJob h;
  HIPCHK(c, hipMemcpy(&h, j->d, sizeof h, hipMemcpyDeviceToHost));
  const size_t n = (size_t)j->inst->h.n, P = j->h.P;
  if (sc) {
    memset(sc, 0, sizeof *sc);
    sc->g = h.g;
    sc->stag = h.stag;
    sc->T_q16 = h.T;
    sc->epoch_ref = h.epoch_ref;
    for (int i = 0; i < kOps; ++i) {
      sc->w_op[i] = h.w_op[i];
      sc->u_op[i] = h.u_op[i];
      sc->v_op[i] = h.v_op[i];
    }
    for (int i = 0; i < 3; ++i) {
      sc->w_k[i] = h.w_k[i];
      sc->u_k[i] = h.u_k[i];
      sc->v_k[i] = h.v_k[i];
    }
    sc->accepted = h.accepted;
  }
  if (cur) HIPCHK(c, hipMemcpy(cur, h.cur, 4 * n * P, hipMemcpyDeviceToHost));
  if (best) HIPCHK(c, hipMemcpy(best, h.best, 4 * n * P, hipMemcpyDeviceToHost));
  if (cur_f) HIPCHK(c, hipMemcpy(cur_f, h.cur_f, 8 * P, hipMemcpyDeviceToHost));
  if (best_f) HIPCHK(c, hipMemcpy(best_f, h.best_f, 8 * P, hipMemcpyDeviceToHost));
  return GX_OK;
}

// Whether x (n entries) is a solution of the instance: a permutation of
// 0..n-1, bits, or values in [lb, ub].
static bool valid_solution(const DevInst &ih, const int32_t *x, std::vector<char> &seen) {
  const int n = ih.n;
  if (ih.kind == KKNAP) {
    for (int i = 0; i < n; ++i)
      if (x[i] != 0 && x[i] != 1) return false;
    return true;
  }
  if (ih.kind == KCOLOR) {
    for (int i = 0; i < n; ++i)
      if (x[i] < ih.lb || x[i] > ih.ub) return false;
    return true;
  }
  seen.assign((size_t)n, 0);
  for (int i = 0; i < n; ++i) {
    if (x[i] < 0 || x[i] >= n || seen[x[i]]) return false;
    seen[x[i]] = 1;
  }
  // the multi-row form ends with a row marker
  return !ih.rows || x[n - 1] >= ih.dn - 1;
}

gx_status gx_job_restore(gx_ctx *c, gx_job *j, const gx_state_scalars *sc, const int32_t *cur, const int64_t *cur_f,
                         const int32_t *best, const int64_t *best_f, const gx_sol_aos *aos) {
  if (!c || !j || !sc || !cur || !cur_f || !best || !best_f) return fail(c, GX_E_INVALID, "null argument");
  if (j->batch) return fail(c, GX_E_INVALID, "batched jobs cannot be restored");
  if (j->h.lex_levels) return fail(c, GX_E_UNSUPPORTED, "jobs in the lexicographic mode cannot be restored");
  if (j->h.aos_scope == 1 && !aos) return fail(c, GX_E_INVALID, "per-solution weights need their records");
  if (sc->g > 0xFFFFFFFEu) return fail(c, GX_E_INVALID, "generation beyond 2^32 - 2");
  const size_t n = (size_t)j->inst->h.n, P = j->h.P;
  std::vector<char> seen;
  for (size_t s = 0; s < P; ++s)
    if (!valid_solution(j->inst->h, cur + s * n, seen) || !valid_solution(j->inst->h, best + s * n, seen))
      return fail(c, GX_E_INVALID, "solution %zu is not a solution of the instance", s);
  HIPCHK(c, hipSetDevice(c->dev));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  DevJob h;
  HIPCHK(c, hipMemcpy(&h, j->d, sizeof h, hipMemcpyDeviceToHost));
  h.g = h.g_stop = sc->g;
  h.stag = sc->stag;
  h.T = sc->T_q16;
  h.epoch_ref = sc->epoch_ref;
  for (int i = 0; i < kOps; ++i) {
    h.w_op[i] = sc->w_op[i];
    h.u_op[i] = sc->u_op[i];
    h.v_op[i] = sc->v_op[i];
  }
  for (int i = 0; i < 3; ++i) {
    h.w_k[i] = sc->w_k[i];
    h.u_k[i] = sc->u_k[i];
    h.v_k[i] = sc->v_k[i];
  }
  h.accepted = sc->accepted;
  h.inst_best = *std::min_element(best_f, best_f + P);
  HIPCHK(c, hipMemcpy(h.cur, cur, 4 * n * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(h.best, best, 4 * n * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(h.cur_f, cur_f, 8 * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(h.best_f, best_f, 8 * P, hipMemcpyHostToDevice));
  if (j->h.aos_scope == 1) HIPCHK(c, hipMemcpy(h.saos, aos, sizeof(SolAos) * P, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(j->d, &h, sizeof h, hipMemcpyHostToDevice));
  j->g_host = sc->g;
  return GX_OK;
}

static void release_batch(gx_batch *b) {
  if (!b || --b->refs > 0) return;
  (void)hipFree(b->arena);
  (void)hipFree(b->jobs_d);
  (void)hipFree(b->items);
  (void)hipFree(b->next);
  delete b;
}

gx_status gx_job_free(gx_ctx *c, gx_job *j) {
  if (!c || !j) return GX_E_INVALID;
  (void)hipStreamSynchronize(c->stream);
  if (j->gexec) (void)hipGraphExecDestroy(j->gexec);
  if (j->ev0) (void)hipEventDestroy(j->ev0);
  if (j->ev1) (void)hipEventDestroy(j->ev1);
  free_bufs(j->bufs);
  release_batch(j->batch);
  c->jobs.erase(std::remove(c->jobs.begin(), c->jobs.end(), j), c->jobs.end());
  delete j;
  return GX_OK;
}

gx_status gx_destroy(gx_ctx *c) {
  if (!c) return GX_E_INVALID;
  (void)hipSetDevice(c->dev);
  (void)hipStreamSynchronize(c->stream);
  while (!c->jobs.empty()) gx_job_free(c, c->jobs.back());
  while (!c->insts.empty()) gx_instance_free(c, c->insts.back());
  fan_free(c->fan);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return GX_OK;
}

gx_status gx_solve_batch(gx_ctx *c, const gx_instance *const *insts, const gx_solve_params *params, int32_t count,
                         gx_job **jobs_out) {
  if (!c || !insts || !params || !jobs_out || count < 1) return fail(c, GX_E_INVALID, "bad batch arguments");
  HIPCHK(c, hipSetDevice(c->dev));
  std::vector<DevJob> hj((size_t)count);
  std::vector<size_t> off((size_t)count);
  size_t total = 0;
  uint32_t max_q = 0, L = 0;
  int max_n = 1, max_mats = 0;
  size_t n_items = 0;
  for (int i = 0; i < count; ++i) {
    gx_instance *in = const_cast<gx_instance *>(insts[i]);
    if (!in) return fail(c, GX_E_INVALID, "instance %d is null", i);
    const gx_solve_params *p = &params[i];
    if (p->generations == 0) return fail(c, GX_E_INVALID, "job %d: generations must be >= 1", i);
    uint32_t P_auto = 0;
    gx_status st;
    if (!p->population && (st = gx_autosize_population(c, in, p, &P_auto))) return st;
    if ((st = fill_job(c, info_of(in), p, hj[i], P_auto, c->max_lds))) {
      const std::string m = c->err;
      return fail(c, st, "job %d: %s", i, m.c_str());
    }
    if (hj[i].stage == SGLB32 && (st = ensure_d32(c, in))) return st;
    const size_t n = (size_t)in->h.n, P = hj[i].P, Q = hj[i].Q;
    off[i] = total;
    total += job_array_bytes(n, P, Q, hj[i].lex_levels != 0);
    max_q = std::max(max_q, hj[i].Q);
    max_n = std::max(max_n, in->h.n);
    max_mats = std::max(max_mats, heur_mats_of(in->h.kind));
    L = std::max(L, chunks_between(0, hj[i].G, hj[i].E));
    n_items += P;
  }
  if (n_items > 0xFFFFFFFFull) return fail(c, GX_E_UNSUPPORTED, "too many solutions in one batch");
  gx_batch *b = new gx_batch();
  auto bail = [&](gx_status s) {
    (void)hipFree(b->arena);
    (void)hipFree(b->jobs_d);
    (void)hipFree(b->items);
    (void)hipFree(b->next);
    delete b;
    return s;
  };
  char *arena = nullptr;
  if (hipMalloc((void **)&arena, total + 256) != hipSuccess) return bail(fail(c, GX_E_NOMEM, "batch arena of %zu bytes", total));
  b->arena = arena;
  if (hipMalloc((void **)&b->jobs_d, sizeof(DevJob) * count) != hipSuccess)
    return bail(fail(c, GX_E_NOMEM, "batch job table"));
  // work items, grouped by kind and staging, heaviest solutions first
  std::vector<ItemRec> recs;
  recs.reserve(n_items);
  for (int i = 0; i < count; ++i) {
    const DevInst &ih = insts[i]->h;
    const double n = ih.n;
    double cost = n;
    if (ih.kind == KQAP) cost = 4.0 * n * n / 3.0;
    else if (ih.kind == KVRP) cost = 8.0 * n;
    cost *= (double)hj[i].C * (double)hj[i].G;
    for (uint32_t s2 = 0; s2 < hj[i].P; ++s2)
      recs.push_back(ItemRec{ih.kind, evolve_variant(ih.kind, hj[i].stage, hj[i].op_mask, hj[i].lex_levels, hj[i].rows), hj[i].lds_bytes, cost,
                             make_uint2((uint32_t)i, s2)});
  }
  std::vector<uint2> items(n_items);
  std::vector<Group> groups;
  gx_status gst = make_groups(c, recs, items.data(), groups);
  if (gst) return bail(gst);
  if (hipMalloc((void **)&b->items, sizeof(uint2) * n_items) != hipSuccess ||
      hipMalloc((void **)&b->next, sizeof(uint32_t) * kMaxGroups) != hipSuccess)
    return bail(fail(c, GX_E_NOMEM, "batch work items"));
  HIPCHK(c, hipMemsetAsync(b->next, 0, sizeof(uint32_t) * kMaxGroups, c->stream));
  if (groups.size() > 1) HIPCHK(c, fan_init(c->fan));
  for (int i = 0; i < count; ++i) carve_job(hj[i], arena + off[i], (size_t)insts[i]->h.n);
  HIPCHK(c, hipMemcpy(b->jobs_d, hj.data(), sizeof(DevJob) * count, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(b->items, items.data(), sizeof(uint2) * n_items, hipMemcpyHostToDevice));
  HIPCHK(c, gxk::init_jobs(b->jobs_d, count, max_q, max_n, max_mats, c->stream));
  HIPCHK(c, gxk::set_stop(b->jobs_d, count, 0, 1, c->stream));
  // handles
  std::vector<gx_job *> made;
  for (int i = 0; i < count; ++i) {
    gx_job *j = new gx_job();
    j->ctx = c;
    j->inst = const_cast<gx_instance *>(insts[i]);
    j->h = hj[i];
    j->d = b->jobs_d + i;
    j->batch = b;
    j->g_host = hj[i].G;
    b->refs++;
    made.push_back(j);
  }
  gx_job *lead = made[0];
  if (hipEventCreate(&lead->ev0) != hipSuccess || hipEventCreate(&lead->ev1) != hipSuccess)
    return fail(c, GX_E_DEVICE, "hipEventCreate failed");
  HIPCHK(c, hipEventRecord(lead->ev0, c->stream));
  DevJob *jd = b->jobs_d;
  const uint2 *itd = b->items;
  uint32_t *next = b->next;
  hipStream_t s = c->stream;
  const uint32_t njobs = (uint32_t)count;
  const Fan *fan = &c->fan;
  bool mig = false;
  for (int i = 0; i < count; ++i) mig |= migrates(hj[i]);
  gx_status st = enqueue_launches(c, lead, L, [=]() {
    return launch_groups(*fan, groups, jd, itd, next, nullptr, njobs, mig, s);
  });
  if (st) {
    for (gx_job *j : made) delete j;
    return bail(st);
  }
  HIPCHK(c, hipEventRecord(lead->ev1, c->stream));
  lead->timed = true;
  lead->launches = L;
  for (int i = 0; i < count; ++i) {
    c->jobs.push_back(made[i]);
    jobs_out[i] = made[i];
  }
  return GX_OK;
}

}  // extern "C"

// ==================================================================== serving
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over one contiguous region (offsets only), 256-byte granules.
class Arena {
 public:
  explicit Arena(size_t cap = 0) { reset(cap); }
  void reset(size_t cap) {
    free_.clear();
    cap_ = cap & ~size_t(255);
    used_ = 0;
    if (cap_) free_[0] = cap_;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t cap() const { return cap_; }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0;
};

enum ReqState { RQ_PENDING, RQ_RESIDENT, RQ_FETCHING, RQ_DONE, RQ_CANCELLED };

// state and cancel are read by the scheduler thread outside the server mutex
// and written by it and by gx_server_cancel / gx_server_poll: both atomic.
struct SrvReq {
  uint64_t ticket = 0, t_submit = 0, t_done = 0;
  std::atomic<int> state{RQ_PENDING};
  std::atomic<bool> cancel{false};
  Prepared pr;
  DevJob hj{};
  size_t inst_bytes = 0, bytes = 0, off = 0, pin_off = 0;
  size_t pin_bytes = 0;   // pinned block: result (4n + 8), then staging of the instance and the job record
  int slot = -1, n = 0, kind = 0, lane = 0;
  uint32_t g = 0;
  hipEvent_t ev = nullptr;
  std::vector<int32_t> sol;
  int64_t f = 0;
  double cost = 0;
};

// One lane per (kind, staging): its requests advance one epoch chunk per
// quantum on the lane's own stream, so lanes of cheap requests are not held to
// the pace of expensive ones.  Work-item lists are double-buffered.
struct SrvLane {
  hipStream_t s = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  uint2 *items_d[2] = {nullptr, nullptr}, *items_h[2] = {nullptr, nullptr};
  uint32_t *slots_d[2] = {nullptr, nullptr}, *slots_h[2] = {nullptr, nullptr};
  size_t items_cap = 0, slots_cap = 0;
  int buf = 0;
  bool wait_staged = false;
};

// lanes: (kind, staging) x LDS class x 3-opt in the operator set, and the
// VRPTW lexicographic kernels (LDS class x 3-opt)
// one lane per kernel and LDS class: 9 kind-stagings with or without the wide
// variant, VRPTW lexicographic (2), VRPTW multi-row (4: wide, lexicographic),
// and the LNS variants (TSP stagings 4, QAP 2, VRPTW 2)
constexpr int kLaneKernels = 32;
constexpr int kLanes = kLaneKernels * kLdsClasses;
// epoch chunks a lane advances per quantum: the launches and the host's
// turnaround are paid once per quantum, and a newly admitted request joins at
// its lane's next quantum.  An epoch of TSP, knapsack or colouring takes tens
// of microseconds, one of QAP or VRPTW several times more.
inline int quantum_epochs(int kind) { return (kind == KQAP || kind == KVRP) ? 4 : 16; }
int lane_of(int kind, int var, uint32_t lds) {
  const int stage = var & 7;
  const int ks = kind == KTSP ? std::min(std::max(stage, 1), 4) - 1
                              : (kind == KQAP ? 4 + (stage == 1) : (kind == KKNAP ? 6 : (kind == KVRP ? 7 : 8)));
  const int x3 = (var & kVarX3) ? 1 : 0, lex = (var & kVarLex) ? 1 : 0;
  int k;
  if (var & kVarLns) k = 24 + (kind == KVRP ? 6 + lex : ks);   // TSP 0-3, QAP 4-5, VRPTW 6-7
  else if (var & kVarRows) k = 20 + x3 + 2 * lex;
  else if (lex) k = 18 + x3;
  else k = 9 * x3 + ks;
  return k * kLdsClasses + lds_class(lds);
}

}  // namespace

struct gx_server {
  gx_ctx *c = nullptr;
  gx_ctx vctx;   // validation messages (guarded by mu)
  gx_server_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SrvReq *> pending;
  std::unordered_map<uint64_t, SrvReq *> reqs;
  uint64_t next_ticket = 1;
  std::vector<SrvReq *> slots;
  std::vector<int> free_slots;
  DevJob *jobs_d = nullptr;
  SrvLane lanes[kLanes];
  uint32_t *next = nullptr;   // work-item counters, one per lane
  hipEvent_t staged = nullptr;   // after the initialisation of newly admitted requests
  hipEvent_t drain[kLanes] = {};   // lane tails, for retiring a cancelled request
  uint64_t resident_items = 0;   // solutions of the resident requests (guarded by mu)
  gx_ctx gctx;                // device facts and messages of the scheduler thread
  char *arena_d = nullptr;
  Arena arena;
  char *pin = nullptr;
  Arena pin_arena;
  hipStream_t s = nullptr;
  std::thread th;
  std::atomic<bool> stop{false};
  gx_server_stats st{};
  std::string err;
};

namespace {

gx_status lane_grow(SrvLane &L, size_t items, size_t slots) {
  if (items > L.items_cap) {
    const size_t cap = std::max<size_t>(items, 2 * L.items_cap);
    for (int b = 0; b < 2; ++b) {
      (void)hipEventSynchronize(L.ev[b]);
      (void)hipFree(L.items_d[b]);
      (void)hipHostFree(L.items_h[b]);
      L.items_d[b] = nullptr;
      L.items_h[b] = nullptr;
      if (hipMalloc((void **)&L.items_d[b], cap * sizeof(uint2)) != hipSuccess ||
          hipHostMalloc((void **)&L.items_h[b], cap * sizeof(uint2), 0) != hipSuccess)
        return GX_E_NOMEM;
    }
    L.items_cap = cap;
  }
  if (slots > L.slots_cap) {
    const size_t cap = std::max<size_t>(slots, 2 * L.slots_cap);
    for (int b = 0; b < 2; ++b) {
      (void)hipEventSynchronize(L.ev[b]);
      (void)hipFree(L.slots_d[b]);
      (void)hipHostFree(L.slots_h[b]);
      L.slots_d[b] = nullptr;
      L.slots_h[b] = nullptr;
      if (hipMalloc((void **)&L.slots_d[b], cap * sizeof(uint32_t)) != hipSuccess ||
          hipHostMalloc((void **)&L.slots_h[b], cap * sizeof(uint32_t), 0) != hipSuccess)
        return GX_E_NOMEM;
    }
    L.slots_cap = cap;
  }
  return GX_OK;
}

void lane_free(SrvLane &L);

hipError_t lane_init(SrvLane &L) {   // streams and events of a lane, on its first use
  hipError_t e = hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&L.ev[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&L.ev[1], hipEventDisableTiming);
  if (e != hipSuccess) lane_free(L);
  return e;
}

void lane_free(SrvLane &L) {
  for (int b = 0; b < 2; ++b) {
    (void)hipFree(L.items_d[b]);
    (void)hipHostFree(L.items_h[b]);
    (void)hipFree(L.slots_d[b]);
    (void)hipHostFree(L.slots_h[b]);
    if (L.ev[b]) (void)hipEventDestroy(L.ev[b]);
  }
  if (L.s) (void)hipStreamDestroy(L.s);
  L = SrvLane{};
}

// Place an admitted request into its arena block and start its initialisation.
gx_status srv_stage(gx_server *S, SrvReq *r) {
  // the request's completion event belongs to the scheduler thread, which
  // creates, records, queries and destroys it: the submitting and polling
  // threads make no HIP calls
  if (!r->ev && hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
    r->ev = nullptr;
    return GX_E_DEVICE;
  }
  char *base = S->arena_d + r->off;
  // host-side copies go through the request's pinned block (after its result
  // area), so the scheduler thread never waits on a pageable copy
  char *stage = S->pin + r->pin_off + pad16(4 * (size_t)r->n + 8);
  DevInst hh;
  DevInst *dd = nullptr;
  // the scheduler thread's own context for messages (vctx belongs to submitters)
  gx_status st = place_instance(&S->gctx, r->pr, base, S->s, &hh, &dd, stage);
  if (st) return st;
  r->hj.inst = dd;
  carve_job(r->hj, base + r->inst_bytes, (size_t)r->n);
  char *jrec = stage + staging_bytes(r->pr);
  memcpy(jrec, &r->hj, sizeof(DevJob));
  if (hipMemcpyAsync(S->jobs_d + r->slot, jrec, sizeof(DevJob), hipMemcpyHostToDevice, S->s) != hipSuccess ||
      gxk::init_jobs(S->jobs_d + r->slot, 1, r->hj.Q, r->n, heur_mats_of(r->pr.h.kind), S->s) != hipSuccess ||
      gxk::set_stop(S->jobs_d + r->slot, 1, 0, 1, S->s) != hipSuccess)
    return GX_E_DEVICE;
  r->g = 0;
  return GX_OK;
}

void srv_release(gx_server *S, SrvReq *r) {   // caller holds mu
  S->arena.release(r->off, r->bytes);
  if (r->pin_off != (size_t)-1) S->pin_arena.release(r->pin_off, r->pin_bytes);
  S->slots[r->slot] = nullptr;
  S->free_slots.push_back(r->slot);
  S->resident_items -= r->hj.P;
  r->slot = -1;
}

void server_loop(gx_server *S) {
  (void)hipSetDevice(S->c->dev);
  uint64_t busy_since = 0;
  std::vector<SrvReq *> admitted, by_lane[kLanes];
  std::vector<ItemRec> recs;
  std::vector<Group> groups;
  while (!S->stop.load()) {
    admitted.clear();
    bool any_resident = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (auto it = S->pending.begin(); it != S->pending.end() && !S->free_slots.empty();) {
        SrvReq *r = *it;
        // enough solutions resident to fill the device: later requests queue
        // in arrival order instead of slowing down every resident one
        if (S->resident_items + r->hj.P > S->cfg.max_items && S->resident_items > 0) break;
        size_t off = 0, poff = 0;
        if (!S->arena.alloc(r->bytes, &off)) {
          ++it;   // does not fit now; smaller requests behind it may
          continue;
        }
        if (!S->pin_arena.alloc(r->pin_bytes, &poff)) {
          S->arena.release(off, r->bytes);
          ++it;
          continue;
        }
        r->off = off;
        r->pin_off = poff;
        r->slot = S->free_slots.back();
        S->free_slots.pop_back();
        S->slots[r->slot] = r;
        r->state = RQ_RESIDENT;
        S->resident_items += r->hj.P;
        S->st.admitted++;
        admitted.push_back(r);
        it = S->pending.erase(it);
      }
      for (SrvReq *r : S->slots)
        if (r) any_resident = true;
      if (!any_resident && S->pending.empty()) {
        if (busy_since) {
          S->st.busy_seconds += (now_ns() - busy_since) * 1e-9;
          busy_since = 0;
        }
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
    }
    if (!busy_since) busy_since = now_ns();
    if (!admitted.empty()) {
      for (SrvReq *r : admitted)
        if (srv_stage(S, r) != GX_OK) r->cancel = true;   // staging failure: reported as cancelled
      (void)hipEventRecord(S->staged, S->s);
      for (SrvLane &L : S->lanes) L.wait_staged = true;
    }
    // ---- quanta: every lane whose older work-item buffer is free advances its
    // running requests by one epoch chunk
    for (auto &v : by_lane) v.clear();
    for (SrvReq *r : S->slots)
      if (r && r->state == RQ_RESIDENT && !r->cancel && r->g < r->hj.G) by_lane[r->lane].push_back(r);
    bool progressed = false;
    uint64_t evals = 0, quanta = 0;
    for (int li = 0; li < kLanes; ++li) {
      SrvLane &L = S->lanes[li];
      std::vector<SrvReq *> &act = by_lane[li];
      if (act.empty()) continue;
      if (!L.s && lane_init(L) != hipSuccess) continue;
      if (hipEventQuery(L.ev[L.buf]) != hipSuccess) continue;
      size_t n_items = 0;
      for (SrvReq *r : act) n_items += r->hj.P;
      if (lane_grow(L, n_items, act.size()) != GX_OK) continue;
      const int b = L.buf;
      recs.clear();
      for (SrvReq *r : act)
        for (uint32_t sl = 0; sl < r->hj.P; ++sl)
          recs.push_back(ItemRec{r->kind, evolve_variant(r->kind, r->hj.stage, r->hj.op_mask, r->hj.lex_levels, r->hj.rows), r->hj.lds_bytes, r->cost,
                                 make_uint2((uint32_t)r->slot, sl)});
      if (make_groups(&S->gctx, recs, L.items_h[b], groups) != GX_OK || groups.size() != 1) continue;
      for (size_t a = 0; a < act.size(); ++a) L.slots_h[b][a] = (uint32_t)act[a]->slot;
      if (L.wait_staged) {
        (void)hipStreamWaitEvent(L.s, S->staged, 0);
        L.wait_staged = false;
      }
      (void)hipMemcpyAsync(L.items_d[b], L.items_h[b], n_items * sizeof(uint2), hipMemcpyHostToDevice, L.s);
      (void)hipMemcpyAsync(L.slots_d[b], L.slots_h[b], act.size() * sizeof(uint32_t), hipMemcpyHostToDevice, L.s);
      const Group &g = groups[0];
      // requests that finish inside the quantum skip its remaining launches
      // (their generation window is empty)
      const int qe = S->cfg.quantum_epochs ? (int)S->cfg.quantum_epochs : quantum_epochs(g.kind);
      bool mig = false;
      for (SrvReq *r : act) mig |= migrates(r->hj);
      for (int q = 0; q < qe; ++q) {
        (void)gxk::evolve_group(g.kind, g.stage, S->jobs_d, L.items_d[b], g.count, S->next + li, g.grid, g.lds, L.s);
        (void)gxk::epoch(S->jobs_d, L.slots_d[b], (uint32_t)act.size(), S->next + li, 1, mig, L.s);
      }
      for (SrvReq *r : act) {
        const uint32_t E = r->hj.E;
        const uint32_t ng = (uint32_t)std::min<uint64_t>(r->hj.G, ((uint64_t)r->g / E + qe) * E);
        evals += (uint64_t)r->hj.P * r->hj.C * (ng - r->g);
        r->g = ng;
        if (r->g == r->hj.G) {   // finished: fetch the best solution asynchronously
          (void)gxk::fetch_best(S->jobs_d + r->slot, 1, L.s);
          char *dst = S->pin + r->pin_off;
          (void)hipMemcpyAsync(dst, r->hj.best_out, 4 * (size_t)r->n, hipMemcpyDeviceToHost, L.s);
          (void)hipMemcpyAsync(dst + 4 * (size_t)r->n, (char *)(S->jobs_d + r->slot) + offsetof(DevJob, best_out_f),
                               8, hipMemcpyDeviceToHost, L.s);
          (void)hipEventRecord(r->ev, L.s);
          r->state = RQ_FETCHING;
        }
      }
      (void)hipEventRecord(L.ev[b], L.s);
      L.buf ^= 1;
      progressed = true;
      ++quanta;
    }
    if (quanta) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.quanta += quanta;
      S->st.move_evals += evals;
    }
    // cancelled residents: retire after all work enqueued so far has drained
    for (SrvReq *r : S->slots)
      if (r && r->cancel && r->state == RQ_RESIDENT) {
        for (int li = 0; li < kLanes; ++li) {
          if (!S->lanes[li].s) continue;
          (void)hipEventRecord(S->drain[li], S->lanes[li].s);
          (void)hipStreamWaitEvent(S->s, S->drain[li], 0);
        }
        if (r->ev) (void)hipEventRecord(r->ev, S->s);
        else (void)hipStreamSynchronize(S->s);   // no event (its creation failed): drain here
        r->state = RQ_FETCHING;
      }
    // completions
    bool done_any = false;
    for (SrvReq *r : S->slots) {
      if (!r || r->state != RQ_FETCHING) continue;
      if (r->ev && hipEventQuery(r->ev) != hipSuccess) continue;
      if (r->ev) (void)hipEventDestroy(r->ev);   // complete: the scheduler's last use of it
      r->ev = nullptr;
      std::lock_guard<std::mutex> lk(S->mu);
      if (!r->cancel) {
        const char *src = S->pin + r->pin_off;
        r->sol.assign((const int32_t *)src, (const int32_t *)src + r->n);
        memcpy(&r->f, src + 4 * (size_t)r->n, 8);
        r->state = RQ_DONE;
        S->st.completed++;
      } else {
        r->state = RQ_CANCELLED;
        S->st.cancelled++;
      }
      r->t_done = now_ns();
      srv_release(S, r);
      done_any = true;
    }
    if (!progressed && !done_any) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  for (SrvLane &L : S->lanes)
    if (L.s) (void)hipStreamSynchronize(L.s);
  (void)hipStreamSynchronize(S->s);
}

}  // namespace

extern "C" {

gx_status gx_server_create(gx_ctx *c, const gx_server_cfg *cfg, gx_server **out) {
  if (!c || !out) return fail(c, GX_E_INVALID, "null argument");
  *out = nullptr;
  HIPCHK(c, hipSetDevice(c->dev));
  gx_server *S = new gx_server();
  S->c = c;
  S->vctx.dev = c->dev;
  S->vctx.info = c->info;
  S->vctx.max_lds = c->max_lds;
  S->cfg.hbm_budget_bytes = cfg && cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (1ull << 30);
  S->cfg.max_resident = cfg && cfg->max_resident ? cfg->max_resident : 1024;
  S->cfg.max_lds_bytes = cfg && cfg->max_lds_bytes ? std::min(cfg->max_lds_bytes, c->max_lds) : std::min(65536u, c->max_lds);
  S->cfg.max_items = cfg && cfg->max_items ? cfg->max_items : 40u * c->info.cus;
  S->cfg.quantum_epochs = cfg ? cfg->quantum_epochs : 0;
  if (S->cfg.quantum_epochs > 1024) {
    delete S;
    return fail(c, GX_E_INVALID, "quantum_epochs <= 1024");
  }
  S->gctx.dev = c->dev;
  S->gctx.info = c->info;
  S->gctx.max_lds = c->max_lds;
  auto bail = [&](const char *what) {
    (void)hipFree(S->arena_d);
    (void)hipFree(S->jobs_d);
    (void)hipFree(S->next);
    (void)hipHostFree(S->pin);
    for (SrvLane &L : S->lanes) lane_free(L);
    for (hipEvent_t &e : S->drain)
      if (e) (void)hipEventDestroy(e);
    if (S->staged) (void)hipEventDestroy(S->staged);
    if (S->s) (void)hipStreamDestroy(S->s);
    delete S;
    return fail(c, GX_E_NOMEM, "server: %s", what);
  };
  if (hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) != hipSuccess) return bail("stream");
  if (hipEventCreateWithFlags(&S->staged, hipEventDisableTiming) != hipSuccess) return bail("events");
  for (int li = 0; li < kLanes; ++li)
    if (hipEventCreateWithFlags(&S->drain[li], hipEventDisableTiming) != hipSuccess) return bail("events");
  if (hipMalloc((void **)&S->next, sizeof(uint32_t) * kLanes) != hipSuccess ||
      hipMemset(S->next, 0, sizeof(uint32_t) * kLanes) != hipSuccess)
    return bail("work-item counters");
  if (hipMalloc((void **)&S->arena_d, S->cfg.hbm_budget_bytes) != hipSuccess) return bail("arena");
  S->arena.reset(S->cfg.hbm_budget_bytes);
  if (hipMalloc((void **)&S->jobs_d, sizeof(DevJob) * S->cfg.max_resident) != hipSuccess) return bail("job table");
  // per resident request: its result and the staging copy of its instance
  const size_t pin_bytes = std::max<size_t>(64u << 20, (size_t)S->cfg.max_resident * 16384);
  if (hipHostMalloc((void **)&S->pin, pin_bytes, 0) != hipSuccess) return bail("pinned results");
  S->pin_arena.reset(pin_bytes);
  S->slots.assign(S->cfg.max_resident, nullptr);
  for (int i = (int)S->cfg.max_resident - 1; i >= 0; --i) S->free_slots.push_back(i);
  S->st.arena_bytes = S->arena.cap();
  S->th = std::thread(server_loop, S);
  *out = S;
  return GX_OK;
}

gx_status gx_server_submit(gx_server *S, const gx_instance_desc *d, const gx_solve_params *p, uint64_t *ticket) {
  if (!S || !d || !p || !ticket) return GX_E_INVALID;
  if (d->is_device_ptr) return GX_E_INVALID;
  SrvReq *r = new SrvReq();
  std::unique_lock<std::mutex> lk(S->mu);
  gx_status st = prepare_instance(&S->vctx, d, r->pr, false);
  if (!st && p->population == 0) st = fail(&S->vctx, GX_E_INVALID, "served requests need a population");
  if (!st && p->generations == 0) st = fail(&S->vctx, GX_E_INVALID, "generations must be >= 1");
  if (!st) {
    InstInfo ii{r->pr.h, nullptr, false, false, r->pr.h.has_xy != 0, r->pr.key};
    for (const auto &a : r->pr.arrs) {
      ii.has_d16 |= a.field == F_D16;
      ii.has_d32 |= a.field == F_D32;
    }
    st = fill_job(&S->vctx, ii, p, r->hj, 0, S->cfg.max_lds_bytes);
    if (!st && r->hj.stage == SGLB32 && !ii.has_d32) st = fail(&S->vctx, GX_E_UNSUPPORTED, "int32 staging needs a matrix");
  }
  if (st) {
    S->err = S->vctx.err;
    delete r;
    return st;
  }
  r->n = r->pr.h.n;
  r->inst_bytes = (r->pr.dev_bytes() + 255) & ~size_t(255);
  r->bytes = r->inst_bytes + job_array_bytes((size_t)r->n, r->hj.P, r->hj.Q, r->hj.lex_levels != 0);
  r->pin_bytes = pad16(4 * (size_t)r->n + 8) + staging_bytes(r->pr) + pad16(sizeof(DevJob));
  if (r->bytes > S->arena.cap() || r->pin_bytes > S->pin_arena.cap()) {
    S->err = "request larger than the server arena";
    delete r;
    return GX_E_UNSUPPORTED;
  }
  const double n = r->n;
  r->cost = (r->pr.h.kind == KQAP ? 4.0 * n * n / 3.0 : (r->pr.h.kind == KVRP ? 8.0 * n : n)) * r->hj.C;
  r->kind = r->pr.h.kind;
  r->lane = lane_of(r->kind, evolve_variant(r->kind, r->hj.stage, r->hj.op_mask, r->hj.lex_levels, r->hj.rows), r->hj.lds_bytes);
  r->ticket = S->next_ticket++;
  r->t_submit = now_ns();
  S->reqs[r->ticket] = r;
  S->pending.push_back(r);
  S->st.submitted++;
  *ticket = r->ticket;
  lk.unlock();
  S->cv.notify_one();
  return GX_OK;
}

gx_status gx_server_poll(gx_server *S, uint64_t ticket, int32_t *sol, int32_t cap, int64_t *obj, uint64_t *t_sub,
                         uint64_t *t_done) {
  if (!S) return GX_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return GX_E_INVALID;
  SrvReq *r = it->second;
  if (r->state == RQ_CANCELLED) {
    S->reqs.erase(it);
    delete r;
    return GX_E_CANCELLED;
  }
  if (r->state != RQ_DONE) return GX_E_NOT_READY;
  if (sol && cap < r->n) return GX_E_INVALID;
  if (sol) memcpy(sol, r->sol.data(), 4 * (size_t)r->n);
  if (obj) *obj = r->f;
  if (t_sub) *t_sub = r->t_submit;
  if (t_done) *t_done = r->t_done;
  S->reqs.erase(it);
  delete r;
  return GX_OK;
}

gx_status gx_server_cancel(gx_server *S, uint64_t ticket) {
  if (!S) return GX_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return GX_E_INVALID;
  SrvReq *r = it->second;
  if (r->state == RQ_PENDING) {
    S->pending.erase(std::remove(S->pending.begin(), S->pending.end(), r), S->pending.end());
    r->state = RQ_CANCELLED;
    S->st.cancelled++;
  } else if (r->state == RQ_RESIDENT || r->state == RQ_FETCHING) {
    r->cancel = true;
  }
  return GX_OK;
}

gx_status gx_server_stats_get(gx_server *S, gx_server_stats *out) {
  if (!S || !out) return GX_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  out->pending = (uint32_t)S->pending.size();
  uint32_t res = 0;
  for (SrvReq *r : S->slots) res += r != nullptr;
  out->resident = res;
  out->arena_used_bytes = S->arena.used();
  out->arena_bytes = S->arena.cap();
  return GX_OK;
}

gx_status gx_server_destroy(gx_server *S) {
  if (!S) return GX_E_INVALID;
  S->stop.store(true);
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipStreamSynchronize(S->s);
  for (auto &kv : S->reqs) {   // the scheduler has stopped: its events are freed here
    if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
    delete kv.second;
  }
  for (SrvLane &L : S->lanes) lane_free(L);
  for (hipEvent_t e : S->drain) (void)hipEventDestroy(e);
  (void)hipEventDestroy(S->staged);
  (void)hipFree(S->arena_d);
  (void)hipFree(S->jobs_d);
  (void)hipFree(S->next);
  (void)hipHostFree(S->pin);
  (void)hipStreamDestroy(S->s);
  delete S;
  return GX_OK;
}

}  // extern "C"
