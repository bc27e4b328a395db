// gx_api.hip -- host runtime behind the C interface in include/gx.h:
// device checks, instance staging, job allocation, launch planning (one
// evolve launch per AOS epoch chunk, replayed from a captured HIP graph),
// results and snapshots.
#include "../../include/gx.h"
#include "gx_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace gx;

struct gx_ctx {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
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

uint32_t encoding_ops(int kind) {
  if (kind == KKNAP) return 1u << OFLIP;
  if (kind == KCOLOR) return 1u << ORESET;
  return (1u << O2OPT) | (1u << OSWAP) | (1u << OINS) | (1u << OOROPT);
}

void free_bufs(std::vector<void *> &b) {
  for (void *p : b) (void)hipFree(p);
  b.clear();
}

}  // namespace

extern "C" {

gx_status gx_exp_tables(uint32_t hi[16], uint32_t lo[256]) {
  if (!hi || !lo) return GX_E_INVALID;
  make_exp_tables(hi, lo);
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
      prop.warpSize != kWave) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return GX_E_DEVICE;
  }
  *out = c;
  return GX_OK;
}

const char *gx_last_error(const gx_ctx *c) { return c ? c->err.c_str() : "null context"; }

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
  const int n = d->n;
  if (n < 1) return fail(c, GX_E_INVALID, "n must be >= 1 (got %d)", n);
  HIPCHK(c, hipSetDevice(c->dev));
  gx_instance *in = new gx_instance();
  DevInst &h = in->h;
  h.kind = d->kind;
  h.n = n;
  h.lb = d->lb;
  h.ub = d->ub;
  h.capacity = d->capacity;
  h.vehicles = d->vehicles;
  h.service = d->service_time;
  h.horizon = d->horizon;
  h.n_edges = d->n_edges;
  std::vector<int32_t> A, B;
  gx_status st = GX_OK;
  auto bail = [&](gx_status s) {
    free_bufs(in->bufs);
    delete in;
    return s;
  };
  auto up = [&](void *dst, const void *src, size_t bytes) -> gx_status {
    HIPCHK(c, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    return GX_OK;
  };
  double fbound = 0;
  if (d->kind == KTSP) {
    if (n > 65535) return bail(fail(c, GX_E_UNSUPPORTED, "TSP n <= 65535"));
    if (d->a_is_coords) {
      if ((st = to_host(c, d, d->a, (size_t)2 * n, A))) return bail(st);
      for (int32_t v : A)
        if (v < 0 || v >= kMaxCoord) return bail(fail(c, GX_E_INVALID, "coordinates must lie in [0, 16384)"));
      int32_t *xy;
      if ((st = dalloc(c, in->bufs, &xy, (size_t)8 * n)) || (st = up(xy, A.data(), (size_t)8 * n))) return bail(st);
      h.xy = xy;
      h.has_xy = 1;
      if (n <= 4096) {
        int16_t *d16;
        if ((st = dalloc(c, in->bufs, &d16, (size_t)2 * n * n))) return bail(st);
        HIPCHK(c, gxk::build_tsp_d16_from_xy(xy, n, d16, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        h.d16 = d16;
      }
      in->max_d = 23171;
    } else {
      if ((st = to_host(c, d, d->a, (size_t)n * n, A))) return bail(st);
      int mx = 0;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const int32_t v = A[(size_t)i * n + j];
          if (v < 0 || v >= (1 << 24) || v != A[(size_t)j * n + i] || (i == j && v != 0))
            return bail(fail(c, GX_E_INVALID, "TSP matrix must be symmetric, zero-diagonal, in [0, 2^24)"));
          mx = std::max(mx, v);
        }
      in->max_d = mx;
      int32_t *d32;
      if ((st = dalloc(c, in->bufs, &d32, (size_t)4 * n * n)) || (st = up(d32, A.data(), (size_t)4 * n * n)))
        return bail(st);
      h.d32 = d32;
      if (mx < 32768) {
        std::vector<int16_t> s16(A.begin(), A.end());
        int16_t *d16;
        if ((st = dalloc(c, in->bufs, &d16, (size_t)2 * n * n)) || (st = up(d16, s16.data(), (size_t)2 * n * n)))
          return bail(st);
        h.d16 = d16;
      }
    }
    fbound = 6.0 * n * (double)std::max(in->max_d, 1);
  } else if (d->kind == KQAP) {
    if (n > kMaxQapN) return bail(fail(c, GX_E_UNSUPPORTED, "QAP n <= %d", kMaxQapN));
    if ((st = to_host(c, d, d->a, (size_t)n * n, A)) || (st = to_host(c, d, d->b, (size_t)n * n, B))) return bail(st);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t ij = (size_t)i * n + j, ji = (size_t)j * n + i;
        if (A[ij] < 0 || A[ij] >= 16384 || B[ij] < 0 || B[ij] >= 16384 || A[ij] != A[ji] || B[ij] != B[ji])
          return bail(fail(c, GX_E_INVALID, "QAP matrices must be symmetric with entries in [0, 16384)"));
      }
    std::vector<int16_t> F(A.begin(), A.end()), D(B.begin(), B.end());
    int16_t *qf, *qd;
    if ((st = dalloc(c, in->bufs, &qf, (size_t)2 * n * n)) || (st = dalloc(c, in->bufs, &qd, (size_t)2 * n * n)) ||
        (st = up(qf, F.data(), (size_t)2 * n * n)) || (st = up(qd, D.data(), (size_t)2 * n * n)))
      return bail(st);
    h.qf = qf;
    h.qd = qd;
    fbound = 4.0 * n * n * 16384.0 * 16384.0;
  } else if (d->kind == KKNAP) {
    if (n > 16384) return bail(fail(c, GX_E_UNSUPPORTED, "knapsack n <= 16384"));
    if ((st = to_host(c, d, d->a, (size_t)n, A)) || (st = to_host(c, d, d->b, (size_t)n, B))) return bail(st);
    int64_t mv = 0, sw = 0, sv = 0;
    for (int i = 0; i < n; ++i) {
      if (A[i] < 0 || A[i] > (1 << 20) || B[i] < 0 || B[i] > (1 << 20))
        return bail(fail(c, GX_E_INVALID, "knapsack weights and values must lie in [0, 2^20]"));
      mv = std::max<int64_t>(mv, B[i]);
      sw += A[i];
      sv += B[i];
    }
    if (d->capacity < 0) return bail(fail(c, GX_E_INVALID, "capacity must be >= 0"));
    h.lambda = mv + 1;
    int32_t *kw, *kv;
    if ((st = dalloc(c, in->bufs, &kw, (size_t)4 * n)) || (st = dalloc(c, in->bufs, &kv, (size_t)4 * n)) ||
        (st = up(kw, A.data(), (size_t)4 * n)) || (st = up(kv, B.data(), (size_t)4 * n)))
      return bail(st);
    h.kw = kw;
    h.kv = kv;
    fbound = 4.0 * ((double)sv + (double)h.lambda * (double)sw);
  } else if (d->kind == KVRP) {
    if (n > kMaxVrpN) return bail(fail(c, GX_E_UNSUPPORTED, "VRPTW n <= %d", kMaxVrpN));
    const int m = n + 1;
    if ((st = to_host(c, d, d->a, (size_t)2 * m, A)) || (st = to_host(c, d, d->b, (size_t)3 * m, B))) return bail(st);
    for (int32_t v : A)
      if (v < 0 || v >= kMaxCoord) return bail(fail(c, GX_E_INVALID, "coordinates must lie in [0, 16384)"));
    for (int i = 0; i < m; ++i) {
      const int32_t q = B[i], r = B[m + i], u = B[2 * m + i];
      if (q < 0 || q > d->capacity || r < 0 || u < 0 || r > (1 << 19) || u > (1 << 19))
        return bail(fail(c, GX_E_INVALID, "VRPTW demand in [0, capacity], times in [0, 2^19]"));
    }
    if (d->capacity < 1 || d->vehicles < 1 || d->service_time < 0 || d->service_time > (1 << 16) ||
        d->horizon < 0 || d->horizon > (1 << 19))
      return bail(fail(c, GX_E_INVALID, "VRPTW capacity, vehicles >= 1; service <= 2^16; horizon in [0, 2^19]"));
    h.dn = m;
    int32_t *xy, *dem, *rdy, *due;
    int16_t *d16;
    if ((st = dalloc(c, in->bufs, &xy, (size_t)8 * m)) || (st = up(xy, A.data(), (size_t)8 * m)) ||
        (st = dalloc(c, in->bufs, &d16, (size_t)2 * m * m)) || (st = dalloc(c, in->bufs, &dem, (size_t)4 * m)) ||
        (st = dalloc(c, in->bufs, &rdy, (size_t)4 * m)) || (st = dalloc(c, in->bufs, &due, (size_t)4 * m)) ||
        (st = up(dem, B.data(), (size_t)4 * m)) || (st = up(rdy, B.data() + m, (size_t)4 * m)) ||
        (st = up(due, B.data() + 2 * m, (size_t)4 * m)))
      return bail(st);
    HIPCHK(c, gxk::build_tsp_d16_from_xy(xy, m, d16, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    h.xy = xy;
    h.has_xy = 1;
    h.d16 = d16;
    h.dem = dem;
    h.rdy = rdy;
    h.due = due;
    fbound = 4.0 * (m * 23171.0 + 100.0 * m * (m * 23171.0 + (1 << 19) + (double)m * (1 << 16)) + 10000.0 * m);
  } else if (d->kind == KCOLOR) {
    if (n > 32767) return bail(fail(c, GX_E_UNSUPPORTED, "colouring n <= 32767"));
    if (d->lb > d->ub || d->lb < -32768 || d->ub > 32767)
      return bail(fail(c, GX_E_INVALID, "colouring needs -32768 <= lb <= ub <= 32767"));
    if (d->n_edges < 0 || d->n_edges > (1 << 20)) return bail(fail(c, GX_E_INVALID, "n_edges in [0, 2^20]"));
    if ((st = to_host(c, d, d->a, (size_t)2 * d->n_edges, A))) return bail(st);
    std::vector<int32_t> off(n + 1, 0), adj((size_t)2 * d->n_edges);
    for (int e = 0; e < d->n_edges; ++e) {
      const int u = A[2 * e], v = A[2 * e + 1];
      if (u < 0 || v < 0 || u >= n || v >= n || u == v)
        return bail(fail(c, GX_E_INVALID, "edge %d out of range or a self loop", e));
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
    int32_t *po, *pa, *pe;
    if ((st = dalloc(c, in->bufs, &po, (size_t)4 * (n + 1))) || (st = up(po, off.data(), (size_t)4 * (n + 1))) ||
        (st = dalloc(c, in->bufs, &pa, std::max<size_t>(16, adj.size() * 4))) ||
        (st = dalloc(c, in->bufs, &pe, std::max<size_t>(16, A.size() * 4))))
      return bail(st);
    if (!adj.empty() && ((st = up(pa, adj.data(), adj.size() * 4)) || (st = up(pe, A.data(), A.size() * 4))))
      return bail(st);
    h.adj_off = po;
    h.adj = pa;
    h.edges = pe;
    fbound = 4.0 * d->n_edges + 4;
  } else {
    return bail(fail(c, GX_E_INVALID, "unknown problem kind %d", d->kind));
  }
  if (fbound >= std::ldexp(1.0, 45)) return bail(fail(c, GX_E_UNSUPPORTED, "objective range exceeds 2^45"));
  DevInst *dd;
  if ((st = dalloc(c, in->bufs, &dd, sizeof(DevInst))) || (st = up(dd, &h, sizeof(DevInst)))) return bail(st);
  in->d = dd;
  in->key = d->instance_key;
  c->insts.push_back(in);
  *out = in;
  return GX_OK;
}

}  // extern "C"

namespace {

uint32_t resolve_stage(const gx_instance *in, uint32_t req) {
  if (in->h.kind != KTSP) return 0;
  if (req != SAUTO) return req;
  const int n = in->h.n;
  if (n <= 128 && in->h.d16) return SLDS16;
  if (in->h.has_xy) return SLDSXY;
  if (in->h.d16) return SGLB16;
  return SGLB32;
}

uint32_t job_lds(const gx_instance *in, uint32_t stage) {
  uint32_t b = lds_bytes_for(in->h.kind, in->h.n, (int)stage);
  if (in->h.kind == KCOLOR) b += (uint32_t)pad16((size_t)8 * in->h.n_edges);
  return std::max<uint32_t>(b, 16);
}

// Validate parameters and fill the constant part of a DevJob.
gx_status fill_job(gx_ctx *c, gx_instance *in, const gx_solve_params *p, DevJob &h, uint32_t P_auto) {
  if (!p) return fail(c, GX_E_INVALID, "null parameters");
  const uint32_t mask = p->op_mask ? (p->op_mask & encoding_ops(in->h.kind)) : encoding_ops(in->h.kind);
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
  const uint32_t stage = resolve_stage(in, p->staging);
  if (in->h.kind == KTSP) {
    if ((stage == SLDS16 || stage == SGLB16) && !in->h.d16)
      return fail(c, GX_E_UNSUPPORTED, "no int16 distance matrix for this instance");
    if (stage == SLDSXY && !in->h.has_xy) return fail(c, GX_E_UNSUPPORTED, "coordinates-in-LDS needs coordinates");
  }
  const uint32_t lds = job_lds(in, stage);
  if (lds > c->max_lds)
    return fail(c, GX_E_UNSUPPORTED, "instance needs %u bytes of LDS per workgroup (device has %u)", lds, c->max_lds);
  memset(&h, 0, sizeof h);
  h.inst = in->d;
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
  h.key = in->key;
  h.alpha = p->alpha_q32;
  h.Q = K * P;
  h.stage = stage;
  h.lds_bytes = lds;
  return GX_OK;
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
  const uint32_t stage = resolve_stage(in, p ? p->staging : 0);
  const uint32_t lds = job_lds(in, stage);
  int occ = 0;
  HIPCHK(c, gxk::occupancy_plain(in->h.kind, (int)stage, lds, &occ));
  occ = std::max(1, std::min(occ, 8));
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
  if ((st = fill_job(c, in, p, h, P_auto))) return bail(st);
  if (h.stage == SGLB32 && (st = ensure_d32(c, in))) return bail(st);
  const size_t n = (size_t)in->h.n;
  if ((st = dalloc(c, j->bufs, &h.cur, 4 * n * h.P)) || (st = dalloc(c, j->bufs, &h.best, 4 * n * h.P)) ||
      (st = dalloc(c, j->bufs, &h.cur_f, (size_t)8 * h.P)) || (st = dalloc(c, j->bufs, &h.best_f, (size_t)8 * h.P)) ||
      (st = dalloc(c, j->bufs, &h.pool, 4 * n * h.Q)) || (st = dalloc(c, j->bufs, &h.pool_f, (size_t)8 * h.Q)) ||
      (st = dalloc(c, j->bufs, &h.sums, 32 * n)) || (st = dalloc(c, j->bufs, &h.best_out, 4 * n)) ||
      (st = dalloc(c, j->bufs, &j->d, sizeof(DevJob))))
    return bail(st);
  if (hipMemcpy(j->d, &h, sizeof(DevJob), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(c, GX_E_DEVICE, "job upload failed"));
  const int mats = in->h.kind == KQAP ? 2 : ((in->h.kind == KTSP || in->h.kind == KVRP) ? 1 : 0);
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
  const int kind = j->inst->h.kind, stage = (int)j->h.stage;
  const uint32_t P = j->h.P, lds = j->h.lds_bytes;
  hipStream_t s = c->stream;
  gx_status st = enqueue_launches(c, j, L, [=]() { return gxk::evolve_plain(dj, kind, stage, P, lds, s); });
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
  for (int i = 0; i < kOps; ++i) out->op_steps[i] = h.tot_u_op[i];
  for (int i = 0; i < 3; ++i) out->k_count[i] = h.tot_u_k[i];
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

static void release_batch(gx_batch *b) {
  if (!b || --b->refs > 0) return;
  (void)hipFree(b->arena);
  (void)hipFree(b->jobs_d);
  (void)hipFree(b->items);
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
  uint32_t max_q = 0, max_lds = 16, L = 0;
  int max_n = 1, max_mats = 0;
  size_t n_items = 0;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  for (int i = 0; i < count; ++i) {
    gx_instance *in = const_cast<gx_instance *>(insts[i]);
    if (!in) return fail(c, GX_E_INVALID, "instance %d is null", i);
    const gx_solve_params *p = &params[i];
    if (p->generations == 0) return fail(c, GX_E_INVALID, "job %d: generations must be >= 1", i);
    uint32_t P_auto = 0;
    gx_status st;
    if (!p->population && (st = gx_autosize_population(c, in, p, &P_auto))) return st;
    if ((st = fill_job(c, in, p, hj[i], P_auto))) return fail(c, st, "job %d: %s", i, c->err.c_str());
    if (hj[i].stage == SGLB32 && (st = ensure_d32(c, in))) return st;
    const size_t n = (size_t)in->h.n, P = hj[i].P, Q = hj[i].Q;
    off[i] = total;
    total += 2 * al(4 * n * P) + 2 * al(8 * P) + al(4 * n * Q) + al(8 * Q) + al(32 * n) + al(4 * n);
    max_q = std::max(max_q, hj[i].Q);
    max_lds = std::max(max_lds, hj[i].lds_bytes);
    max_n = std::max(max_n, in->h.n);
    max_mats = std::max(max_mats, in->h.kind == KQAP ? 2 : ((in->h.kind == KTSP || in->h.kind == KVRP) ? 1 : 0));
    L = std::max(L, chunks_between(0, hj[i].G, hj[i].E));
    n_items += P;
  }
  if (n_items > 0xFFFFFFFFull) return fail(c, GX_E_UNSUPPORTED, "too many solutions in one batch");
  gx_batch *b = new gx_batch();
  auto bail = [&](gx_status s) {
    (void)hipFree(b->arena);
    (void)hipFree(b->jobs_d);
    (void)hipFree(b->items);
    delete b;
    return s;
  };
  char *arena = nullptr;
  if (hipMalloc((void **)&arena, total + 256) != hipSuccess) return bail(fail(c, GX_E_NOMEM, "batch arena of %zu bytes", total));
  b->arena = arena;
  if (hipMalloc((void **)&b->jobs_d, sizeof(DevJob) * count) != hipSuccess)
    return bail(fail(c, GX_E_NOMEM, "batch job table"));
  // work items, heaviest solutions first so that the tail of a launch is short
  std::vector<std::pair<double, uint2>> it;
  it.reserve(n_items);
  for (int i = 0; i < count; ++i) {
    const DevInst &ih = insts[i]->h;
    const double n = ih.n;
    double cost = n;
    if (ih.kind == KQAP) cost = 4.0 * n * n / 3.0;
    else if (ih.kind == KVRP) cost = 8.0 * n;
    cost *= (double)hj[i].C * (double)hj[i].G;
    for (uint32_t s2 = 0; s2 < hj[i].P; ++s2) it.push_back({-cost, make_uint2((uint32_t)i, s2)});
  }
  std::stable_sort(it.begin(), it.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
  std::vector<uint2> items(n_items);
  for (size_t k = 0; k < n_items; ++k) items[k] = it[k].second;
  if (hipMalloc((void **)&b->items, sizeof(uint2) * n_items) != hipSuccess)
    return bail(fail(c, GX_E_NOMEM, "batch work items"));
  for (int i = 0; i < count; ++i) {
    const size_t n = (size_t)insts[i]->h.n, P = hj[i].P, Q = hj[i].Q;
    char *q = arena + off[i];
    auto take = [&](size_t bytes) {
      char *r = q;
      q += al(bytes);
      return r;
    };
    hj[i].cur = (int32_t *)take(4 * n * P);
    hj[i].best = (int32_t *)take(4 * n * P);
    hj[i].cur_f = (int64_t *)take(8 * P);
    hj[i].best_f = (int64_t *)take(8 * P);
    hj[i].pool = (int32_t *)take(4 * n * Q);
    hj[i].pool_f = (int64_t *)take(8 * Q);
    hj[i].sums = (int64_t *)take(32 * n);
    hj[i].best_out = (int32_t *)take(4 * n);
  }
  HIPCHK(c, hipMemcpy(b->jobs_d, hj.data(), sizeof(DevJob) * count, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(b->items, items.data(), sizeof(uint2) * n_items, hipMemcpyHostToDevice));
  HIPCHK(c, gxk::init_jobs(b->jobs_d, count, max_q, max_n, max_mats, c->stream));
  HIPCHK(c, gxk::set_stop(b->jobs_d, count, 0, 1, c->stream));
  int occ = 0;
  HIPCHK(c, gxk::occupancy_items(max_lds, &occ));
  const uint32_t grid = (uint32_t)std::min<size_t>(n_items, (size_t)c->info.cus * std::max(1, occ));
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
  const uint32_t ni = (uint32_t)n_items, lds = max_lds;
  hipStream_t s = c->stream;
  gx_status st = enqueue_launches(c, lead, L, [=]() { return gxk::evolve_items(jd, itd, ni, grid, lds, s); });
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
