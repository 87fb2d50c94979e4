// C ABI of the FORA library: argument checks, host-side FP64 planning of the
// per-query constants, workspace layout, and the launch sequence
//   zero state -> init -> push rounds -> plan -> walks -> estimate + top-k.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

// A captured batched pipeline, valid for fixed buffers and shapes.
struct CapturedGraph {
  int batch = 0, kmax = 0, rounds = 0;
  bool index_only = false;  // the walk launch shape differs for index-only calls
  void *ws = nullptr, *ids = nullptr, *vals = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct fora_graph {
  fora::GraphDev dev;
  int2* info_owned = nullptr;
  int* flags_owned = nullptr;  // 3 ints: check flags, max degree, hub count
  int32_t* in_rowptr_owned = nullptr;
  int32_t* in_colidx_owned = nullptr;
  int32_t* inhub_node_owned = nullptr;
  fora::u64* inhub_base_owned = nullptr;
  fora::u64* rec_owned = nullptr;
  uint32_t* rec_q_owned = nullptr;
  int32_t* rank_owned = nullptr;
  // FORA+ index
  fora::u64* idx_off_owned = nullptr;
  int32_t* idx_dest_owned = nullptr;
  int64_t idx_total = 0;
  double idx_alpha = 0.0, idx_wpd = 0.0;
  uint32_t idx_key0 = 0, idx_key1 = 0;
  int device = 0;
  int cus = 256;
  // pinned host slots for the small read-backs of the push loop
  std::mutex mu;
  uint64_t* pinned = nullptr;
  std::vector<int> free_slots;
  fora_tuning tuning{8, 512, 4, 0, fora::kPullRatio, 0, 1};
  std::mutex graph_mu;
  std::list<CapturedGraph> graphs;  // most recently used first
};

namespace fora {
namespace {

constexpr int kPinnedSlots = 64;
constexpr int kMaxRounds = 20000;

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define FORA_HIP(expr)                                                                \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(FORA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct PinnedSlot {
  fora_graph* g;
  int slot;
  uint64_t* p;
  explicit PinnedSlot(fora_graph* gr) : g(gr), slot(-1), p(nullptr) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->free_slots.empty()) {
      slot = g->free_slots.back();
      g->free_slots.pop_back();
      p = g->pinned + (size_t)slot * 8;
    }
  }
  ~PinnedSlot() {
    if (slot >= 0) {
      std::lock_guard<std::mutex> lk(g->mu);
      g->free_slots.push_back(slot);
    }
  }
};

// dist: the query's source is a distribution (its src field is not used)
int check_query(const fora_graph* g, const fora_query& q, bool dist = false) {
  const int32_t n = g->dev.n;
  if (!dist && (q.src < 0 || q.src >= n)) return fail(FORA_E_ARG, "source out of range");
  if (!(q.alpha > 0.0 && q.alpha < 1.0)) return fail(FORA_E_ARG, "alpha must be in (0,1)");
  if (!(q.eps > 0.0 && q.eps < 1.0)) return fail(FORA_E_ARG, "eps must be in (0,1)");
  if (!(q.delta > 0.0 && q.delta <= 1.0)) return fail(FORA_E_ARG, "delta must be in (0,1]");
  if (!(q.pf > 0.0 && q.pf < 1.0)) return fail(FORA_E_ARG, "pf must be in (0,1)");
  if (q.k < 1 || q.k > n || q.k > FORA_MAX_K) return fail(FORA_E_ARG, "k must be in [1, min(n, FORA_MAX_K)]");
  if (!(q.rmax <= 0.0 || std::isfinite(q.rmax))) return fail(FORA_E_ARG, "rmax must be finite");
  if ((q.flags & ~(FORA_PRUNE_ZERO_HOP | FORA_BALANCE | FORA_USE_INDEX | FORA_WALK_COUNTS)) != 0 ||
      q.reserved != 0)
    return fail(FORA_E_ARG, "unknown query flags");
  if (q.flags & FORA_USE_INDEX) {
    if (!g->idx_dest_owned) return fail(FORA_E_ARG, "FORA_USE_INDEX without an index");
    if (std::floor(std::ldexp(q.alpha, 32)) != std::floor(std::ldexp(g->idx_alpha, 32)))
      return fail(FORA_E_ARG, "the index was built for another alpha");
    if (q.flags & FORA_PRUNE_ZERO_HOP)
      return fail(FORA_E_ARG, "FORA_USE_INDEX does not combine with FORA_PRUNE_ZERO_HOP");
  }
  if ((q.flags & FORA_BALANCE) && !(q.walk_cost >= 0.0 && std::isfinite(q.walk_cost)))
    return fail(FORA_E_ARG, "walk_cost must be finite and >= 0");
  return FORA_OK;
}

// Algorithm 2 and eqn:rmax (section 3.2), in FP64 on the host:
//   omega_unit = (2 eps/3 + 2) ln(2/p_f) / (eps^2 delta)
//   r_max      = eps / sqrt(m) * sqrt(delta / ((2 eps/3 + 2) ln(2/p_f))),
//                or eps^2 delta / ((2 eps/3 + 2) ln(2/p_f)) when m r_max > 1.
QueryDev plan_query(const fora_graph* g, const fora_query& q, bool dist = false) {
  QueryDev d{};
  const double c = 2.0 * q.eps / 3.0 + 2.0;
  const double L = std::log(2.0 / q.pf);
  const double cl = c * L;
  d.omega_unit = cl / ((q.eps * q.eps) * q.delta);
  double rmax = q.eps / std::sqrt((double)g->dev.m) * std::sqrt(q.delta / cl);
  if ((double)g->dev.m * rmax > 1.0) rmax = (q.eps * q.eps) * q.delta / cl;
  if (q.rmax > 0.0) rmax = q.rmax;
  d.rmax = rmax;
  d.alpha = q.alpha;
  d.src = q.src;
  d.k = q.k;
  d.key0 = dist ? kDistKey0 : (uint32_t)q.src;
  d.key1 = (uint32_t)(q.seed & 0xFFFFFFFFull);
  if (dist) d.src = 0;
  d.t_alpha = (uint32_t)std::floor(std::ldexp(q.alpha, 32));
  d.flags = q.flags;
  d.walk_cost = (q.flags & FORA_BALANCE) ? q.walk_cost : 0.0;
  if (q.flags & FORA_USE_INDEX) {  // the index's walks: keyed by the index key
    d.key0 = g->idx_key0;
    d.key1 = g->idx_key1;
  }
  return d;
}

int error_code_from_flags(int flags) {
  if (flags & kErrBadDist)
    return fail(FORA_E_ARG, "source distribution entries must lie in [0, 1]");
  if (flags & kErrBadPlan)
    return fail(FORA_E_ARG, "walk plan nodes must be strictly increasing ids in [0, n)");
  if (flags & kErrOmegaOverflow)
    return fail(FORA_E_OVERFLOW, "walk count overflow (some omega_v >= 2^32)");
  if (flags & kErrFrontierOverflow) return fail(FORA_E_OVERFLOW, "frontier overflow");
  if (flags & kErrLogOverflow) return fail(FORA_E_OVERFLOW, "frontier log capacity too small");
  if (flags & kErrTopk) return fail(FORA_E_HIP, "top-k selection inconsistent");
  return FORA_OK;
}

int walk_blocks(const fora_graph* g) { return g->cus * g->tuning.walk_blocks_per_cu; }
int push_blocks(const fora_graph* g) { return g->cus * g->tuning.push_blocks_per_cu; }
int walk_chunk(const fora_graph* g) { return g->tuning.walk_chunk; }
constexpr size_t kMaxCapturedGraphs = 8;

void drop_graphs(fora_graph* g) {
  std::lock_guard<std::mutex> lk(g->graph_mu);
  for (auto& c : g->graphs) {
    if (c.exec) (void)hipGraphExecDestroy(c.exec);
    if (c.graph) (void)hipGraphDestroy(c.graph);
  }
  g->graphs.clear();
}

struct Call {
  Layout L;
  Ws w;
  int walk_chunk = 0;  // walk ids per work-queue grab for this call
  bool index_only = false;
};

// Index walks end at once, so small chunks make the work-queue counter the
// bottleneck, and their end points (many at the start node) are all that is
// left to cost: a call whose queries all read the index grabs larger chunks
// and always sums end points in LDS first.
constexpr int kIndexWalkChunk = 32768;

int call_chunk(const fora_graph* g, const Call& c) {
  return c.walk_chunk ? c.walk_chunk : g->tuning.walk_chunk;
}

bool call_agg(const fora_graph* g, const Call& c) {
  return c.index_only || g->tuning.walk_agg != 0;
}

int prepare(const fora_graph* g, int batch, void* d_ws, size_t ws_bytes, Call& c) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  if (batch < 1 || batch > FORA_MAX_BATCH) return fail(FORA_E_ARG, "batch out of range");
  if (!d_ws) return fail(FORA_E_ARG, "null workspace");
  if (((uintptr_t)d_ws & 255) != 0) return fail(FORA_E_ARG, "workspace must be 256-byte aligned");
  c.L = make_layout(g->dev, batch);
  if (ws_bytes < c.L.total) return fail(FORA_E_NOMEM, "workspace too small");
  c.w = carve(c.L, d_ws);
  return FORA_OK;
}

// Push rounds until the frontier is empty; the host checks the frontier size
// after every group of rounds.
int run_push(fora_graph* g, const Call& c, int batch, hipStream_t s, bool stats,
             int32_t* log, int64_t log_cap, int* rounds_out, int first_round = 0) {
  PinnedSlot ps(g);
  if (!ps.p) return fail(FORA_E_NOMEM, "too many concurrent calls on one graph");
  int t = first_round, group = 4;
  for (;;) {
    for (int i = 0; i < group; ++i, ++t)
      FORA_HIP(launch_push_round(g->dev, c.w, c.L, batch, t, push_blocks(g),
                                 g->tuning.pull_ratio, log, log_cap, s));
    FORA_HIP(hipMemcpyAsync(ps.p, &c.w.ctrl->fr_cnt[t & 1], sizeof(uint64_t),
                            hipMemcpyDeviceToHost, s));
    FORA_HIP(hipStreamSynchronize(s));
    if (*ps.p == 0) break;
    if (t >= kMaxRounds) return fail(FORA_E_OVERFLOW, "push did not converge");
    group = std::min(group * 2, 16);
  }
  if (rounds_out) *rounds_out = t;
  return FORA_OK;
}

// Events bracketing the phases of one call (created only when stats are asked).
struct PhaseEvents {
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  explicit PhaseEvents(bool enable) : on(enable) {
    if (!on) return;
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        on = false;
        break;
      }
  }
  ~PhaseEvents() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int i, hipStream_t s) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  float ms(int i) const {
    float t = 0.f;
    if (on) (void)hipEventElapsedTime(&t, ev[i], ev[i + 1]);
    return t;
  }
};

int finish(fora_graph* g, const Call& c, int batch, hipStream_t s, fora_stats* h_stats,
           const std::vector<QueryDev>& qd, const PhaseEvents* pe = nullptr) {
  int flags = 0;
  FORA_HIP(hipMemcpyAsync(&flags, &c.w.ctrl->error, sizeof(int), hipMemcpyDeviceToHost, s));
  std::vector<StatSlot> slots;
  if (h_stats) {
    slots.resize((size_t)batch * kStatSlots);
    FORA_HIP(hipMemcpyAsync(slots.data(), c.w.qstats, sizeof(StatSlot) * slots.size(),
                            hipMemcpyDeviceToHost, s));
  }
  FORA_HIP(hipStreamSynchronize(s));
  const int rc = error_code_from_flags(flags);
  if (rc != FORA_OK) return rc;
  if (h_stats) {
    for (int b = 0; b < batch; ++b) {
      fora_stats& o = h_stats[b];
      std::memset(&o, 0, sizeof(o));
      u64 r_sum_fx = 0;
      for (int k = 0; k < kStatSlots; ++k) {
        const StatSlot& q = slots[(size_t)b * kStatSlots + k];
        o.rounds = std::max(o.rounds, q.rounds);
        o.term_violations += q.term_violations;
        o.pushes += (int64_t)q.pushes;
        o.edge_ops += (int64_t)q.edge_ops;
        o.plan_entries += (int64_t)q.entries;
        o.walks += q.walks;
        o.steps += q.steps;
        r_sum_fx += q.r_sum_fx;
        o.pull_rounds += (uint32_t)q.pull_rounds;
        o.balance_stopped |= (uint32_t)(q.balance_stopped != 0);
      }
      o.r_sum = std::ldexp((double)r_sum_fx, -62);
      o.rmax = qd[b].rmax;
      o.omega_unit = qd[b].omega_unit;
      o.t_alpha = qd[b].t_alpha;
      if (pe && pe->on) {
        o.ms_push = pe->ms(0);
        o.ms_plan = pe->ms(1);
        o.ms_walk = pe->ms(2);
        o.ms_topk = pe->ms(3);
      }
    }
  }
  (void)g;
  return FORA_OK;
}

// Everything after the query upload, as one sequence of launches on `s`.
hipError_t enqueue_pipeline(fora_graph* g, const Call& c, int batch, int rounds, int kmax,
                            void* d_ws, int32_t* d_ids, float* d_vals, hipStream_t s) {
  hipError_t e = launch_fill_zero((char*)d_ws + c.L.zero_begin, c.L.zero_end - c.L.zero_begin, s);
  if (e == hipSuccess) e = launch_init_queries(g->dev, c.w, batch, s);
  for (int t = 0; t < rounds && e == hipSuccess; ++t)
    e = launch_push_round(g->dev, c.w, c.L, batch, t, push_blocks(g), g->tuning.pull_ratio,
                          nullptr, 0, s);
  if (e == hipSuccess) e = launch_push_gate(c.w, rounds, s);
  if (e == hipSuccess) e = launch_plan(g->dev, c.w, c.L, batch, s);
  if (e == hipSuccess) e = launch_walks(g->dev, c.w, walk_blocks(g), call_chunk(g, c),
                                 call_agg(g, c), s);
  if (e == hipSuccess) e = launch_topk(g->dev, c.w, c.L, batch, kmax, d_ids, d_vals, s);
  return e;
}

// Find or capture the graph for these buffers and shapes.
int graph_for(fora_graph* g, const Call& c, int batch, int kmax, void* d_ws, int32_t* d_ids,
              float* d_vals, hipStream_t s, hipGraphExec_t* out) {
  const int rounds = g->tuning.graph_rounds;
  std::lock_guard<std::mutex> lk(g->graph_mu);
  for (auto it = g->graphs.begin(); it != g->graphs.end(); ++it) {
    if (it->batch == batch && it->kmax == kmax && it->rounds == rounds && it->ws == d_ws &&
        it->ids == (void*)d_ids && it->vals == (void*)d_vals &&
        it->index_only == c.index_only) {
      g->graphs.splice(g->graphs.begin(), g->graphs, it);
      *out = g->graphs.front().exec;
      return FORA_OK;
    }
  }
  CapturedGraph cg;
  cg.batch = batch;
  cg.kmax = kmax;
  cg.rounds = rounds;
  cg.index_only = c.index_only;
  cg.ws = d_ws;
  cg.ids = d_ids;
  cg.vals = d_vals;
  hipStream_t cs = nullptr;
  FORA_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t e1 = enqueue_pipeline(g, c, batch, rounds, kmax, d_ws, d_ids, d_vals, cs);
    e = hipStreamEndCapture(cs, &cg.graph);
    if (e1 != hipSuccess) e = e1;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  (void)s;
  if (e != hipSuccess) {
    if (cg.graph) (void)hipGraphDestroy(cg.graph);
    return fail(FORA_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
  }
  g->graphs.push_front(cg);
  while (g->graphs.size() > kMaxCapturedGraphs) {
    CapturedGraph& old = g->graphs.back();
    (void)hipGraphExecDestroy(old.exec);
    (void)hipGraphDestroy(old.graph);
    g->graphs.pop_back();
  }
  *out = cg.exec;
  return FORA_OK;
}

int run_queries_graph(fora_graph* g, const Call& c, int batch, const std::vector<QueryDev>& qd,
                      int kmax, void* d_ws, int32_t* d_ids, float* d_vals, fora_stats* h_stats,
                      hipStream_t s) {
  hipGraphExec_t exec = nullptr;
  int rc = graph_for(g, c, batch, kmax, d_ws, d_ids, d_vals, s, &exec);
  if (rc != FORA_OK) return rc;
  FORA_HIP(hipMemcpyAsync(c.w.queries, qd.data(), sizeof(QueryDev) * batch,
                          hipMemcpyHostToDevice, s));
  FORA_HIP(hipGraphLaunch(exec, s));
  int skip = 0;
  FORA_HIP(hipMemcpyAsync(&skip, &c.w.ctrl->skip, sizeof(int), hipMemcpyDeviceToHost, s));
  FORA_HIP(hipStreamSynchronize(s));
  if (skip) {
    // some frontier outlived the captured rounds: finish on the host
    const int zero = 0;
    FORA_HIP(hipMemcpyAsync(&c.w.ctrl->skip, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    rc = run_push(g, c, batch, s, true, nullptr, 0, nullptr, g->tuning.graph_rounds);
    if (rc != FORA_OK) return rc;
    FORA_HIP(launch_plan(g->dev, c.w, c.L, batch, s));
    FORA_HIP(launch_walks(g->dev, c.w, walk_blocks(g), call_chunk(g, c),
                                 call_agg(g, c), s));
    FORA_HIP(launch_topk(g->dev, c.w, c.L, batch, kmax, d_ids, d_vals, s));
  }
  return finish(g, c, batch, s, h_stats, qd, nullptr);
}

// d_sigma (nullable): double[batch][n], each query's source distribution
// eager_only: never capture or replay a HIP graph, and time no phases (the
// allocation-free entry point: both would allocate)
int run_queries(fora_graph* g, int batch, const fora_query* qs, int kmax, void* d_ws,
                size_t ws_bytes, int32_t* d_ids, float* d_vals, fora_stats* h_stats,
                hipStream_t s, const double* d_sigma = nullptr, bool eager_only = false) {
  if (!qs) return fail(FORA_E_ARG, "null queries");
  if (!d_ids || !d_vals) return fail(FORA_E_ARG, "null output");
  Call c;
  int rc = prepare(g, batch, d_ws, ws_bytes, c);
  if (rc != FORA_OK) return rc;
  std::vector<QueryDev> qd(batch);
  bool all_index = true;
  for (int b = 0; b < batch; ++b) {
    rc = check_query(g, qs[b], d_sigma != nullptr);
    if (rc != FORA_OK) return rc;
    if (qs[b].k > kmax) return fail(FORA_E_ARG, "kmax smaller than a query's k");
    qd[b] = plan_query(g, qs[b], d_sigma != nullptr);
    all_index = all_index && (qs[b].flags & FORA_USE_INDEX);
  }
  c.walk_chunk = all_index ? std::max(walk_chunk(g), kIndexWalkChunk) : walk_chunk(g);
  c.index_only = all_index;
  FORA_HIP(hipSetDevice(g->device));
  if (g->tuning.graph_rounds > 0 && !d_sigma && !eager_only)
    return run_queries_graph(g, c, batch, qd, kmax, d_ws, d_ids, d_vals, h_stats, s);
  FORA_HIP(launch_fill_zero((char*)d_ws + c.L.zero_begin, c.L.zero_end - c.L.zero_begin, s));
  FORA_HIP(hipMemcpyAsync(c.w.queries, qd.data(), sizeof(QueryDev) * batch,
                          hipMemcpyHostToDevice, s));
  PhaseEvents pe(h_stats != nullptr && !eager_only);
  pe.mark(0, s);
  if (d_sigma)
    FORA_HIP(launch_init_dist(g->dev, c.w, c.L, batch, d_sigma, s));
  else
    FORA_HIP(launch_init_queries(g->dev, c.w, batch, s));
  rc = run_push(g, c, batch, s, true, nullptr, 0, nullptr);
  if (rc != FORA_OK) return rc;
  pe.mark(1, s);
  FORA_HIP(launch_plan(g->dev, c.w, c.L, batch, s));
  pe.mark(2, s);
  FORA_HIP(launch_walks(g->dev, c.w, walk_blocks(g), call_chunk(g, c),
                                 call_agg(g, c), s));
  pe.mark(3, s);
  FORA_HIP(launch_topk(g->dev, c.w, c.L, batch, kmax, d_ids, d_vals, s));
  pe.mark(4, s);
  return finish(g, c, batch, s, h_stats, qd, &pe);
}

}  // namespace

Layout make_layout(const GraphDev& g, int32_t batch) {
  const int32_t n = g.n;
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  };
  const size_t cap = (size_t)batch * (size_t)n;
  L.cap = (int64_t)cap;
  L.hub_cap = (int64_t)batch * (int64_t)std::max(g.n_hubs, 1);
  L.tiles_per_row = (n + kPlanTile - 1) / kPlanTile;
  L.plan_tiles = L.tiles_per_row * batch;
  L.topk_blocks = (n + kTopkTile - 1) / kTopkTile;
  // written before being read
  L.queries = take(sizeof(QueryDev) * batch);
  L.mode = take(4 * (size_t)batch);
  L.pull_list = take(4 * (size_t)batch);
  L.tile_cnt = take(4 * (size_t)L.plan_tiles);
  L.tile_walks = take(8 * (size_t)L.plan_tiles);
  L.tile_eoff = take(8 * (size_t)L.plan_tiles);
  L.tile_woff = take(8 * (size_t)L.plan_tiles);
  L.sel = take(16 * (size_t)batch);
  L.cand_key = take(4 * (size_t)FORA_MAX_K * batch);
  L.cand_id = take(4 * (size_t)FORA_MAX_K * batch);
  L.blk_ties = take(4 * (size_t)L.topk_blocks * batch);
  // cleared at the start of every call, up to and including incd
  L.ctrl = take(sizeof(Ctrl));
  L.zero_begin = L.ctrl;
  L.qstats = take(sizeof(StatSlot) * (size_t)kStatSlots * batch);
  L.r = take(8 * cap);
  L.q = take(4 * cap);
  L.hist = take(4 * (size_t)kHistBins * batch);
  L.cand_cnt = take(4 * (size_t)batch);
  L.ecnt = take(8 * 2 * (size_t)kStatSlots * batch);
  L.stop = take(4 * (size_t)batch);
  // Phase region: the push's arrays and the walk phase's arrays are never
  // live at once, so they share it (8 B x 4 against 8 B x 5 per node and
  // query). The walk view's sums are cleared by the plan, after the push.
  const size_t phase = align_up(off, 256);
  const size_t pg = (size_t)pull_group_for(batch);
  L.incd = take(8 * (((size_t)batch + pg - 1) / pg * pg) * (size_t)n);  // whole pull groups
  L.zero_end = align_up(off, 256);
  L.fr0 = take(8 * cap);
  L.fr1 = take(8 * cap);
  L.frx = take(8 * cap);
  L.hub_idx = take(8 * (size_t)L.hub_cap);
  L.hub_base = take(8 * (size_t)L.hub_cap);
  const size_t push_end = off;
  off = phase;
  L.acc = take(8 * cap);
  L.cnt = take(8 * cap);
  L.plan_gi = take(8 * cap);
  L.plan_off = take(8 * (cap + 1));
  L.plan_wfx = take(8 * cap);
  // the estimate is formed after the walks, when the plan is no longer read
  L.pi = L.plan_gi;
  off = std::max(off, push_end);
  L.total = align_up(off, 256);
  return L;
}

Ws carve(const Layout& L, void* base) {
  char* p = (char*)base;
  Ws w{};
  w.ctrl = (Ctrl*)(p + L.ctrl);
  w.qstats = (QueryStatsDev*)(p + L.qstats);
  w.queries = (QueryDev*)(p + L.queries);
  w.r = (u64*)(p + L.r);
  w.q = (float*)(p + L.q);
  w.cnt = (u64*)(p + L.cnt);
  w.acc = (u64*)(p + L.acc);
  w.pi = (float*)(p + L.pi);
  w.fr[0] = (u64*)(p + L.fr0);
  w.fr[1] = (u64*)(p + L.fr1);
  w.frx = (u64*)(p + L.frx);
  w.hub_idx = (u64*)(p + L.hub_idx);
  w.hub_base = (u64*)(p + L.hub_base);
  w.incd = (u64*)(p + L.incd);
  w.ecnt = (u64*)(p + L.ecnt);
  w.mode = (int32_t*)(p + L.mode);
  w.pull_list = (int32_t*)(p + L.pull_list);
  w.stop = (int32_t*)(p + L.stop);
  w.plan_gi = (u64*)(p + L.plan_gi);
  w.plan_off = (u64*)(p + L.plan_off);
  w.plan_wfx = (u64*)(p + L.plan_wfx);
  w.tile_cnt = (uint32_t*)(p + L.tile_cnt);
  w.tile_walks = (u64*)(p + L.tile_walks);
  w.tile_eoff = (u64*)(p + L.tile_eoff);
  w.tile_woff = (u64*)(p + L.tile_woff);
  w.hist = (uint32_t*)(p + L.hist);
  w.sel = (uint32_t*)(p + L.sel);
  w.cand_key = (uint32_t*)(p + L.cand_key);
  w.cand_id = (int32_t*)(p + L.cand_id);
  w.cand_cnt = (uint32_t*)(p + L.cand_cnt);
  w.blk_ties = (uint32_t*)(p + L.blk_ties);
  return w;
}

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 256;
  return cus > 0 ? cus : 256;
}

}  // namespace fora

using namespace fora;

namespace {

// Reverse (in-edge) CSR and the list of nodes whose in-degree needs pieces,
// for pull-mode push rounds. Allocated once per graph handle.
int build_reverse(fora_graph* g, hipStream_t s) {
  const int32_t n = g->dev.n;
  const int64_t m = g->dev.m;
  int32_t* cursor = nullptr;
  uint32_t* tsum = nullptr;
  int32_t* list = nullptr;
  const int64_t tiles = (n + 2047) / 2048;
  const int32_t list_cap = (int32_t)std::min<int64_t>(n, m / (kHubDeg + 1) + 1);
  auto release = [&]() {
    if (cursor) (void)hipFree(cursor);
    if (tsum) (void)hipFree(tsum);
    if (list) (void)hipFree(list);
  };
  if (hipMalloc(&g->in_rowptr_owned, sizeof(int32_t) * ((size_t)n + 1)) != hipSuccess ||
      hipMalloc(&g->in_colidx_owned, sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1)) !=
          hipSuccess ||
      hipMalloc(&cursor, sizeof(int32_t) * (size_t)n) != hipSuccess ||
      hipMalloc(&tsum, sizeof(uint32_t) * (size_t)tiles) != hipSuccess ||
      hipMalloc(&list, sizeof(int32_t) * ((size_t)list_cap + 1)) != hipSuccess) {
    release();
    return fail(FORA_E_NOMEM, "hipMalloc of the reverse graph failed");
  }
  std::vector<int32_t> in_rowptr((size_t)n + 1);
  int32_t count = 0;
  hipError_t e = launch_build_reverse(g->dev, g->in_rowptr_owned, g->in_colidx_owned, cursor,
                                      tsum, s);
  if (e == hipSuccess) e = launch_fill_zero(list + list_cap, sizeof(int32_t), s);
  if (e == hipSuccess)
    e = launch_list_inhubs(g->in_rowptr_owned, n, list, list + list_cap, list_cap, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&count, list + list_cap, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(in_rowptr.data(), g->in_rowptr_owned, sizeof(int32_t) * in_rowptr.size(),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<int32_t> hubs;
  if (e == hipSuccess && count > 0) {
    hubs.resize((size_t)std::min(count, list_cap));
    e = hipMemcpy(hubs.data(), list, sizeof(int32_t) * hubs.size(), hipMemcpyDeviceToHost);
  }
  release();
  if (e != hipSuccess) return fail(FORA_E_HIP, std::string("reverse graph: ") + hipGetErrorString(e));
  std::sort(hubs.begin(), hubs.end());
  std::vector<u64> base(hubs.size());
  u64 pieces = 0;
  for (size_t i = 0; i < hubs.size(); ++i) {
    base[i] = pieces;
    const int32_t d = in_rowptr[hubs[i] + 1] - in_rowptr[hubs[i]];
    pieces += (u64)((d + kHubPiece - 1) / kHubPiece);
  }
  if (!hubs.empty()) {
    if (hipMalloc(&g->inhub_node_owned, sizeof(int32_t) * hubs.size()) != hipSuccess ||
        hipMalloc(&g->inhub_base_owned, sizeof(u64) * hubs.size()) != hipSuccess)
      return fail(FORA_E_NOMEM, "hipMalloc of the in-hub table failed");
    if (hipMemcpy(g->inhub_node_owned, hubs.data(), sizeof(int32_t) * hubs.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->inhub_base_owned, base.data(), sizeof(u64) * base.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      return fail(FORA_E_HIP, "upload of the in-hub table failed");
  }
  g->dev.in_rowptr = g->in_rowptr_owned;
  g->dev.in_colidx = g->in_colidx_owned;
  g->dev.n_inhubs = (int32_t)hubs.size();
  g->dev.inhub_node = g->inhub_node_owned;
  g->dev.inhub_base = g->inhub_base_owned;
  g->dev.inhub_pieces = pieces;
  return FORA_OK;
}

// Degree rank of every node (GraphDev::rank).
int build_rank(fora_graph* g, hipStream_t s) {
  const int32_t n = g->dev.n;
  size_t bytes = 0;
  if (degree_rank_scratch_bytes(n, &bytes) != hipSuccess)
    return fail(FORA_E_HIP, "degree rank: sort sizing failed");
  void* scratch = nullptr;
  if (hipMalloc(&g->rank_owned, sizeof(int32_t) * (size_t)n) != hipSuccess ||
      hipMalloc(&scratch, bytes) != hipSuccess) {
    if (scratch) (void)hipFree(scratch);
    return fail(FORA_E_NOMEM, "hipMalloc of the degree rank failed");
  }
  g->dev.rank = g->rank_owned;
  hipError_t e = launch_degree_rank(g->dev, g->rank_owned, scratch, bytes, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(scratch);
  if (e != hipSuccess) return fail(FORA_E_HIP, std::string("degree rank: ") + hipGetErrorString(e));
  return FORA_OK;
}

// Walk records (one 8-byte header plus one 8-byte unit per out-edge per
// node); n + m < 2^32 always holds for 32-bit CSR offsets and node ids, so
// record starts fit 32 bits. A slot also carries the neighbour's id when
// record start, degree and id fit 64 bits together (for example n = 2^20,
// m = 1.7e7: 25 + 19 + 20 bits).
// mode: the tuning's record_ids (0: (start, degree) slots; 1: ids where
// they fit; 2: ids with a 4-bit degree field, which sends every degree of
// 15 or more to the header)
int build_records(fora_graph* g, int mode, hipStream_t s) {
  const int64_t n = g->dev.n;
  const int64_t units = g->dev.m + n;
  int qb = 1, ib = 1;
  while ((1ll << qb) < units) ++qb;  // record starts are below n + m
  while ((1ll << ib) < n) ++ib;      // ids are below n
  const int db = 64 - qb - ib;
  // The slot format, applied to the graph only once the scratch is there.
  // A degree the field cannot hold is stored as all ones and read from the
  // node's header by the walk; with a field of at least kMinDegBits bits that
  // happens only for hubs, whose headers stay in L2.
  constexpr int kMinDegBits = 12;
  int fq = 32, fd = 32, fid = 0;
  const bool all_fit = db >= 1 && db <= 32 && (int64_t)g->dev.max_deg < (1ll << db) - 1;
  if (mode == 1 && db > 32) {  // small graphs: a 32-bit degree field always fits
    fq = qb;
    fid = 1;
  } else if (mode == 1 && (all_fit || (db >= kMinDegBits && db <= 32))) {
    fq = qb;
    fd = db;
    fid = 1;
  } else if (mode == 2 && db >= 4) {
    fq = qb;
    fd = 4;
    fid = 1;
  }
  const int64_t tiles = (n + 2047) / 2048;
  int32_t* tmp = nullptr;
  uint32_t* tsum = nullptr;
  auto release = [&]() {
    if (tmp) (void)hipFree(tmp);
    if (tsum) (void)hipFree(tsum);
  };
  if ((!g->rec_owned && hipMalloc(&g->rec_owned, sizeof(u64) * (size_t)units) != hipSuccess) ||
      (!g->rec_q_owned &&
       hipMalloc(&g->rec_q_owned, sizeof(uint32_t) * ((size_t)n + 1)) != hipSuccess) ||
      hipMalloc(&tmp, sizeof(int32_t) * (2 * (size_t)n + 1)) != hipSuccess ||
      hipMalloc(&tsum, sizeof(uint32_t) * (size_t)tiles) != hipSuccess) {
    release();
    return fail(FORA_E_NOMEM, "hipMalloc of the walk records failed");
  }
  g->dev.rec = g->rec_owned;
  g->dev.rec_q = g->rec_q_owned;
  g->dev.slot_qbits = fq;
  g->dev.slot_dbits = fd;
  g->dev.slot_ids = fid;
  hipError_t e = launch_build_records(g->dev, g->rec_q_owned, g->rec_owned, tmp, tsum, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess) return fail(FORA_E_HIP, std::string("walk records: ") + hipGetErrorString(e));
  return FORA_OK;
}

// ---- workspace for callers that cannot allocate -----------------------------
// A file-scope device array that fora_ssppr_static uses as its workspace. Each
// device holds its own copy from the time the library's code is loaded on it
// until the process ends. Host code never passes the array's name to a kernel
// (on the host it is a stand-in, not a device address): the device address is
// looked up once per device with hipGetSymbolAddress and kept here.
constexpr size_t kStaticScratchBytes = (size_t)FORA_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up on
// the first call made with that device current).
int static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(FORA_E_ARG, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FORA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return FORA_OK;
}

}  // namespace

extern "C" {

const char* fora_last_error(void) { return g_err.c_str(); }

int fora_build_csr(int32_t n, int64_t m, const int32_t* d_rowptr, const int32_t* d_colidx,
                   void* stream, fora_graph** out) {
  if (!out) return fail(FORA_E_ARG, "null output handle");
  *out = nullptr;
  if (n < 1) return fail(FORA_E_ARG, "n must be >= 1");
  if (m < 0 || m >= (int64_t)1 << 31) return fail(FORA_E_ARG, "m must be in [0, 2^31)");
  if (!d_rowptr || (m > 0 && !d_colidx)) return fail(FORA_E_ARG, "null CSR array");
  hipStream_t s = (hipStream_t)stream;
  fora_graph* g = new fora_graph();
  g->dev.n = n;
  g->dev.m = m;
  g->dev.rowptr = d_rowptr;
  g->dev.colidx = d_colidx;
  auto cleanup = [&](int code, const std::string& msg) {
    if (g->in_rowptr_owned) (void)hipFree(g->in_rowptr_owned);
    if (g->in_colidx_owned) (void)hipFree(g->in_colidx_owned);
    if (g->inhub_node_owned) (void)hipFree(g->inhub_node_owned);
    if (g->inhub_base_owned) (void)hipFree(g->inhub_base_owned);
    if (g->rec_owned) (void)hipFree(g->rec_owned);
    if (g->rec_q_owned) (void)hipFree(g->rec_q_owned);
    if (g->rank_owned) (void)hipFree(g->rank_owned);
    if (g->idx_off_owned) (void)hipFree(g->idx_off_owned);
    if (g->idx_dest_owned) (void)hipFree(g->idx_dest_owned);
    if (g->info_owned) (void)hipFree(g->info_owned);
    if (g->flags_owned) (void)hipFree(g->flags_owned);
    if (g->pinned) (void)hipHostFree(g->pinned);
    delete g;
    return fail(code, msg);
  };
  if (hipGetDevice(&g->device) != hipSuccess) return cleanup(FORA_E_HIP, "hipGetDevice failed");
  g->cus = device_cu_count();
  if (hipMalloc(&g->info_owned, sizeof(int2) * (size_t)n) != hipSuccess)
    return cleanup(FORA_E_NOMEM, "hipMalloc of the node table failed");
  if (hipMalloc(&g->flags_owned, 3 * sizeof(int)) != hipSuccess)
    return cleanup(FORA_E_NOMEM, "hipMalloc failed");
  if (hipHostMalloc((void**)&g->pinned, sizeof(uint64_t) * 8 * kPinnedSlots, 0) != hipSuccess)
    return cleanup(FORA_E_NOMEM, "hipHostMalloc failed");
  for (int i = kPinnedSlots - 1; i >= 0; --i) g->free_slots.push_back(i);
  g->dev.info = g->info_owned;
  int host_flags[3] = {0, 0, 0};
  if (hipMemcpyAsync(g->flags_owned, host_flags, sizeof(host_flags), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      launch_graph_check(g->dev, g->flags_owned, g->flags_owned + 1, g->flags_owned + 2,
                         g->info_owned, s) !=
          hipSuccess ||
      hipMemcpyAsync(host_flags, g->flags_owned, sizeof(host_flags), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return cleanup(FORA_E_HIP, std::string("graph check failed: ") +
                                   hipGetErrorString(hipGetLastError()));
  if (host_flags[0] & kErrGraphRowptr) return cleanup(FORA_E_GRAPH, "malformed rowptr");
  if (host_flags[0] & kErrGraphTarget) return cleanup(FORA_E_GRAPH, "target id out of range");
  if (host_flags[0] & kErrGraphDangling)
    return cleanup(FORA_E_GRAPH, "a node has out-degree 0 (dangling)");
  g->dev.max_deg = host_flags[1];
  g->dev.n_hubs = host_flags[2];
  int rrc = build_rank(g, s);
  if (rrc == FORA_OK) rrc = build_reverse(g, s);
  if (rrc == FORA_OK) rrc = build_records(g, g->tuning.record_ids, s);
  if (rrc != FORA_OK) {
    const std::string msg = g_err;
    return cleanup(rrc, msg);
  }
  *out = g;
  return FORA_OK;
}

int fora_get_tuning(const fora_graph* g, fora_tuning* out) {
  if (!g || !out) return fail(FORA_E_ARG, "null argument");
  *out = g->tuning;
  return FORA_OK;
}

int fora_set_tuning(fora_graph* g, const fora_tuning* t) {
  if (!g || !t) return fail(FORA_E_ARG, "null argument");
  if (t->walk_blocks_per_cu < 1 || t->walk_blocks_per_cu > 32)
    return fail(FORA_E_ARG, "walk_blocks_per_cu must be in [1, 32]");
  if (t->push_blocks_per_cu < 1 || t->push_blocks_per_cu > 32)
    return fail(FORA_E_ARG, "push_blocks_per_cu must be in [1, 32]");
  if (t->walk_chunk < 64 || t->walk_chunk > 65536 || (t->walk_chunk & 63) != 0)
    return fail(FORA_E_ARG, "walk_chunk must be a multiple of 64 in [64, 65536]");
  if (t->graph_rounds < 0 || t->graph_rounds > kMaxRoundsLogged)
    return fail(FORA_E_ARG, "graph_rounds must be in [0, 4096]");
  if (t->pull_ratio < 0) return fail(FORA_E_ARG, "pull_ratio must be >= 0");
  if (t->walk_agg != 0 && t->walk_agg != 1) return fail(FORA_E_ARG, "walk_agg must be 0 or 1");
  if (t->record_ids < 0 || t->record_ids > 2)
    return fail(FORA_E_ARG, "record_ids must be 0, 1 or 2");
  drop_graphs(g);
  if (t->record_ids != g->tuning.record_ids) {
    FORA_HIP(hipSetDevice(g->device));
    FORA_HIP(hipDeviceSynchronize());  // no call may still read the records
    const int rc = build_records(g, t->record_ids, nullptr);
    if (rc != FORA_OK) return rc;
  }
  g->tuning = *t;
  return FORA_OK;
}

int fora_free_graph(fora_graph* g) {
  if (!g) return FORA_OK;
  drop_graphs(g);
  if (g->in_rowptr_owned) (void)hipFree(g->in_rowptr_owned);
  if (g->in_colidx_owned) (void)hipFree(g->in_colidx_owned);
  if (g->inhub_node_owned) (void)hipFree(g->inhub_node_owned);
  if (g->inhub_base_owned) (void)hipFree(g->inhub_base_owned);
  if (g->rec_owned) (void)hipFree(g->rec_owned);
  if (g->rec_q_owned) (void)hipFree(g->rec_q_owned);
  if (g->rank_owned) (void)hipFree(g->rank_owned);
  if (g->idx_off_owned) (void)hipFree(g->idx_off_owned);
  if (g->idx_dest_owned) (void)hipFree(g->idx_dest_owned);
  if (g->info_owned) (void)hipFree(g->info_owned);
  if (g->flags_owned) (void)hipFree(g->flags_owned);
  if (g->pinned) (void)hipHostFree(g->pinned);
  delete g;
  return FORA_OK;
}

int fora_graph_info(const fora_graph* g, int32_t* n, int64_t* m, int32_t* max_degree) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  if (n) *n = g->dev.n;
  if (m) *m = g->dev.m;
  if (max_degree) *max_degree = g->dev.max_deg;
  return FORA_OK;
}

int fora_workspace_size(const fora_graph* g, int32_t batch, size_t* bytes) {
  if (!g || !bytes) return fail(FORA_E_ARG, "null argument");
  if (batch < 1 || batch > FORA_MAX_BATCH) return fail(FORA_E_ARG, "batch out of range");
  *bytes = make_layout(g->dev, batch).total;
  return FORA_OK;
}

int fora_workspace_views(const fora_graph* g, int32_t batch, void* d_ws, fora_views* v) {
  if (!g || !d_ws || !v) return fail(FORA_E_ARG, "null argument");
  if (batch < 1 || batch > FORA_MAX_BATCH) return fail(FORA_E_ARG, "batch out of range");
  const Layout L = make_layout(g->dev, batch);
  const Ws w = carve(L, d_ws);
  v->residue_fx = (uint64_t*)w.r;
  v->reserve = w.q;
  v->walk_count = (uint64_t*)w.cnt;
  v->walk_weight_fx = (uint64_t*)w.acc;
  v->pi_hat = w.pi;
  return FORA_OK;
}

int fora_ssppr(const fora_graph* g, int32_t src, double alpha, double eps, double delta,
               double pf, int32_t k, double opt_rmax, uint64_t seed, void* d_ws,
               size_t ws_bytes, int32_t* d_topk_ids, float* d_topk_vals, fora_stats* h_stats,
               void* stream) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  fora_query q{};
  q.src = src;
  q.k = k;
  q.alpha = alpha;
  q.eps = eps;
  q.delta = delta;
  q.pf = pf;
  q.rmax = opt_rmax;
  q.seed = seed;
  return run_queries(const_cast<fora_graph*>(g), 1, &q, k, d_ws, ws_bytes, d_topk_ids,
                     d_topk_vals, h_stats, (hipStream_t)stream);
}

int fora_ssppr_static(const fora_graph* g, int32_t src, double alpha, double eps, double delta,
                      double pf, int32_t k, double opt_rmax, uint64_t seed, int32_t* d_topk_ids,
                      float* d_topk_vals, fora_stats* h_stats, void* stream) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  const size_t need = make_layout(g->dev, 1).total;
  if (need > kStaticScratchBytes)
    return fail(FORA_E_NOMEM, "the graph needs " + std::to_string(need) +
                                  " bytes of workspace, above the static scratch of " +
                                  std::to_string(kStaticScratchBytes) + " bytes");
  FORA_HIP(hipSetDevice(g->device));
  void* ws = nullptr;
  const int rc = static_scratch(g->device, &ws);
  if (rc != FORA_OK) return rc;
  fora_query q{};
  q.src = src;
  q.k = k;
  q.alpha = alpha;
  q.eps = eps;
  q.delta = delta;
  q.pf = pf;
  q.rmax = opt_rmax;
  q.seed = seed;
  return run_queries(const_cast<fora_graph*>(g), 1, &q, k, ws, kStaticScratchBytes, d_topk_ids,
                     d_topk_vals, h_stats, (hipStream_t)stream, nullptr, true);
}

int fora_ssppr_batch(const fora_graph* g, int32_t batch, const fora_query* h_queries,
                     int32_t kmax, void* d_ws, size_t ws_bytes, int32_t* d_ids, float* d_vals,
                     fora_stats* h_stats, void* stream) {
  if (kmax < 1 || kmax > FORA_MAX_K) return fail(FORA_E_ARG, "kmax out of range");
  return run_queries(const_cast<fora_graph*>(g), batch, h_queries, kmax, d_ws, ws_bytes, d_ids,
                     d_vals, h_stats, (hipStream_t)stream);
}

int fora_dist_batch(const fora_graph* g, int32_t batch, const fora_query* h_queries,
                    const double* d_sigma, int32_t kmax, void* d_ws, size_t ws_bytes,
                    int32_t* d_ids, float* d_vals, fora_stats* h_stats, void* stream) {
  if (kmax < 1 || kmax > FORA_MAX_K) return fail(FORA_E_ARG, "kmax out of range");
  if (!d_sigma) return fail(FORA_E_ARG, "null source distributions");
  return run_queries(const_cast<fora_graph*>(g), batch, h_queries, kmax, d_ws, ws_bytes, d_ids,
                     d_vals, h_stats, (hipStream_t)stream, d_sigma);
}

int fora_build_index(fora_graph* g, double alpha, double walks_per_degree, uint32_t key0,
                     uint32_t key1, void* stream) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(FORA_E_ARG, "alpha must be in (0,1)");
  if (!(walks_per_degree >= 0.0 && std::isfinite(walks_per_degree)))
    return fail(FORA_E_ARG, "walks_per_degree must be finite and >= 0");
  if (std::ceil((double)g->dev.max_deg * walks_per_degree) >= 4294967296.0)
    return fail(FORA_E_OVERFLOW, "omega_max(v) >= 2^32 for the largest degree");
  hipStream_t s = (hipStream_t)stream;
  FORA_HIP(hipSetDevice(g->device));
  drop_graphs(g);  // captured pipelines hold the old index pointers
  if (g->idx_off_owned) (void)hipFree(g->idx_off_owned);
  if (g->idx_dest_owned) (void)hipFree(g->idx_dest_owned);
  g->idx_off_owned = nullptr;
  g->idx_dest_owned = nullptr;
  g->dev.idx_off = nullptr;
  g->dev.idx_dest = nullptr;
  g->idx_total = 0;
  const int64_t n = g->dev.n;
  const int64_t tiles = (n + 2047) / 2048;
  u64 *off = nullptr, *plan_gi = nullptr, *tsum = nullptr;
  Ctrl* ctrl = nullptr;
  QueryDev* qd = nullptr;
  StatSlot* qs = nullptr;
  int32_t* dest = nullptr;
  auto release = [&](bool keep) {
    if (plan_gi) (void)hipFree(plan_gi);
    if (tsum) (void)hipFree(tsum);
    if (ctrl) (void)hipFree(ctrl);
    if (qd) (void)hipFree(qd);
    if (qs) (void)hipFree(qs);
    if (!keep) {
      if (off) (void)hipFree(off);
      if (dest) (void)hipFree(dest);
    }
  };
  if (hipMalloc(&off, sizeof(u64) * (size_t)(n + 1)) != hipSuccess ||
      hipMalloc(&plan_gi, sizeof(u64) * (size_t)n) != hipSuccess ||
      hipMalloc(&tsum, sizeof(u64) * (size_t)tiles) != hipSuccess ||
      hipMalloc(&ctrl, sizeof(Ctrl)) != hipSuccess ||
      hipMalloc(&qd, sizeof(QueryDev)) != hipSuccess ||
      hipMalloc(&qs, sizeof(StatSlot) * kStatSlots) != hipSuccess) {
    release(false);
    return fail(FORA_E_NOMEM, "hipMalloc for the index build failed");
  }
  u64 total = 0;
  hipError_t e = launch_index_plan(g->dev, walks_per_degree, off, plan_gi, tsum, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&total, off + n, sizeof(u64), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release(false);
    return fail(FORA_E_HIP, std::string("index plan: ") + hipGetErrorString(e));
  }
  if (hipMalloc(&dest, sizeof(int32_t) * (size_t)std::max<u64>(total, 1)) != hipSuccess) {
    release(false);
    return fail(FORA_E_NOMEM, "hipMalloc of the index failed");
  }
  std::vector<unsigned char> zero(sizeof(Ctrl), 0);
  Ctrl* hc = reinterpret_cast<Ctrl*>(zero.data());
  hc->walks = total;
  hc->entries = (u64)n;
  QueryDev hq{};
  hq.key0 = key0;
  hq.key1 = key1;
  hq.alpha = alpha;
  hq.t_alpha = (uint32_t)std::floor(std::ldexp(alpha, 32));
  e = hipMemcpyAsync(ctrl, zero.data(), sizeof(Ctrl), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(qd, &hq, sizeof(QueryDev), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_fill_zero(qs, sizeof(StatSlot) * kStatSlots, s);
  if (e == hipSuccess && total > 0)
    e = launch_index_walks(g->dev, plan_gi, off, ctrl, qd, qs, dest, walk_blocks(g),
                           walk_chunk(g), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    release(false);
    return fail(FORA_E_HIP, std::string("index walks: ") + hipGetErrorString(e));
  }
  release(true);
  g->idx_off_owned = off;
  g->idx_dest_owned = dest;
  g->idx_total = (int64_t)total;
  g->idx_alpha = alpha;
  g->idx_wpd = walks_per_degree;
  g->idx_key0 = key0;
  g->idx_key1 = key1;
  g->dev.idx_off = off;
  g->dev.idx_dest = dest;
  return FORA_OK;
}

int fora_index_info(const fora_graph* g, int64_t* total, double* alpha, double* walks_per_degree,
                    uint32_t* key0, uint32_t* key1) {
  if (!g) return fail(FORA_E_ARG, "null graph");
  if (total) *total = g->idx_dest_owned ? g->idx_total : 0;
  if (alpha) *alpha = g->idx_alpha;
  if (walks_per_degree) *walks_per_degree = g->idx_wpd;
  if (key0) *key0 = g->idx_key0;
  if (key1) *key1 = g->idx_key1;
  return FORA_OK;
}

int fora_index_export(const fora_graph* g, uint64_t* d_off, int32_t* d_dest, void* stream) {
  if (!g || !d_off || !d_dest) return fail(FORA_E_ARG, "null argument");
  if (!g->idx_dest_owned) return fail(FORA_E_ARG, "no index");
  hipStream_t s = (hipStream_t)stream;
  FORA_HIP(hipMemcpyAsync(d_off, g->idx_off_owned, sizeof(u64) * ((size_t)g->dev.n + 1),
                          hipMemcpyDeviceToDevice, s));
  if (g->idx_total > 0)
    FORA_HIP(hipMemcpyAsync(d_dest, g->idx_dest_owned, sizeof(int32_t) * (size_t)g->idx_total,
                            hipMemcpyDeviceToDevice, s));
  FORA_HIP(hipStreamSynchronize(s));
  return FORA_OK;
}

int fora_topk_workspace_size(const fora_graph* g, int32_t batch, int32_t kmax, size_t* bytes) {
  if (!g || !bytes) return fail(FORA_E_ARG, "null argument");
  if (batch < 1 || batch > FORA_MAX_BATCH) return fail(FORA_E_ARG, "batch out of range");
  if (kmax < 1 || kmax > FORA_MAX_K) return fail(FORA_E_ARG, "kmax out of range");
  const size_t rows = (size_t)batch * (size_t)kmax;
  *bytes = align_up(make_layout(g->dev, batch).total, 256) + align_up(rows * 4, 256) * 2 +
           align_up((size_t)batch * 4, 256) * 4;
  return FORA_OK;
}

// Algorithm 5: iterations of Algorithm 2 at halving delta for the queries
// that have not stopped yet; finished rows move from the staging rows at
// the end of the workspace to their final places.
int fora_topk_batch(const fora_graph* gc, int32_t batch, const fora_query* h_queries,
                    int32_t kmax, void* d_ws, size_t ws_bytes, int32_t* d_ids, float* d_vals,
                    fora_stats* h_stats, int32_t* h_iterations, double* h_delta, void* stream) {
  fora_graph* g = const_cast<fora_graph*>(gc);
  hipStream_t s = (hipStream_t)stream;
  if (!g || !h_queries || !d_ws || !d_ids || !d_vals) return fail(FORA_E_ARG, "null argument");
  size_t need = 0;
  int rc = fora_topk_workspace_size(g, batch, kmax, &need);
  if (rc != FORA_OK) return rc;
  if (ws_bytes < need) return fail(FORA_E_NOMEM, "workspace smaller than fora_topk_workspace_size");
  const int32_t n = g->dev.n;
  for (int b = 0; b < batch; ++b) {
    fora_query q = h_queries[b];
    q.delta = 1.0;  // replaced per iteration
    rc = check_query(g, q);
    if (rc != FORA_OK) return rc;
    if (q.k > kmax) return fail(FORA_E_ARG, "kmax smaller than a query's k");
  }
  // staging rows and small index arrays after the batched workspace
  const size_t rows = (size_t)batch * (size_t)kmax;
  char* p = (char*)d_ws + align_up(make_layout(g->dev, batch).total, 256);
  int32_t* st_ids = (int32_t*)p;
  p += align_up(rows * 4, 256);
  float* st_vals = (float*)p;
  p += align_up(rows * 4, 256);
  int32_t* d_k = (int32_t*)p;
  p += align_up((size_t)batch * 4, 256);
  float* d_kth = (float*)p;
  p += align_up((size_t)batch * 4, 256);
  int32_t* d_from = (int32_t*)p;
  p += align_up((size_t)batch * 4, 256);
  int32_t* d_to = (int32_t*)p;
  const size_t ws_main = make_layout(g->dev, batch).total;

  std::vector<int32_t> remaining(batch);
  for (int b = 0; b < batch; ++b) remaining[b] = b;
  std::vector<fora_query> qv;
  std::vector<fora_stats> st;
  std::vector<int32_t> ks, from, to;
  std::vector<float> kth;
  std::vector<double> delta_now(batch);
  for (int it = 0; !remaining.empty(); ++it) {
    const int B = (int)remaining.size();
    qv.assign(B, fora_query{});
    ks.resize(B);
    std::vector<char> last(B);
    for (int i = 0; i < B; ++i) {
      const fora_query& q0 = h_queries[remaining[i]];
      fora_query q = q0;
      const double top = 1.0 / (double)q0.k;
      const double floor_n = 1.0 / (double)n;
      double d = std::ldexp(top, -it);
      last[i] = !(d > floor_n);  // the sequence ends with one iteration at 1/n
      if (last[i]) d = floor_n;
      q.delta = d;
      q.eps = q0.eps / 2.0;
      q.pf = q0.pf / ((double)n * std::max(std::log2((double)n / (double)q0.k), 1.0));
      q.seed = q0.seed + (uint64_t)it;
      qv[i] = q;
      ks[i] = q0.k;
      delta_now[remaining[i]] = d;
    }
    st.assign(B, fora_stats{});
    rc = run_queries(g, B, qv.data(), kmax, d_ws, ws_main, st_ids, st_vals, st.data(), s);
    if (rc != FORA_OK) return rc;
    FORA_HIP(hipMemcpyAsync(d_k, ks.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    FORA_HIP(launch_topk_kth(st_vals, kmax, d_k, B, d_kth, s));
    kth.resize(B);
    FORA_HIP(hipMemcpyAsync(kth.data(), d_kth, sizeof(float) * B, hipMemcpyDeviceToHost, s));
    FORA_HIP(hipStreamSynchronize(s));
    from.clear();
    to.clear();
    std::vector<int32_t> next;
    for (int i = 0; i < B; ++i) {
      const int b = remaining[i];
      const double bound = (1.0 + h_queries[b].eps) * delta_now[b];
      if ((double)kth[i] >= bound || last[i]) {
        from.push_back(i);
        to.push_back(b);
        if (h_stats) h_stats[b] = st[i];
        if (h_iterations) h_iterations[b] = it + 1;
        if (h_delta) h_delta[b] = delta_now[b];
      } else {
        next.push_back(b);
      }
    }
    if (!from.empty()) {
      const int c = (int)from.size();
      FORA_HIP(hipMemcpyAsync(d_from, from.data(), sizeof(int32_t) * c, hipMemcpyHostToDevice, s));
      FORA_HIP(hipMemcpyAsync(d_to, to.data(), sizeof(int32_t) * c, hipMemcpyHostToDevice, s));
      FORA_HIP(launch_copy_rows(st_ids, st_vals, kmax, d_from, d_to, c, d_ids, d_vals, s));
      FORA_HIP(hipStreamSynchronize(s));
    }
    remaining.swap(next);
  }
  return FORA_OK;
}

int fora_push_only(const fora_graph* gc, int32_t src, double alpha, double rmax,
                   const double* d_sigma, void* d_ws, size_t ws_bytes, int32_t max_rounds,
                   int32_t* h_round_sizes, int32_t* d_frontiers, int64_t frontier_cap,
                   fora_stats* h_stats, void* stream) {
  fora_graph* g = const_cast<fora_graph*>(gc);
  hipStream_t s = (hipStream_t)stream;
  Call c;
  int rc = prepare(g, 1, d_ws, ws_bytes, c);
  if (rc != FORA_OK) return rc;
  if (!d_sigma && (src < 0 || src >= g->dev.n)) return fail(FORA_E_ARG, "source out of range");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(FORA_E_ARG, "alpha must be in (0,1)");
  if (!(rmax > 0.0 && std::isfinite(rmax))) return fail(FORA_E_ARG, "rmax must be > 0");
  if (max_rounds < 0) return fail(FORA_E_ARG, "max_rounds < 0");
  if (d_frontiers && frontier_cap < 0) return fail(FORA_E_ARG, "frontier_cap < 0");
  QueryDev qd{};
  qd.src = d_sigma ? 0 : src;
  qd.k = 1;
  qd.alpha = alpha;
  qd.rmax = rmax;
  qd.omega_unit = 1.0;
  FORA_HIP(hipSetDevice(g->device));
  FORA_HIP(launch_fill_zero((char*)d_ws + c.L.zero_begin, c.L.zero_end - c.L.zero_begin, s));
  FORA_HIP(hipMemcpyAsync(c.w.queries, &qd, sizeof(qd), hipMemcpyHostToDevice, s));
  if (d_sigma)
    FORA_HIP(launch_init_dist(g->dev, c.w, c.L, 1, d_sigma, s));
  else
    FORA_HIP(launch_init_queries(g->dev, c.w, 1, s));
  int rounds = 0;
  rc = run_push(g, c, 1, s, true, d_frontiers, d_frontiers ? frontier_cap : 0, &rounds);
  if (rc != FORA_OK) return rc;
  std::vector<QueryDev> qv(1, qd);
  fora_stats st{};
  rc = finish(g, c, 1, s, &st, qv);
  if (rc != FORA_OK) return rc;
  if (st.rounds > max_rounds && h_round_sizes)
    return fail(FORA_E_OVERFLOW, "more rounds than max_rounds");
  if (st.rounds > kMaxRoundsLogged && h_round_sizes)
    return fail(FORA_E_OVERFLOW, "too many rounds to log");
  if (h_round_sizes && st.rounds > 0) {
    std::vector<uint64_t> rs(st.rounds);
    FORA_HIP(hipMemcpy(rs.data(), c.w.ctrl->round_size, sizeof(uint64_t) * st.rounds,
                       hipMemcpyDeviceToHost));
    for (int i = 0; i < st.rounds; ++i) h_round_sizes[i] = (int32_t)rs[i];
  }
  if (h_stats) *h_stats = st;
  return FORA_OK;
}

int fora_walk_only(const fora_graph* gc, int64_t entries, const int32_t* d_v,
                   const uint64_t* d_omega, const double* d_w, uint32_t key0, uint32_t key1,
                   double alpha, void* d_ws, size_t ws_bytes, uint64_t* h_steps,
                   void* stream) {
  fora_graph* g = const_cast<fora_graph*>(gc);
  hipStream_t s = (hipStream_t)stream;
  Call c;
  int rc = prepare(g, 1, d_ws, ws_bytes, c);
  if (rc != FORA_OK) return rc;
  if (entries < 0 || entries > g->dev.n) return fail(FORA_E_ARG, "entries must be in [0, n]");
  if (entries > 0 && (!d_v || !d_omega || !d_w)) return fail(FORA_E_ARG, "null plan array");
  if (!(alpha > 0.0 && alpha < 1.0)) return fail(FORA_E_ARG, "alpha must be in (0,1)");
  QueryDev qd{};
  qd.key0 = key0;
  qd.key1 = key1;
  qd.alpha = alpha;
  qd.t_alpha = (uint32_t)std::floor(std::ldexp(alpha, 32));
  qd.flags = FORA_WALK_COUNTS;
  FORA_HIP(hipSetDevice(g->device));
  FORA_HIP(launch_fill_zero((char*)d_ws + c.L.zero_begin, c.L.zero_end - c.L.zero_begin, s));
  FORA_HIP(hipMemcpyAsync(c.w.queries, &qd, sizeof(qd), hipMemcpyHostToDevice, s));
  FORA_HIP(launch_clear_walk_sums(c.w, c.L, s));
  if (entries > 0) {
    FORA_HIP(launch_walk_plan_from_host(g->dev, c.w, entries, d_v, d_omega, d_w, s));
    FORA_HIP(launch_walks(g->dev, c.w, walk_blocks(g), call_chunk(g, c),
                                 call_agg(g, c), s));
  }
  std::vector<QueryDev> qv(1, qd);
  fora_stats st{};
  rc = finish(g, c, 1, s, &st, qv);
  if (rc != FORA_OK) return rc;
  if (h_steps) *h_steps = st.steps;
  return FORA_OK;
}

int fora_features(const fora_graph* g, int32_t count, const int32_t* d_srcs, double alpha,
                  double eps, double delta, double pf, float* d_features, void* stream) {
  if (!g || count < 0 || (count > 0 && (!d_srcs || !d_features)))
    return fail(FORA_E_ARG, "bad argument");
  fora_query q{};
  q.src = 0;
  q.k = 1;
  q.alpha = alpha;
  q.eps = eps;
  q.delta = delta;
  q.pf = pf;
  const int rc = check_query(g, q);
  if (rc != FORA_OK) return rc;
  const QueryDev qd = plan_query(g, q);
  FORA_HIP(launch_features(g->dev, count, d_srcs, alpha, eps, qd.rmax, d_features,
                           (hipStream_t)stream));
  return FORA_OK;
}

int fora_mlp_forward(int32_t count, const float* d_x, const float* d_params, float* d_y,
                     float* d_acts, void* stream) {
  if (count < 0 || (count > 0 && (!d_x || !d_params || !d_y)))
    return fail(FORA_E_ARG, "bad argument");
  FORA_HIP(launch_mlp_forward(count, d_x, d_params, d_y, d_acts, (hipStream_t)stream));
  return FORA_OK;
}

int fora_mlp_backward(int32_t count, const float* d_x, const float* d_params,
                      const float* d_acts, const float* d_y, const float* d_target,
                      float* d_grad, float* d_loss, float* d_scratch, void* stream) {
  if (count < 1 || !d_x || !d_params || !d_acts || !d_y || !d_target || !d_grad || !d_loss ||
      !d_scratch)
    return fail(FORA_E_ARG, "bad argument");
  FORA_HIP(launch_mlp_backward(count, d_x, d_params, d_acts, d_y, d_target, d_grad, d_loss,
                               d_scratch, (hipStream_t)stream));
  return FORA_OK;
}

int fora_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, float lr,
                   float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!d_params || !d_grad || !d_m || !d_v || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f) ||
      !(beta1 < 1.0f) || !(beta2 >= 0.0f) || !(beta2 < 1.0f) || !(eps > 0.0f))
    return fail(FORA_E_ARG, "bad argument");
  FORA_HIP(launch_adam(d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, step,
                       (hipStream_t)stream));
  return FORA_OK;
}

int fora_mlp_to_bf16(const float* d_params, uint16_t* d_params_bf16, void* stream) {
  if (!d_params || !d_params_bf16) return fail(FORA_E_ARG, "bad argument");
  FORA_HIP(launch_to_bf16(FORA_MLP_PARAMS, d_params, d_params_bf16, (hipStream_t)stream));
  return FORA_OK;
}

int fora_mlp_forward_bf16(int32_t count, const float* d_x, const uint16_t* d_params_bf16,
                          float* d_y, void* stream) {
  if (count < 0 || (count > 0 && (!d_x || !d_params_bf16 || !d_y)))
    return fail(FORA_E_ARG, "bad argument");
  FORA_HIP(launch_mlp_forward_bf16(count, d_x, d_params_bf16, d_y, (hipStream_t)stream));
  return FORA_OK;
}

int fora_predict_rmax(const fora_graph* g, int32_t count, const int32_t* d_srcs, double alpha,
                      double eps, double delta, double pf, const uint16_t* d_params_bf16,
                      double log_lo, double log_hi, float* d_scratch, double* d_rmax,
                      int32_t* h_fallbacks, void* stream) {
  if (!g || count < 0 || (count > 0 && (!d_srcs || !d_params_bf16 || !d_scratch || !d_rmax)) ||
      !(log_lo <= log_hi))
    return fail(FORA_E_ARG, "bad argument");
  if (count == 0) {
    if (h_fallbacks) *h_fallbacks = 0;
    return FORA_OK;
  }
  fora_query q{};
  q.k = 1;
  q.alpha = alpha;
  q.eps = eps;
  q.delta = delta;
  q.pf = pf;
  int rc = check_query(g, q);
  if (rc != FORA_OK) return rc;
  const QueryDev qd = plan_query(g, q);
  hipStream_t s = (hipStream_t)stream;
  float* feat = d_scratch;
  float* y = d_scratch + (size_t)count * FORA_MLP_FEATURES;
  // the fallback counter follows the features and the outputs
  int* fb = (int*)(d_scratch + (size_t)count * 8);
  FORA_HIP(launch_fill_zero(fb, sizeof(int), s));
  FORA_HIP(launch_features(g->dev, count, d_srcs, alpha, eps, qd.rmax, feat, s));
  FORA_HIP(launch_mlp_forward_bf16(count, feat, d_params_bf16, y, s));
  FORA_HIP(launch_rmax_from_output(count, y, qd.rmax, log_lo, log_hi, d_rmax, fb, s));
  if (h_fallbacks) {
    int v = 0;
    FORA_HIP(hipMemcpyAsync(&v, fb, sizeof(int), hipMemcpyDeviceToHost, s));
    FORA_HIP(hipStreamSynchronize(s));
    *h_fallbacks = v;
  }
  return FORA_OK;
}

int fora_push_sweep(const fora_graph* gc, int32_t batch, const fora_query* h_queries,
                    int32_t nthr, const double* h_mult, void* d_ws, size_t ws_bytes,
                    int64_t* h_edge_ops, uint64_t* h_walks, void* stream) {
  fora_graph* g = const_cast<fora_graph*>(gc);
  hipStream_t s = (hipStream_t)stream;
  if (!h_queries || !h_mult || !h_edge_ops || !h_walks || nthr < 1)
    return fail(FORA_E_ARG, "bad argument");
  for (int i = 0; i < nthr; ++i) {
    if (!(h_mult[i] > 0.0) || !std::isfinite(h_mult[i]) || (i > 0 && !(h_mult[i] < h_mult[i - 1])))
      return fail(FORA_E_ARG, "multipliers must be positive and strictly decreasing");
  }
  Call c;
  int rc = prepare(g, batch, d_ws, ws_bytes, c);
  if (rc != FORA_OK) return rc;
  std::vector<QueryDev> qd(batch), base(batch);
  for (int b = 0; b < batch; ++b) {
    fora_query q = h_queries[b];
    q.rmax = 0.0;
    q.flags = 0;  // the sweep measures Algorithm 1 and 2 as they stand
    q.walk_cost = 0.0;
    rc = check_query(g, q);
    if (rc != FORA_OK) return rc;
    base[b] = plan_query(g, q);
  }
  FORA_HIP(hipSetDevice(g->device));
  // W per query lives in the top-k histogram area, unused by this call
  u64* walks = (u64*)c.w.hist;
  FORA_HIP(launch_fill_zero((char*)d_ws + c.L.zero_begin, c.L.zero_end - c.L.zero_begin, s));
  int t = 0;
  std::vector<StatSlot> slots((size_t)batch * kStatSlots);
  std::vector<u64> w(batch);
  for (int i = 0; i < nthr; ++i) {
    for (int b = 0; b < batch; ++b) {
      qd[b] = base[b];
      qd[b].rmax = base[b].rmax * h_mult[i];
    }
    FORA_HIP(hipMemcpyAsync(c.w.queries, qd.data(), sizeof(QueryDev) * batch,
                            hipMemcpyHostToDevice, s));
    if (i == 0) FORA_HIP(launch_init_queries(g->dev, c.w, batch, s));
    else FORA_HIP(launch_seed_frontier(g->dev, c.w, c.L, batch, t, s));
    int rounds = 0;
    rc = run_push(g, c, batch, s, true, nullptr, 0, &rounds, t);
    if (rc != FORA_OK) return rc;
    t = rounds;
    FORA_HIP(launch_fill_zero(walks, sizeof(u64) * batch, s));
    FORA_HIP(launch_count_walks(g->dev, c.w, c.L, batch, walks, s));
    FORA_HIP(hipMemcpyAsync(w.data(), walks, sizeof(u64) * batch, hipMemcpyDeviceToHost, s));
    FORA_HIP(hipMemcpyAsync(slots.data(), c.w.qstats, sizeof(StatSlot) * slots.size(),
                            hipMemcpyDeviceToHost, s));
    FORA_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < batch; ++b) {
      int64_t e = 0;
      for (int k = 0; k < kStatSlots; ++k) e += (int64_t)slots[(size_t)b * kStatSlots + k].edge_ops;
      h_edge_ops[(size_t)b * nthr + i] = e;
      h_walks[(size_t)b * nthr + i] = w[b];
    }
  }
  int flags = 0;
  FORA_HIP(hipMemcpy(&flags, &c.w.ctrl->error, sizeof(int), hipMemcpyDeviceToHost));
  return error_code_from_flags(flags);
}

int fora_graph_rank(const fora_graph* g, int32_t* d_rank, void* stream) {
  if (!g || !d_rank) return fail(FORA_E_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  FORA_HIP(hipMemcpyAsync(d_rank, g->dev.rank, sizeof(int32_t) * (size_t)g->dev.n,
                          hipMemcpyDeviceToDevice, s));
  FORA_HIP(hipStreamSynchronize(s));
  return FORA_OK;
}

int fora_philox(int64_t count, const uint32_t* d_ctr, uint32_t key0, uint32_t key1,
                uint32_t* d_out, void* stream) {
  if (count < 0) return fail(FORA_E_ARG, "count < 0");
  if (count > 0 && (!d_ctr || !d_out)) return fail(FORA_E_ARG, "null array");
  FORA_HIP(launch_philox(count, d_ctr, key0, key1, d_out, (hipStream_t)stream));
  return FORA_OK;
}

}  // extern "C"
