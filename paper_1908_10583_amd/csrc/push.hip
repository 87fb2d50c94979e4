// Forward Push (Algorithm 1) as synchronous rounds over a frontier queue.
//
// Round t, for every query of the batch at once:
//   F_t = { v : r(v) > r_max * d(v) }   (kept as a queue, built by round t-1)
//   snapshot: x_v = r(v); r(v) = 0; q(v) += alpha x_v; inc_v = (1-alpha) x_v / d(v)
//   scatter:  r(u) += inc_v for u in N_out(v); the one increment that lifts
//             r(u) over r_max * d(u) appends u to F_{t+1}.
// Snapshot and scatter are separate launches, so every frontier residue is
// read before any increment of the same round lands. The residue test is
// made in FP64 on the FP32 residue (never a division).
//
// Load balance: entries of degree <= kHubDeg are expanded per block (a block
// takes 256 entries, scans their degrees in LDS and spreads the edges over
// its threads). Entries of larger degree are listed by the snapshot and cut
// into pieces of kHubPiece edges that any block may take, so a hub does not
// hold up a round on one block.
#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kScatterBlock = 256;
constexpr unsigned kQueueCap = 1024;  // LDS-staged next-frontier entries per block

__global__ void k_init_queries(const QueryDev* Q, int batch, int n, const int2* info, float* r,
                               u64* fr0, Ctrl* ctrl) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int s = Q[b].src;
  r[(size_t)b * n + s] = 1.0f;
  if (1.0 > Q[b].rmax * (double)info[s].y) {
    const u64 pos = atomicAdd(&ctrl->fr_cnt[0], 1ull);
    fr0[pos] = ((u64)b << 32) | (uint32_t)s;
  }
}

hipError_t launch_init_queries(const GraphDev& g, const Ws& w, int batch, hipStream_t s) {
  k_init_queries<<<(batch + 255) / 256, 256, 0, s>>>(w.queries, batch, g.n, g.info, w.r,
                                                     w.fr[0], w.ctrl);
  return hipGetLastError();
}

// Per-query counters are staged in LDS (dynamic: 12 bytes per query) and
// added to the block's stat slot.
__global__ __launch_bounds__(256) void k_push_snapshot(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, float* __restrict__ frx,
    float* __restrict__ r, float* __restrict__ q, const QueryDev* __restrict__ Q,
    StatSlot* slots, const int2* __restrict__ info, int n, int batch, int stats,
    int32_t* frontier_log, int64_t log_cap, u64 cap, u64* hub_idx, u64* hub_base,
    u64 hub_cap) {
  extern __shared__ unsigned char smem[];
  u64* s_edges = (u64*)smem;
  uint32_t* s_push = (uint32_t*)(s_edges + batch);
  if (stats) {
    for (int i = threadIdx.x; i < batch; i += blockDim.x) {
      s_edges[i] = 0;
      s_push[i] = 0;
    }
    __syncthreads();
  }
  u64 cnt = ctrl->fr_cnt[t & 1];
  if (cnt > cap) cnt = cap;  // an overflow was already flagged by the producer
  const u64 log_base = ctrl->log_len;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->fr_cnt[(t + 1) & 1] = 0;
    if (t < kMaxRoundsLogged) ctrl->round_size[t] = cnt;
  }
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (u64)gridDim.x * blockDim.x) {
    const u64 e = fr_in[i];
    const int b = (int)(e >> 32);
    const int v = (int)(uint32_t)e;
    const size_t gi = (size_t)b * n + v;
    const float x = r[gi];
    r[gi] = 0.0f;
    const double alpha = Q[b].alpha;
    q[gi] = (float)((double)q[gi] + alpha * (double)x);
    const int d = info[v].y;
    frx[i] = (float)(((1.0 - alpha) * (double)x) / (double)d);
    if (d > kHubDeg) {
      const u64 pieces = (u64)((d + kHubPiece - 1) / kHubPiece);
      const u64 old = atomicAdd(&ctrl->hub_ctr[t & 1], (1ull << 40) | pieces);
      const u64 slot = old >> 40;
      if (slot < hub_cap) {
        hub_idx[slot] = i;
        hub_base[slot] = old & ((1ull << 40) - 1);
      } else {
        atomicOr(&ctrl->error, kErrFrontierOverflow);
      }
    }
    if (stats) {
      atomicAdd(&s_push[b], 1u);
      atomicAdd(&s_edges[b], (u64)d);
    }
    if (frontier_log) {
      const u64 pos = log_base + i;
      if (pos < (u64)log_cap) frontier_log[pos] = v;
      else atomicOr(&ctrl->error, kErrLogOverflow);
    }
  }
  if (stats) {
    __syncthreads();
    const int slot = blockIdx.x & (kStatSlots - 1);
    for (int b = threadIdx.x; b < batch; b += blockDim.x) {
      if (s_push[b]) {
        StatSlot* st = &slots[(size_t)b * kStatSlots + slot];
        atomicAdd(&st->pushes, (u64)s_push[b]);
        atomicAdd(&st->edge_ops, s_edges[b]);
        atomicMax(&st->rounds, t + 1);
      }
    }
  }
}

// Apply one residue increment; the increment that lifts r(u) over its
// threshold enqueues u (staged in LDS, spilling to the global queue).
__device__ __forceinline__ void push_edge(int b, int u, float inc, double rmax,
                                          float* __restrict__ r, int n,
                                          const int2* __restrict__ info, unsigned* s_qn,
                                          u64* s_queue, u64* out_cnt, u64* fr_out, u64 cap,
                                          Ctrl* ctrl) {
  const size_t gi = (size_t)b * n + u;
  const float old = unsafeAtomicAdd(&r[gi], inc);
  const float now = old + inc;
  // every threshold is at least r_max (d >= 1): cheap pre-filter
  if ((double)now > rmax) {
    const double thr = rmax * (double)info[u].y;
    if ((double)old <= thr && (double)now > thr) {
      const u64 ent = ((u64)b << 32) | (uint32_t)u;
      const unsigned slot = atomicAdd(s_qn, 1u);
      if (slot < kQueueCap) {
        s_queue[slot] = ent;
      } else {
        const u64 pos = atomicAdd(out_cnt, 1ull);
        if (pos < cap) fr_out[pos] = ent;
        else atomicOr(&ctrl->error, kErrFrontierOverflow);
      }
    }
  }
}

__global__ __launch_bounds__(kScatterBlock) void k_push_scatter(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, const float* __restrict__ frx,
    u64* __restrict__ fr_out, u64 cap, float* __restrict__ r, const QueryDev* __restrict__ Q,
    const int2* __restrict__ info, const int32_t* __restrict__ colidx, int n,
    const u64* __restrict__ hub_idx, const u64* __restrict__ hub_base, u64 hub_cap) {
  __shared__ u64 s_pre[kScatterBlock];
  __shared__ int32_t s_start[kScatterBlock];
  __shared__ uint32_t s_ent_b[kScatterBlock];
  __shared__ float s_inc[kScatterBlock];
  __shared__ double s_rmax[kScatterBlock];
  __shared__ u64 s_queue[kQueueCap];
  __shared__ unsigned s_qn;
  __shared__ u64 s_qbase;
  __shared__ u64 s_tmp[kScatterBlock / 64];

  u64 cnt = ctrl->fr_cnt[t & 1];
  if (cnt > cap) cnt = cap;
  const u64 hubs = ctrl->hub_ctr[t & 1];
  u64 nhub = hubs >> 40;
  if (nhub > hub_cap) nhub = hub_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctrl->log_len += cnt;
    ctrl->hub_ctr[(t + 1) & 1] = 0;
  }
  u64* out_cnt = &ctrl->fr_cnt[(t + 1) & 1];
  if (threadIdx.x == 0) s_qn = 0;
  __syncthreads();

  auto flush = [&]() {
    __syncthreads();
    const unsigned qn = s_qn < kQueueCap ? s_qn : kQueueCap;
    if (threadIdx.x == 0) s_qbase = qn ? atomicAdd(out_cnt, (u64)qn) : 0ull;
    __syncthreads();
    for (unsigned k = threadIdx.x; k < qn; k += kScatterBlock) {
      const u64 pos = s_qbase + k;
      if (pos < cap) fr_out[pos] = s_queue[k];
      else atomicOr(&ctrl->error, kErrFrontierOverflow);
    }
    __syncthreads();
    if (threadIdx.x == 0) s_qn = 0;
    __syncthreads();
  };

  // pieces of split (high-degree) entries, shared by all blocks
  const u64 total_pieces = (hubs & ((1ull << 40) - 1));
  for (u64 p = blockIdx.x; p < total_pieces && nhub; p += gridDim.x) {
    // owner: the last split entry whose first piece is <= p
    u64 lo = 0, hi = nhub - 1;
    while (lo < hi) {
      const u64 mid = (lo + hi + 1) >> 1;
      if (hub_base[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const u64 i = hub_idx[lo];
    const u64 e = fr_in[i];
    const int b = (int)(e >> 32);
    const int v = (int)(uint32_t)e;
    const int2 inf = info[v];
    const float inc = frx[i];
    const double rmax = Q[b].rmax;
    const int64_t first = (int64_t)(p - hub_base[lo]) * kHubPiece;
    const int64_t last = first + kHubPiece < inf.y ? first + kHubPiece : inf.y;
    for (int64_t k = first + threadIdx.x; k < last; k += kScatterBlock)
      push_edge(b, colidx[(int64_t)inf.x + k], inc, rmax, r, n, info, &s_qn, s_queue, out_cnt,
                fr_out, cap, ctrl);
    // all threads read the queue length after the barrier, so the decision
    // to flush (which contains barriers) is the same for the whole block
    __syncthreads();
    const bool full = s_qn > kQueueCap / 2;
    if (full) flush();
  }
  flush();

  // entries of degree <= kHubDeg, 256 per block-chunk
  for (u64 base = (u64)blockIdx.x * kScatterBlock; base < cnt;
       base += (u64)gridDim.x * kScatterBlock) {
    const u64 i = base + threadIdx.x;
    u64 deg = 0;
    if (i < cnt) {
      const u64 e = fr_in[i];
      const int v = (int)(uint32_t)e;
      const int b = (int)(e >> 32);
      const int2 inf = info[v];
      s_start[threadIdx.x] = inf.x;
      s_ent_b[threadIdx.x] = (uint32_t)b;
      s_inc[threadIdx.x] = frx[i];
      s_rmax[threadIdx.x] = Q[b].rmax;
      deg = inf.y > kHubDeg ? 0ull : (u64)inf.y;
    }
    u64 total;
    const u64 pre = block_exclusive_scan(deg, s_tmp, total);
    s_pre[threadIdx.x] = pre;
    __syncthreads();
    const int last = (int)((cnt - base < (u64)kScatterBlock) ? (cnt - base) : kScatterBlock) - 1;
    for (u64 k = threadIdx.x; k < total; k += kScatterBlock) {
      // owner entry: the largest j with s_pre[j] <= k among entries of
      // non-zero (expanded) degree
      int lo = 0, hi = last;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      push_edge((int)s_ent_b[lo], colidx[(int64_t)s_start[lo] + (int64_t)(k - s_pre[lo])],
                s_inc[lo], s_rmax[lo], r, n, info, &s_qn, s_queue, out_cnt, fr_out, cap, ctrl);
    }
    flush();
  }
}

hipError_t launch_push_round(const GraphDev& g, const Ws& w, const Layout& L, int batch, int t,
                             int blocks, bool stats, int32_t* frontier_log, int64_t log_cap,
                             hipStream_t s) {
  const int par = t & 1;
  const size_t smem = stats ? (size_t)batch * (sizeof(u64) + sizeof(uint32_t)) : 0;
  const u64 cap = (u64)L.cap;
  k_push_snapshot<<<blocks, 256, smem, s>>>(t, w.ctrl, w.fr[par], w.frx, w.r, w.q, w.queries,
                                            w.qstats, g.info, g.n, batch, stats ? 1 : 0,
                                            frontier_log, log_cap, cap, w.hub_idx, w.hub_base,
                                            (u64)L.hub_cap);
  k_push_scatter<<<blocks, kScatterBlock, 0, s>>>(t, w.ctrl, w.fr[par], w.frx, w.fr[par ^ 1],
                                                  cap, w.r, w.queries, g.info, g.colidx, g.n,
                                                  w.hub_idx, w.hub_base, (u64)L.hub_cap);
  return hipGetLastError();
}

}  // namespace fora
