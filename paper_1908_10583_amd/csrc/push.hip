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

// Per-query counters are staged in LDS (dynamic: 12 bytes per query).
__global__ __launch_bounds__(256) void k_push_snapshot(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, float* __restrict__ frx,
    float* __restrict__ r, float* __restrict__ q, const QueryDev* __restrict__ Q,
    QueryStatsDev* QS, const int2* __restrict__ info, int n, int batch, int stats,
    int32_t* frontier_log, int64_t log_cap, u64 cap) {
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
    for (int b = threadIdx.x; b < batch; b += blockDim.x) {
      if (s_push[b]) {
        atomicAdd(&QS[b].pushes, (u64)s_push[b]);
        atomicAdd(&QS[b].edge_ops, s_edges[b]);
        atomicMax(&QS[b].rounds, t + 1);
      }
    }
  }
}

__global__ __launch_bounds__(kScatterBlock) void k_push_scatter(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, const float* __restrict__ frx,
    u64* __restrict__ fr_out, u64 cap, float* __restrict__ r, const QueryDev* __restrict__ Q,
    const int2* __restrict__ info, const int32_t* __restrict__ colidx, int n) {
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
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->log_len += cnt;
  u64* out_cnt = &ctrl->fr_cnt[(t + 1) & 1];
  if (threadIdx.x == 0) s_qn = 0;

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
      deg = (u64)inf.y;
    }
    u64 total;
    const u64 pre = block_exclusive_scan(deg, s_tmp, total);
    s_pre[threadIdx.x] = pre;
    __syncthreads();
    const int last = (int)((cnt - base < (u64)kScatterBlock) ? (cnt - base) : kScatterBlock) - 1;
    for (u64 k = threadIdx.x; k < total; k += kScatterBlock) {
      // owner entry: the largest j with s_pre[j] <= k (degrees are >= 1)
      int lo = 0, hi = last;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      const int b = (int)s_ent_b[lo];
      const int u = colidx[(int64_t)s_start[lo] + (int64_t)(k - s_pre[lo])];
      const float inc = s_inc[lo];
      const double rmax = s_rmax[lo];
      const size_t gi = (size_t)b * n + u;
      const float old = unsafeAtomicAdd(&r[gi], inc);
      const float now = old + inc;
      // every threshold is at least r_max (d >= 1): cheap pre-filter
      if ((double)now > rmax) {
        const double thr = rmax * (double)info[u].y;
        if ((double)old <= thr && (double)now > thr) {
          const u64 ent = ((u64)b << 32) | (uint32_t)u;
          const unsigned slot = atomicAdd(&s_qn, 1u);
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
  }
}

hipError_t launch_push_round(const GraphDev& g, const Ws& w, int batch, int t, int blocks,
                             bool stats, int32_t* frontier_log, int64_t log_cap,
                             hipStream_t s) {
  const int par = t & 1;
  const size_t smem = stats ? (size_t)batch * (sizeof(u64) + sizeof(uint32_t)) : 0;
  const u64 cap = (u64)batch * (u64)g.n;
  k_push_snapshot<<<blocks, 256, smem, s>>>(t, w.ctrl, w.fr[par], w.frx, w.r, w.q, w.queries,
                                            w.qstats, g.info, g.n, batch, stats ? 1 : 0,
                                            frontier_log, log_cap, cap);
  k_push_scatter<<<blocks, kScatterBlock, 0, s>>>(t, w.ctrl, w.fr[par], w.frx, w.fr[par ^ 1],
                                                  cap, w.r, w.queries, g.info, g.colidx, g.n);
  return hipGetLastError();
}

}  // namespace fora
