// Forward Push (Algorithm 1) as synchronous rounds over a frontier queue.
//
// Round t, for every query of the batch at once:
//   F_t = { v : r(v) > r_max * d(v) }   (kept as a queue, built by round t-1)
//   snapshot: x_v = r(v); r(v) = 0; q(v) += alpha x_v; inc_v = (1-alpha) x_v / d(v)
//   then r(u) += sum of inc_v over v in F_t with u in N_out(v), and every u
//   whose residue now exceeds r_max * d(u) joins F_{t+1}.
// The snapshot is its own launch, so every frontier residue is read before
// any increment of the same round lands. Residues are unsigned fixed point
// with 62 fraction bits: inc_v is formed once in FP64 and rounded to it, and
// the sums are integer additions, so the result does not depend on the order
// in which increments land (nor on the batch a query runs in). The push test
// compares the integer residue with floor(r_max d(v) 2^62), which is the
// exact test against the FP64 threshold (never a division).
//
// The increments are applied in one of two ways, chosen per query and round:
// * push (sparse rounds): each frontier edge does a memory-side 64-bit
//   integer atomic on r(u); the increment that lifts r(u) over its threshold
//   enqueues u.
//   Entries of degree <= kHubDeg are expanded per block (256 entries, degrees
//   scanned in LDS); larger ones are cut into kHubPiece-edge pieces that any
//   block may take.
// * pull (dense rounds, frontier edges * pull_ratio > n + m, pull_ratio from
//   the tuning, kPullRatio by default): every node sums
//   the dense increments of its in-neighbours over the reverse graph (LDS
//   accumulation, no atomics to HBM), then updates r(u) once and tests it.
//   The dense increments sit at each node's degree rank (GraphDev::rank),
//   and the reverse graph stores in-neighbours by rank, so the gathers of
//   high-degree nodes' increments (the most frequent ones) share lines.
//   Queries are taken in groups of G = pull_group_for(batch) (16 for
//   large batches), whose increments for one node form one unit (128 bytes,
//   one line, at G = 16): a pull reads each in-edge's source once per group, so the
//   random reads per in-edge do not grow with the number of pulling
//   queries.
//   Nodes of in-degree above kHubDeg are summed in pieces by any block and
//   added with one atomic per piece.
#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kScatterBlock = 256;
// Position of query b's increment for the node of degree rank rk, with G
// queries per unit (a power of two).
__device__ __forceinline__ size_t incd_index(int b, int32_t rk, int n, int G) {
  return ((size_t)(b / G) * (size_t)n + (size_t)rk) * (size_t)G + (size_t)(b % G);
}

// The G increments of unit w of a group's rows.
template <int G>
__device__ __forceinline__ void load_unit(const u64* __restrict__ grow, int32_t w,
                                          u64 (&v)[G]) {
  if constexpr (G == 1) {
    v[0] = grow[w];
  } else {
    static_assert(G % 2 == 0, "units of two");
    const ulonglong2* u = reinterpret_cast<const ulonglong2*>(grow) + (size_t)w * (G / 2);
#pragma unroll
    for (int h = 0; h < G / 2; ++h) {
      const ulonglong2 x = u[h];
      v[2 * h] = x.x;
      v[2 * h + 1] = x.y;
    }
  }
}
constexpr unsigned kQueueCap = 1024;  // LDS-staged next-frontier entries per block

// FORA_BALANCE: the push stops once its residue increments reach the
// estimated walk cost (1 - alpha mass) (1 - alpha) omega_unit walk_cost, with
// mass the residue pushed so far (an exact integer sum of fixed-point x).
__device__ __forceinline__ bool balance_met(const QueryDev& q, u64 edge_ops, u64 mass_fx) {
  const double mass = fx_to_double(mass_fx);
  const double est = (1.0 - q.alpha * mass) * (1.0 - q.alpha) * q.omega_unit * q.walk_cost;
  return (double)edge_ops >= est;
}

__global__ void k_init_queries(const QueryDev* Q, int batch, int n, const int2* info, u64* r,
                               u64* fr0, Ctrl* ctrl, int32_t* stop, StatSlot* slots) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int s = Q[b].src;
  r[(size_t)b * n + s] = kFxOne;
  if ((Q[b].flags & FORA_BALANCE) && balance_met(Q[b], 0, 0ull)) {
    stop[b] = 1;
    slots[(size_t)b * kStatSlots].balance_stopped = 1;
  }
  if (kFxOne > fx_threshold(Q[b].rmax, info[s].y)) {
    const u64 pos = atomicAdd(&ctrl->fr_cnt[0], 1ull);
    fr0[pos] = ((u64)b << 32) | (uint32_t)s;
  }
}

hipError_t launch_init_queries(const GraphDev& g, const Ws& w, int batch, hipStream_t s) {
  k_init_queries<<<(batch + 255) / 256, 256, 0, s>>>(w.queries, batch, g.n, g.info, w.r,
                                                     w.fr[0], w.ctrl, w.stop, w.qstats);
  return hipGetLastError();
}

// Source distributions (section 6.2, the extension of Algorithm 1): the initial
// residue is sigma (rounded to the fixed point) instead of e_s; q starts at
// zero (the zero-filled rows). An entry outside [0, 1] is flagged.
__global__ void k_init_dist(const double* __restrict__ sigma, const QueryDev* Q, int batch,
                            int n, u64* r, Ctrl* ctrl, int32_t* stop, StatSlot* slots) {
  const u64 total = (u64)batch * (u64)n;
  bool bad = false;
  for (u64 gi = (u64)blockIdx.x * blockDim.x + threadIdx.x; gi < total;
       gi += (u64)gridDim.x * blockDim.x) {
    const double x = sigma[gi];
    const bool ok = x >= 0.0 && x <= 1.0;  // false for NaN
    bad |= !ok;
    r[gi] = ok ? fx_from_double(x) : 0ull;
  }
  if (bad) atomicOr(&ctrl->error, kErrBadDist);
  const u64 b = (u64)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < (u64)batch && (Q[b].flags & FORA_BALANCE) && balance_met(Q[b], 0, 0ull)) {
    stop[b] = 1;
    slots[b * kStatSlots].balance_stopped = 1;
  }
}

hipError_t launch_init_dist(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                            const double* sigma, hipStream_t s) {
  const u64 total = (u64)batch * (u64)g.n;
  const int blocks = (int)std::min<u64>(std::max<u64>((total + 255) / 256, 1), 16384);
  k_init_dist<<<blocks, 256, 0, s>>>(sigma, w.queries, batch, g.n, w.r, w.ctrl, w.stop,
                                     w.qstats);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_seed_frontier(g, w, L, batch, 0, s);
}

// Per-query counters are staged in LDS (dynamic: 12 bytes per query) and
// added to the block's stat slot and to this round's frontier-edge slot.
__global__ __launch_bounds__(256) void k_push_snapshot(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, u64* __restrict__ frx,
    u64* __restrict__ r, float* __restrict__ q, u64* __restrict__ incd,
    const QueryDev* __restrict__ Q, StatSlot* slots, u64* ecnt, const int2* __restrict__ info,
    const int32_t* __restrict__ rank, const int32_t* __restrict__ stop, int n, int batch,
    int32_t* frontier_log, int64_t log_cap, u64 cap, u64* hub_idx,
    u64* hub_base, u64 hub_cap) {
  extern __shared__ unsigned char smem[];
  u64* s_edges = (u64*)smem;
  uint32_t* s_push = (uint32_t*)(s_edges + batch);
  for (int i = threadIdx.x; i < batch; i += blockDim.x) {
    s_edges[i] = 0;
    s_push[i] = 0;
  }
  __syncthreads();
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
    if (stop[b] != 0 && t + 1 >= stop[b]) continue;  // the balance rule ended this push
    const size_t gi = (size_t)b * n + v;
    const u64 x_fx = r[gi];
    r[gi] = 0ull;
    if (Q[b].flags & FORA_BALANCE)
      atomicAdd(&slots[(size_t)b * kStatSlots + (blockIdx.x & (kStatSlots - 1))].mass_fx, x_fx);
    const double alpha = Q[b].alpha;
    const double x = fx_to_double(x_fx);
    q[gi] = (float)((double)q[gi] + alpha * x);
    const int d = info[v].y;
    const u64 inc = fx_from_double(((1.0 - alpha) * x) / (double)d);
    frx[i] = inc;
    incd[incd_index(b, rank[v], n, pull_group_for(batch))] = inc;
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
    atomicAdd(&s_push[b], 1u);
    atomicAdd(&s_edges[b], (u64)d);
    if (frontier_log) {
      const u64 pos = log_base + i;
      if (pos < (u64)log_cap) frontier_log[pos] = v;
      else atomicOr(&ctrl->error, kErrLogOverflow);
    }
  }
  __syncthreads();
  const int slot = blockIdx.x & (kStatSlots - 1);
  u64* ec = ecnt + (size_t)(t & 1) * batch * kStatSlots;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    if (s_push[b]) {
      StatSlot* st = &slots[(size_t)b * kStatSlots + slot];
      atomicAdd(&st->pushes, (u64)s_push[b]);
      atomicAdd(&st->edge_ops, s_edges[b]);
      atomicMax(&st->rounds, t + 1);
      atomicAdd(&ec[(size_t)b * kStatSlots + slot], s_edges[b]);
    }
  }
}

// One block: choose pull or push for every query's round t; list the
// groups of pull_group_for(batch) queries with a pulling member; clear the
// next round's frontier-edge slots.
__global__ __launch_bounds__(256) void k_push_mode(int t, Ctrl* ctrl, u64* ecnt, int32_t* mode,
                                                   int32_t* pull_list, StatSlot* slots,
                                                   const QueryDev* __restrict__ Q,
                                                   int32_t* stop, int batch, u64 n_plus_m,
                                                   int pull_ratio) {
  __shared__ int32_t s_tmp[4];
  const u64* ec = ecnt + (size_t)(t & 1) * batch * kStatSlots;
  u64* ec_next = ecnt + (size_t)((t + 1) & 1) * batch * kStatSlots;
  int32_t carry = 0;
  for (int base = 0; base < batch; base += 256) {
    const int b = base + threadIdx.x;
    int32_t pull = 0;
    if (b < batch) {
      u64 edges = 0;
      for (int k = 0; k < kStatSlots; ++k) edges += ec[(size_t)b * kStatSlots + k];
      pull = (pull_ratio > 0 && edges > 0 && edges * (u64)pull_ratio > n_plus_m) ? 1 : 0;
      mode[b] = pull;
      if (pull) slots[(size_t)b * kStatSlots].pull_rounds += 1;
      // FORA_BALANCE: the test before round t+1, over everything pushed so far
      if ((Q[b].flags & FORA_BALANCE) && stop[b] == 0) {
        u64 fc = 0, mass = 0;
        for (int k = 0; k < kStatSlots; ++k) {
          fc += slots[(size_t)b * kStatSlots + k].edge_ops;
          mass += slots[(size_t)b * kStatSlots + k].mass_fx;
        }
        if (balance_met(Q[b], fc, mass)) {
          stop[b] = t + 2;
          slots[(size_t)b * kStatSlots].balance_stopped = 1;
        }
      }
    }
    // aligned runs of G lanes hold one group (base is a multiple of 256)
    const unsigned G = (unsigned)pull_group_for(batch);
    const unsigned lane = threadIdx.x & 63;
    const u64 bal = __ballot(pull != 0);
    const int32_t gmask = (int32_t)((bal >> (lane & ~(G - 1))) & ((1ull << G) - 1));
    const int32_t lead = ((lane & (G - 1)) == 0 && gmask != 0) ? 1 : 0;
    int32_t tot;
    const int32_t pos = carry + block_exclusive_scan(lead, s_tmp, tot);
    if (lead) pull_list[pos] = ((b / (int)G) << 16) | gmask;
    carry += tot;
  }
  for (size_t i = threadIdx.x; i < (size_t)batch * kStatSlots; i += 256) ec_next[i] = 0;
  if (threadIdx.x == 0) ctrl->npull = carry;
}

struct NextQueue {
  u64* s_queue;
  unsigned* s_qn;
  u64* s_qbase;
  u64* out_cnt;
  u64* fr_out;
  u64 cap;
  Ctrl* ctrl;

  __device__ __forceinline__ void push(u64 ent) const {
    const unsigned slot = atomicAdd(s_qn, 1u);
    if (slot < kQueueCap) {
      s_queue[slot] = ent;
    } else {
      const u64 pos = atomicAdd(out_cnt, 1ull);
      if (pos < cap) fr_out[pos] = ent;
      else atomicOr(&ctrl->error, kErrFrontierOverflow);
    }
  }
  // block-uniform: every thread of the block must call it
  __device__ __forceinline__ void flush() const {
    __syncthreads();
    const unsigned qn = *s_qn < kQueueCap ? *s_qn : kQueueCap;
    if (threadIdx.x == 0) *s_qbase = qn ? atomicAdd(out_cnt, (u64)qn) : 0ull;
    __syncthreads();
    for (unsigned k = threadIdx.x; k < qn; k += blockDim.x) {
      const u64 pos = *s_qbase + k;
      if (pos < cap) fr_out[pos] = s_queue[k];
      else atomicOr(&ctrl->error, kErrFrontierOverflow);
    }
    __syncthreads();
    if (threadIdx.x == 0) *s_qn = 0;
    __syncthreads();
  }
};

// Apply one residue increment in push mode; the increment that lifts r(u)
// over its threshold enqueues u.
__device__ __forceinline__ void push_edge(int b, int u, u64 inc, double rmax, u64 thr1,
                                          u64* __restrict__ r, int n,
                                          const int2* __restrict__ info, const NextQueue& nq) {
  const size_t gi = (size_t)b * n + u;
  const u64 old = atomicAdd(&r[gi], inc);
  const u64 now = old + inc;
  // every threshold is at least the degree-1 one (d >= 1): cheap pre-filter
  if (now > thr1) {
    const u64 thr = fx_threshold(rmax, info[u].y);
    if (old <= thr && now > thr) nq.push(((u64)b << 32) | (uint32_t)u);
  }
}

// Items: (chunk of kScatterBlock destination nodes, pull group), then
// (piece of a high-in-degree node, pull group). A chunk item scans the
// chunk's in-degrees, finds each in-edge's owner, and reads the source's
// increment unit once; each pulling member of the group sums its own
// increment into its LDS row. The nodes that cross their thresholds are
// appended to the next frontier with one reservation per chunk item (a
// block scan of the per-node crossing counts), not through a queue.
template <int G>
__global__ __launch_bounds__(kScatterBlock) void k_push_pull(
    int t, Ctrl* ctrl, u64* __restrict__ fr_out, u64 cap, u64* __restrict__ r,
    const u64* __restrict__ incd, const QueryDev* __restrict__ Q,
    const int32_t* __restrict__ pull_list, const int2* __restrict__ info,
    const int32_t* __restrict__ in_rowptr, const int32_t* __restrict__ in_colidx,
    const int32_t* __restrict__ inhub_node, const u64* __restrict__ inhub_base, int n_inhubs,
    u64 inhub_pieces, int n) {
  __shared__ u64 s_pre[kScatterBlock];
  __shared__ int32_t s_start[kScatterBlock];
  __shared__ u64 s_sum[G][kScatterBlock];
  __shared__ u64 s_tmp[kScatterBlock / 64];
  __shared__ u64 s_tmpu[kScatterBlock / 64];
  __shared__ u64 s_base;
  const int ngroups = ctrl->npull;
  if (ngroups == 0) return;  // uniform
  u64* out_cnt = &ctrl->fr_cnt[(t + 1) & 1];
  const u64 chunks = ((u64)n + kScatterBlock - 1) / kScatterBlock;
  const u64 chunk_items = chunks * (u64)ngroups;
  const u64 items = chunk_items + inhub_pieces * (u64)ngroups;
  for (u64 it = blockIdx.x; it < items; it += gridDim.x) {
    const bool is_chunk = it < chunk_items;
    const u64 gidx = is_chunk ? it / chunks : (it - chunk_items) / inhub_pieces;
    const int32_t entry = pull_list[gidx];
    const int grp = entry >> 16;
    const unsigned mask = (unsigned)entry & 0xFFFFu;
    const u64* grow = incd + (size_t)grp * n * G;
    if (is_chunk) {
      const u64 j = it % chunks;
      const int u0 = (int)(j * kScatterBlock);
      const int u = u0 + (int)threadIdx.x;
      u64 deg = 0;
      if (u < n) {
        const int32_t a = in_rowptr[u], c = in_rowptr[u + 1];
        s_start[threadIdx.x] = a;
        deg = (c - a) > kHubDeg ? 0ull : (u64)(c - a);
      }
      for (int g = 0; g < G; ++g) s_sum[g][threadIdx.x] = 0ull;
      u64 total;
      const u64 pre = block_exclusive_scan(deg, s_tmp, total);
      s_pre[threadIdx.x] = pre;
      __syncthreads();
      const int last = (n - u0 < kScatterBlock ? n - u0 : kScatterBlock) - 1;
      // merge path: thread t takes the in-edges [t per, (t + 1) per) of the
      // chunk in order, sums each node's run in registers and adds the sums
      // to LDS where a node's run ends
      const u64 per = (total + kScatterBlock - 1) / kScatterBlock;
      u64 k = (u64)threadIdx.x * per;
      const u64 kend = k + per < total ? k + per : total;
      if (k < kend) {
        // owner of k: the largest index with s_pre <= k (it has in-edges)
        int lo = 0, hi = last;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        u64 run_end = lo < last ? s_pre[lo + 1] : total;
        u64 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0ull;
        auto flush = [&](int node) {
#pragma unroll
          for (int g = 0; g < G; ++g) {
            if (((mask >> g) & 1u) && acc[g] != 0ull) atomicAdd(&s_sum[g][node], acc[g]);
            acc[g] = 0ull;
          }
        };
        for (; k < kend; ++k) {
          while (k >= run_end) {  // the node's run ended: move to the next with in-edges
            flush(lo);
            ++lo;
            run_end = lo < last ? s_pre[lo + 1] : total;
          }
          u64 v[G];
          load_unit<G>(grow, in_colidx[(int64_t)s_start[lo] + (int64_t)(k - s_pre[lo])], v);
#pragma unroll
          for (int g = 0; g < G; ++g) acc[g] += v[g];
        }
        flush(lo);
      }
      __syncthreads();
      // bit g: member g's residue at u is now over its threshold (u was not
      // in this round's frontier, so this is its only crossing)
      unsigned cross = 0u;
      if (u < n) {
        const int d_u = info[u].y;
        for (int g = 0; g < G; ++g) {
          const u64 add = s_sum[g][threadIdx.x];
          if (((mask >> g) & 1u) && add != 0ull) {
            const int b = grp * G + g;
            const size_t gi = (size_t)b * n + u;
            const u64 now = r[gi] + add;
            r[gi] = now;
            if (now > fx_threshold(Q[b].rmax, d_u)) cross |= 1u << g;
          }
        }
      }
      // the chunk's next-frontier entries: one reservation for the block
      u64 tot;
      u64 pos = block_exclusive_scan((u64)__popc(cross), s_tmp, tot);
      if (tot != 0ull) {  // uniform
        if (threadIdx.x == 0) s_base = atomicAdd(out_cnt, tot);
        __syncthreads();
        pos += s_base;
        for (unsigned m = cross; m != 0u; m &= m - 1u, ++pos) {
          const int b = grp * G + __ffs(m) - 1;
          if (pos < cap) fr_out[pos] = ((u64)b << 32) | (uint32_t)u;
          else atomicOr(&ctrl->error, kErrFrontierOverflow);
        }
      }
    } else {
      // a piece of a node with large in-degree
      const u64 p = (it - chunk_items) % inhub_pieces;
      int lo = 0, hi = n_inhubs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inhub_base[mid] <= p) lo = mid;
        else hi = mid - 1;
      }
      const int u = inhub_node[lo];
      const int64_t a = in_rowptr[u], c = in_rowptr[u + 1];
      const int64_t first = a + (int64_t)(p - inhub_base[lo]) * kHubPiece;
      const int64_t end = first + kHubPiece < c ? first + kHubPiece : c;
      u64 part[G];
#pragma unroll
      for (int g = 0; g < G; ++g) part[g] = 0ull;
      for (int64_t k = first + threadIdx.x; k < end; k += kScatterBlock) {
        u64 v[G];
        load_unit<G>(grow, in_colidx[k], v);
#pragma unroll
        for (int g = 0; g < G; ++g) part[g] += v[g];
      }
      u64 sums[G];
      for (int g = 0; g < G; ++g)
        sums[g] = ((mask >> g) & 1u) ? block_sum(part[g], s_tmpu) : 0ull;
      if (threadIdx.x == 0) {
        const int d_u = info[u].y;
        for (int g = 0; g < G; ++g) {
          if (!((mask >> g) & 1u) || sums[g] == 0ull) continue;
          const int b = grp * G + g;
          const size_t gi = (size_t)b * n + u;
          const u64 old = atomicAdd(&r[gi], sums[g]);
          const u64 now = old + sums[g];
          const u64 thr = fx_threshold(Q[b].rmax, d_u);
          if (old <= thr && now > thr) {
            const u64 pos = atomicAdd(out_cnt, 1ull);
            if (pos < cap) fr_out[pos] = ((u64)b << 32) | (uint32_t)u;
            else atomicOr(&ctrl->error, kErrFrontierOverflow);
          }
        }
      }
    }
    __syncthreads();  // LDS rows are rewritten by the next item
  }
}

__global__ __launch_bounds__(kScatterBlock) void k_push_scatter(
    int t, Ctrl* ctrl, const u64* __restrict__ fr_in, const u64* __restrict__ frx,
    u64* __restrict__ fr_out, u64 cap, u64* __restrict__ r, u64* __restrict__ incd,
    const int32_t* __restrict__ mode, const int32_t* __restrict__ stop,
    const QueryDev* __restrict__ Q, const int2* __restrict__ info,
    const int32_t* __restrict__ colidx, const int32_t* __restrict__ rank, int n,
    int pull_group, const u64* __restrict__ hub_idx,
    const u64* __restrict__ hub_base, u64 hub_cap) {
  __shared__ u64 s_pre[kScatterBlock];
  __shared__ int32_t s_start[kScatterBlock];
  __shared__ uint32_t s_ent_b[kScatterBlock];
  __shared__ u64 s_inc[kScatterBlock];
  __shared__ double s_rmax[kScatterBlock];
  __shared__ u64 s_thr1[kScatterBlock];
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
  const NextQueue nq{s_queue, &s_qn, &s_qbase, &ctrl->fr_cnt[(t + 1) & 1], fr_out, cap, ctrl};
  if (threadIdx.x == 0) s_qn = 0;
  // the dense increments were read by the pull launch; clear them
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < cnt;
       i += (u64)gridDim.x * blockDim.x) {
    const u64 e = fr_in[i];
    incd[incd_index((int)(e >> 32), rank[(uint32_t)e], n, pull_group)] = 0ull;
  }
  __syncthreads();

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
    if (mode[b]) continue;  // uniform per block: this query pulls this round
    const int v = (int)(uint32_t)e;
    const int2 inf = info[v];
    const u64 inc = frx[i];
    const double rmax = Q[b].rmax;
    const u64 thr1 = fx_threshold(rmax, 1);
    const int64_t first = (int64_t)(p - hub_base[lo]) * kHubPiece;
    const int64_t last = first + kHubPiece < inf.y ? first + kHubPiece : inf.y;
    for (int64_t k = first + threadIdx.x; k < last; k += kScatterBlock)
      push_edge(b, colidx[(int64_t)inf.x + k], inc, rmax, thr1, r, n, info, nq);
    // all threads read the queue length after the barrier, so the decision
    // to flush (which contains barriers) is the same for the whole block
    __syncthreads();
    const bool full = s_qn > kQueueCap / 2;
    if (full) nq.flush();
  }
  nq.flush();

  // entries of degree <= kHubDeg of push-mode queries, 256 per block-chunk
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
      s_thr1[threadIdx.x] = fx_threshold(Q[b].rmax, 1);
      const bool skip = mode[b] || (stop[b] != 0 && t + 1 >= stop[b]);
      deg = (inf.y > kHubDeg || skip) ? 0ull : (u64)inf.y;
    }
    u64 total;
    const u64 pre = block_exclusive_scan(deg, s_tmp, total);
    s_pre[threadIdx.x] = pre;
    __syncthreads();
    const int last = (int)((cnt - base < (u64)kScatterBlock) ? (cnt - base) : kScatterBlock) - 1;
    for (u64 k = threadIdx.x; k < total; k += kScatterBlock) {
      // owner entry: the largest j with s_pre[j] <= k; it has a non-zero
      // expanded degree (entries of expanded degree 0 never own an edge)
      int lo = 0, hi = last;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= k) lo = mid;
        else hi = mid - 1;
      }
      push_edge((int)s_ent_b[lo], colidx[(int64_t)s_start[lo] + (int64_t)(k - s_pre[lo])],
                s_inc[lo], s_rmax[lo], s_thr1[lo], r, n, info, nq);
    }
    nq.flush();
  }
}

// Frontier from scratch: every (query, node) whose residue exceeds the
// query's current threshold (used when a threshold is lowered mid-way).
__global__ __launch_bounds__(256) void k_seed_frontier(int t, Ctrl* ctrl,
                                                       const u64* __restrict__ r,
                                                       const QueryDev* __restrict__ Q,
                                                       const int2* __restrict__ info, int n,
                                                       int batch, u64* fr, u64 cap) {
  const u64 total = (u64)batch * (u64)n;
  const int lane = threadIdx.x & 63;
  for (u64 base = (u64)blockIdx.x * blockDim.x; base < total; base += (u64)gridDim.x * blockDim.x) {
    const u64 gi = base + threadIdx.x;
    bool over = false;
    int b = 0, v = 0;
    if (gi < total) {
      b = (int)(gi / (u64)n);
      v = (int)(gi - (u64)b * n);
      over = r[gi] > fx_threshold(Q[b].rmax, info[v].y);
    }
    const u64 mask = __ballot(over);
    u64 pos0 = 0;
    if (lane == 0 && mask) pos0 = atomicAdd(&ctrl->fr_cnt[t & 1], (u64)__popcll(mask));
    pos0 = __shfl(pos0, 0, 64);
    if (over) {
      const u64 pos = pos0 + lane_rank(mask);
      if (pos < cap) fr[pos] = ((u64)b << 32) | (uint32_t)v;
      else atomicOr(&ctrl->error, kErrFrontierOverflow);
    }
  }
}

hipError_t launch_seed_frontier(const GraphDev& g, const Ws& w, const Layout& L, int batch, int t,
                                hipStream_t s) {
  const u64 total = (u64)batch * (u64)g.n;
  const int blocks = (int)std::min<u64>((total + 255) / 256, 16384);
  k_seed_frontier<<<blocks, 256, 0, s>>>(t, w.ctrl, w.r, w.queries, g.info, g.n, batch,
                                         w.fr[t & 1], (u64)L.cap);
  return hipGetLastError();
}

hipError_t launch_push_round(const GraphDev& g, const Ws& w, const Layout& L, int batch, int t,
                             int blocks, int pull_ratio, int32_t* frontier_log, int64_t log_cap,
                             hipStream_t s) {
  const int par = t & 1;
  const size_t smem = (size_t)batch * (sizeof(u64) + sizeof(uint32_t));
  const u64 cap = (u64)L.cap;
  k_push_snapshot<<<blocks, 256, smem, s>>>(t, w.ctrl, w.fr[par], w.frx, w.r, w.q, w.incd,
                                            w.queries, w.qstats, w.ecnt, g.info, g.rank, w.stop,
                                            g.n, batch,
                                            frontier_log, log_cap, cap, w.hub_idx, w.hub_base,
                                            (u64)L.hub_cap);
  k_push_mode<<<1, 256, 0, s>>>(t, w.ctrl, w.ecnt, w.mode, w.pull_list, w.qstats, w.queries,
                                w.stop, batch, (u64)g.n + (u64)g.m, pull_ratio);
  const int pg = pull_group_for(batch);
  auto pull = pg == 16 ? k_push_pull<16> : (pg == 4 ? k_push_pull<4> : k_push_pull<1>);
  pull<<<blocks, kScatterBlock, 0, s>>>(t, w.ctrl, w.fr[par ^ 1], cap, w.r, w.incd, w.queries,
                                        w.pull_list, g.info, g.in_rowptr, g.in_colidx,
                                        g.inhub_node, g.inhub_base, g.n_inhubs, g.inhub_pieces,
                                        g.n);
  k_push_scatter<<<blocks, kScatterBlock, 0, s>>>(t, w.ctrl, w.fr[par], w.frx, w.fr[par ^ 1],
                                                  cap, w.r, w.incd, w.mode, w.stop, w.queries,
                                                  g.info, g.colidx, g.rank, g.n, pg, w.hub_idx,
                                                  w.hub_base, (u64)L.hub_cap);
  return hipGetLastError();
}

}  // namespace fora
