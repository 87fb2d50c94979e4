// Random walks with restart from the walk plan (Algorithm 2's walk loop).
//
// Walk g (a global id) belongs to plan entry e with plan_off[e] <= g <
// plan_off[e+1]; it is walk j = g - plan_off[e] of start node v for query b.
// Step s of the walk draws one Philox4x32-10 block with key (source, seed)
// and counter (v, j, s, 0): it stops at the current node x if word 0 is
// below floor(alpha * 2^32); otherwise it moves to out-neighbour
// floor(U * d(x) / 2^64) of x, where U = word1 * 2^32 + word2. At its end
// point t it adds its entry's fixed-point weight to acc[t], and 1 to cnt[t]
// if the query asked for walk counts (FORA_WALK_COUNTS).
// With FORA_PRUNE_ZERO_HOP (Algorithm 3) the step-0 block only chooses the
// first move: every walk starts at a random out-neighbour of v.
//
// With FORA_USE_INDEX (FORA+, section 3.3) walk j of v, if j < omega_max(v),
// is read from the graph's walk-destination index instead of being run: the
// index holds the end points of the same walks (keyed by the index key), so
// results are the same as running them. STORE builds that index.
//
// With AGG, a wave first adds its end points to a wave-private LDS table
// keyed by (query, node) and moves the table's sums to HBM when it holds
// kAggFlushAt keys and at the end; repeated end points (walks from one start
// node that stop there or at its few neighbours) then cost one HBM atomic
// pair per flush instead of one per walk. The sums are integers, so the
// result is the same either way.
//
// Moves read the walk records (GraphDev): a move loads one 8-byte unit of
// the current record, which holds the chosen neighbour's record start and
// out-degree (and its id, where the graph's sizes let the three fit), so
// each move is one dependent load. Without ids in the slots, the end node's
// id is read from its record's header where the walk stops; a degree too
// wide for its field (a hub's) is read from the header when it is reached.
//
// Schedule: a persistent grid; each wavefront takes chunks of `chunk`
// consecutive walk ids from a device work queue and keeps all 64 lanes busy:
// a lane whose walk ends takes the next id of the chunk at once (ballot +
// lane rank), so geometric walk lengths do not leave lanes idle. The entry of
// a new id is found by a shuffle binary search over a 64-entry window of
// plan offsets that the wave keeps in registers. Per-query step totals go to
// one of kStatSlots slots per query, chosen by wave, so that lanes crossing a
// query boundary at the same time do not all add to one address.
#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kWalkBlock = 256;
constexpr int kWalkWaves = kWalkBlock / 64;
// end-point aggregation: a wave-private LDS table of (query, node) keys
constexpr int kAggSlots = 256;
constexpr int kAggProbes = 4;
constexpr int kAggFlushAt = 160;  // keys held before the wave flushes its table
constexpr u64 kAggEmpty = ~0ull;

struct AggTable {
  u64* key;
  u64* cnt;
  u64* acc;
};

// Adds one end point to the wave's table; false if no slot was found within
// kAggProbes probes (the caller then adds it to HBM directly). *fresh is set
// when the key took a new slot.
__device__ __forceinline__ bool agg_add(const AggTable& t, u64 gi, u64 wfx, bool count,
                                        bool* fresh) {
  uint32_t h = (uint32_t)(gi * 0x9E3779B97F4A7C15ull >> 56);  // 8-bit multiplicative hash
  for (int p = 0; p < kAggProbes; ++p) {
    const uint32_t s = (h + (uint32_t)p) & (kAggSlots - 1);
    const u64 old = atomicCAS(&t.key[s], kAggEmpty, gi);
    if (old == kAggEmpty || old == gi) {
      *fresh = old == kAggEmpty;
      if (count) atomicAdd(&t.cnt[s], 1ull);
      atomicAdd(&t.acc[s], wfx);
      return true;
    }
  }
  return false;
}

// Wave-uniform: moves every held key to HBM and empties the table.
__device__ __forceinline__ void agg_flush(const AggTable& t, u64* __restrict__ cnt,
                                          u64* __restrict__ acc) {
  __builtin_amdgcn_wave_barrier();
  for (int s = threadIdx.x & 63; s < kAggSlots; s += 64) {
    const u64 k = t.key[s];
    if (k != kAggEmpty) {
      if (t.cnt[s] != 0) atomicAdd(&cnt[k], t.cnt[s]);
      atomicAdd(&acc[k], t.acc[s]);
      t.key[s] = kAggEmpty;
      t.cnt[s] = 0;
      t.acc[s] = 0;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Largest e in [0, E) with off[e] <= target, by 64-way probing (wave-uniform).
__device__ __forceinline__ u64 wave_find_entry(const u64* __restrict__ off, u64 E, u64 target) {
  const int lane = threadIdx.x & 63;
  u64 lo = 0, hi = E;  // off[lo] <= target (off[0] = 0); hi == E or off[hi] > target
  while (hi - lo > 64) {
    const u64 step = (hi - lo + 63) / 64;
    const u64 p = lo + (u64)lane * step;
    const bool ok = p < hi && off[p] <= target;
    const u64 mask = __ballot(ok);
    const int top = 63 - __builtin_clzll(mask);
    lo = lo + (u64)top * step;
    const u64 nh = lo + step;
    hi = nh < hi ? nh : hi;
  }
  const u64 p = lo + (u64)lane;
  const bool ok = p < hi && off[p] <= target;
  const u64 mask = __ballot(ok);
  return lo + (u64)(63 - __builtin_clzll(mask));
}

// STORE: the index build; walk g's end point goes to store[g] (no weights).
template <bool AGG, bool STORE>
__global__ __launch_bounds__(kWalkBlock) void k_walks(
    const u64* __restrict__ plan_gi, const u64* __restrict__ plan_off,
    const u64* __restrict__ plan_wfx, Ctrl* ctrl, const QueryDev* __restrict__ Q,
    QueryStatsDev* QS, const int2* __restrict__ info, const u64* __restrict__ rec,
    const uint32_t* __restrict__ rec_q, int qbits, int dbits, int slot_ids,
    const u64* __restrict__ idx_off, const int32_t* __restrict__ idx_dest, int n,
    u64* __restrict__ cnt, u64* __restrict__ acc, int32_t* __restrict__ store, int chunk) {
  __shared__ u64 s_agg[AGG ? 3 * kWalkWaves * kAggSlots : 1];
  if (ctrl->error || ctrl->skip) return;
  const u64 W = ctrl->walks;
  const u64 E = ctrl->entries;
  const u64 nchunks = (W + chunk - 1) / (u64)chunk;
  const int lane = threadIdx.x & 63;
  const int slot = (int)(((blockIdx.x << 2) + (threadIdx.x >> 6)) & (kStatSlots - 1));
  const u64 qmask = (1ull << qbits) - 1;  // qbits <= 32, dbits <= 32
  const u64 dmask = (1ull << dbits) - 1;
  const int ishift = qbits + dbits;        // < 64 where slot_ids is set

  AggTable agg{};
  unsigned agg_fill = 0;  // wave-uniform count of keys in the table
  if (AGG) {
    u64* base = s_agg + (size_t)(threadIdx.x >> 6) * 3 * kAggSlots;
    agg = AggTable{base, base + kAggSlots, base + 2 * kAggSlots};
    for (int s = lane; s < kAggSlots; s += 64) {
      agg.key[s] = kAggEmpty;
      agg.cnt[s] = 0;
      agg.acc[s] = 0;
    }
    __builtin_amdgcn_wave_barrier();
  }
  bool active = false;
  int b = 0;
  uint32_t v = 0, j = 0, step = 0, k0 = 0, k1 = 0, ta = 0;
  int32_t x = 0;
  uint32_t q = 0, deg = 1;  // record start and out-degree of x
  bool forced = false;      // FORA_PRUNE_ZERO_HOP: the next step must move
  bool indexed = false;     // FORA_USE_INDEX: x is the stored end point of the walk
  bool counts = false;      // FORA_WALK_COUNTS
  u64 gid = 0;              // the walk's global id (STORE)
  u64 wfx = 0;
  int stat_b = -1;
  u64 stat_steps = 0;

  u64 cursor = 0, cend = 0, ebase = 0;
  u64 woff = ~0ull;  // plan_off[ebase + lane], or all-ones past the end
  bool more = true;

  for (;;) {
    const u64 free_mask = __ballot(!active);
    if (free_mask != 0 && more) {
      if (cursor >= cend) {
        u64 c = 0;
        if (lane == 0) c = atomicAdd(&ctrl->chunk_next, 1ull);
        c = __shfl(c, 0, 64);
        if (c >= nchunks) {
          more = false;
        } else {
          cursor = c * (u64)chunk;
          cend = cursor + chunk < W ? cursor + chunk : W;
          ebase = wave_find_entry(plan_off, E, cursor);
          woff = (ebase + lane <= E) ? plan_off[ebase + lane] : ~0ull;
        }
      }
      if (more) {
        // ids below the window's last offset map into the window
        const u64 wlast = __shfl(woff, 63, 64);
        const u64 limit = cend < wlast ? cend : wlast;
        const u64 navail = limit - cursor;
        const unsigned nfree = (unsigned)__popcll(free_mask);
        const unsigned nassign = (u64)nfree < navail ? nfree : (unsigned)navail;
        const unsigned rank = lane_rank(free_mask);
        const u64 id = cursor + rank;
        // largest L with woff_L <= id (all lanes run the search)
        int lo = 0;
#pragma unroll
        for (int s = 32; s > 0; s >>= 1) {
          const u64 o = __shfl(woff, lo + s, 64);
          if (o <= id) lo += s;
        }
        const u64 o_lo = __shfl(woff, lo, 64);
        if (!active && rank < nassign) {
          const u64 e = ebase + (u64)lo;
          const u64 gi = plan_gi[e];
          wfx = STORE ? 0ull : plan_wfx[e];
          b = (int)(gi >> 32);
          v = (uint32_t)gi;
          j = (uint32_t)(id - o_lo);
          gid = id;
          x = (int32_t)v;
          step = 0;
          k0 = Q[b].key0;
          k1 = Q[b].key1;
          ta = Q[b].t_alpha;
          forced = (Q[b].flags & FORA_PRUNE_ZERO_HOP) != 0;
          counts = (Q[b].flags & FORA_WALK_COUNTS) != 0;
          indexed = false;
          if (!STORE && (Q[b].flags & FORA_USE_INDEX)) {
            // walk j of v is stored if j < omega_max(v); later ones run live
            const u64 o0 = idx_off[v];
            if ((u64)j < idx_off[v + 1] - o0) {
              x = idx_dest[o0 + j];
              indexed = true;
            }
          }
          if (!indexed) {
            deg = (uint32_t)info[v].y;
            q = rec_q[v];
          }
          active = true;
        }
        cursor += nassign;
        if (cursor < cend) {
          int lc = 0;
#pragma unroll
          for (int s = 32; s > 0; s >>= 1) {
            const u64 o = __shfl(woff, lc + s, 64);
            if (o <= cursor) lc += s;
          }
          if (lc > 0) {
            ebase += (u64)lc;
            woff = (ebase + lane <= E) ? plan_off[ebase + lane] : ~0ull;
          }
        }
      }
    }
    if (!__any(active)) {
      if (!more) break;
      continue;
    }
    if (AGG && agg_fill > kAggFlushAt) {
      agg_flush(agg, cnt, acc);
      agg_fill = 0;
    }
    bool fresh = false;
    if (active) {
      uint4 y = make_uint4(0u, 0u, 0u, 0u);
      if (!indexed) y = philox4x32_10(make_uint4(v, j, step, 0u), k0, k1);
      if (indexed || (!forced && y.x < ta)) {
        if (!indexed && step != 0 && !slot_ids) x = (int32_t)(rec[q] >> 32);  // header's id
        const size_t t = (size_t)b * n + x;
        if (STORE) {
          store[gid] = x;
        } else if (!AGG || !agg_add(agg, (u64)t, wfx, counts, &fresh)) {
          if (counts) atomicAdd(&cnt[t], 1ull);
          atomicAdd(&acc[t], wfx);
        }
        if (b != stat_b) {
          if (stat_b >= 0) atomicAdd(&QS[(size_t)stat_b * kStatSlots + slot].steps, stat_steps);
          stat_b = b;
          stat_steps = 0;
        }
        stat_steps += step;
        active = false;
      } else {
        // the chosen neighbour's record start and degree (and id), in one unit
        const uint32_t idx = mul_shift_index(y.y, y.z, deg);
        const u64 u = rec[(size_t)q + 1 + idx];
        q = (uint32_t)(u & qmask);
        deg = (uint32_t)((u >> qbits) & dmask);
        if (deg == (uint32_t)dmask) deg = (uint32_t)rec[q];  // too wide: the header's
        if (slot_ids) x = (int32_t)(u >> ishift);
        ++step;
        forced = false;
      }
    }
    if (AGG) agg_fill += (unsigned)__popcll(__ballot(fresh));
  }
  if (AGG) agg_flush(agg, cnt, acc);
  // per-query step totals: one atomic per wave when the wave saw one query
  const int b0 = __shfl(stat_b, 0, 64);
  const u64 mine = (stat_b == b0) ? stat_steps : 0ull;
  const u64 sum = wave_sum(mine);
  if (lane == 0 && b0 >= 0) atomicAdd(&QS[(size_t)b0 * kStatSlots + slot].steps, sum);
  if (stat_b != b0 && stat_b >= 0)
    atomicAdd(&QS[(size_t)stat_b * kStatSlots + slot].steps, stat_steps);
}

hipError_t launch_walks(const GraphDev& g, const Ws& w, int blocks, int chunk, bool agg,
                        hipStream_t s) {
  if (agg)
    k_walks<true, false><<<blocks, kWalkBlock, 0, s>>>(
        w.plan_gi, w.plan_off, w.plan_wfx, w.ctrl, w.queries, w.qstats, g.info, g.rec, g.rec_q,
        g.slot_qbits, g.slot_dbits, g.slot_ids, g.idx_off, g.idx_dest, g.n, w.cnt, w.acc, nullptr, chunk);
  else
    k_walks<false, false><<<blocks, kWalkBlock, 0, s>>>(
        w.plan_gi, w.plan_off, w.plan_wfx, w.ctrl, w.queries, w.qstats, g.info, g.rec, g.rec_q,
        g.slot_qbits, g.slot_dbits, g.slot_ids, g.idx_off, g.idx_dest, g.n, w.cnt, w.acc, nullptr, chunk);
  return hipGetLastError();
}

// The index build: plan (v, omega_max(v)) for every node with offsets off,
// one query entry Q (the index key), end points into dest.
hipError_t launch_index_walks(const GraphDev& g, const u64* plan_gi, const u64* off, Ctrl* ctrl,
                              const QueryDev* Q, QueryStatsDev* QS, int32_t* dest, int blocks,
                              int chunk, hipStream_t s) {
  k_walks<false, true><<<blocks, kWalkBlock, 0, s>>>(plan_gi, off, nullptr, ctrl, Q, QS, g.info,
                                                     g.rec, g.rec_q, g.slot_qbits, g.slot_dbits,
                                                     g.slot_ids, nullptr, nullptr, g.n,
                                                     nullptr, nullptr, dest, chunk);
  return hipGetLastError();
}

}  // namespace fora
