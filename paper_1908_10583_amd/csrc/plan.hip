// Walk plan (Algorithm 2, the loop over nodes with residue): for every
// (query b, node v) with r(v) > 0,
//   omega_v = ceil(r(v) * omega_unit)          (FP64 from the fixed-point residue)
//   weight  = round(r(v) / omega_v * 2^62)     (unsigned fixed point)
// and an exclusive scan of omega_v over (b, v) in row-major order gives every
// walk a global id. With FORA_PRUNE_ZERO_HOP (Algorithm 3) the walks carry
// r'(v) = (1 - alpha) r(v) instead. Also collects r_sum per query (an exact
// integer sum of the fixed-point residues) and counts residues left above
// r_max * d(v) (must be zero after the push).
#include <algorithm>

#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kPlanThreads = 256;
constexpr int kPlanPerThread = kPlanTile / kPlanThreads;  // 8 consecutive nodes
constexpr int kScanThreads = 1024;

// Tile pass 1: entries and walks per tile, per-query totals.
__global__ __launch_bounds__(kPlanThreads) void k_plan_count(
    const u64* __restrict__ r, const QueryDev* __restrict__ Q, QueryStatsDev* QS,
    const int2* __restrict__ info, int n, int tiles_per_row, uint32_t* tile_cnt,
    u64* tile_walks, Ctrl* ctrl) {
  __shared__ u64 s_r[kPlanTile];
  __shared__ u64 s_tmp[kPlanThreads / 64];
  if (ctrl->skip) return;  // uniform: the push has not finished (graph replay)
  const int b = blockIdx.y;
  const int v0 = blockIdx.x * kPlanTile;
  const u64* row = r + (size_t)b * n;
  for (int k = threadIdx.x; k < kPlanTile; k += kPlanThreads) {
    const int v = v0 + k;
    s_r[k] = v < n ? row[v] : 0ull;
  }
  __syncthreads();
  const double wu = Q[b].omega_unit;
  const double rmax = Q[b].rmax;
  const double scale = (Q[b].flags & FORA_PRUNE_ZERO_HOP) ? 1.0 - Q[b].alpha : 1.0;
  u64 c = 0, walks = 0, viol = 0, rs = 0;
  bool ovf = false;
#pragma unroll
  for (int k = 0; k < kPlanPerThread; ++k) {
    const int lv = threadIdx.x * kPlanPerThread + k;
    const u64 rfx = s_r[lv];
    if (rfx != 0ull) {
      const double rv = fx_to_double(rfx);
      const double om = ceil((scale == 1.0 ? rv : scale * rv) * wu);
      ovf |= om >= 4294967296.0;
      ++c;
      walks += (u64)om;
      rs += rfx;
      if (rfx > fx_threshold(rmax, info[v0 + lv].y)) ++viol;
    }
  }
  if (ovf) atomicOr(&ctrl->error, kErrOmegaOverflow);
  const u64 tc = block_sum(c, s_tmp);
  const u64 tw = block_sum(walks, s_tmp);
  const u64 tv = block_sum(viol, s_tmp);
  const u64 trs = block_sum(rs, s_tmp);
  if (threadIdx.x == 0) {
    const size_t tile = (size_t)b * tiles_per_row + blockIdx.x;
    tile_cnt[tile] = (uint32_t)tc;
    tile_walks[tile] = tw;
    StatSlot* st = &QS[(size_t)b * kStatSlots + (blockIdx.x & (kStatSlots - 1))];
    if (tc) {
      atomicAdd(&st->entries, tc);
      atomicAdd(&st->walks, tw);
      atomicAdd(&st->r_sum_fx, trs);
    }
    if (tv) atomicAdd(&st->term_violations, (int)tv);
  }
}

// One block scans all tile counts (exclusive); writes totals and the sentinel.
__global__ __launch_bounds__(kScanThreads) void k_plan_scan(
    const uint32_t* tile_cnt, const u64* tile_walks, int64_t ntiles, u64* tile_eoff,
    u64* tile_woff, u64* plan_off, Ctrl* ctrl) {
  __shared__ u64 s_tmp[kScanThreads / 64];
  if (ctrl->skip) {
    if (threadIdx.x == 0) {
      ctrl->entries = 0;
      ctrl->walks = 0;
    }
    return;
  }
  u64 carry_e = 0, carry_w = 0;
  for (int64_t base = 0; base < ntiles; base += kScanThreads) {
    const int64_t i = base + threadIdx.x;
    const u64 ce = i < ntiles ? (u64)tile_cnt[i] : 0ull;
    const u64 cw = i < ntiles ? tile_walks[i] : 0ull;
    u64 te, tw;
    const u64 pe = block_exclusive_scan(ce, s_tmp, te);
    const u64 pw = block_exclusive_scan(cw, s_tmp, tw);
    if (i < ntiles) {
      tile_eoff[i] = carry_e + pe;
      tile_woff[i] = carry_w + pw;
    }
    carry_e += te;
    carry_w += tw;
  }
  if (threadIdx.x == 0) {
    ctrl->entries = carry_e;
    ctrl->walks = carry_w;
    plan_off[carry_e] = carry_w;
    ctrl->chunk_next = 0;
  }
}

// Tile pass 2: write the plan entries in (query, node) order.
__global__ __launch_bounds__(kPlanThreads) void k_plan_write(
    const u64* __restrict__ r, const QueryDev* __restrict__ Q, int n, int tiles_per_row,
    const u64* tile_eoff, const u64* tile_woff, u64* plan_gi, u64* plan_off, u64* plan_wfx,
    const Ctrl* ctrl) {
  __shared__ u64 s_r[kPlanTile];
  __shared__ u64 s_tmp[kPlanThreads / 64];
  if (ctrl->skip) return;
  const int b = blockIdx.y;
  const int v0 = blockIdx.x * kPlanTile;
  const u64* row = r + (size_t)b * n;
  for (int k = threadIdx.x; k < kPlanTile; k += kPlanThreads) {
    const int v = v0 + k;
    s_r[k] = v < n ? row[v] : 0ull;
  }
  __syncthreads();
  const size_t tile = (size_t)b * tiles_per_row + blockIdx.x;
  const double wu = Q[b].omega_unit;
  const double scale = (Q[b].flags & FORA_PRUNE_ZERO_HOP) ? 1.0 - Q[b].alpha : 1.0;
  u64 c = 0, walks = 0;
  double om[kPlanPerThread];
#pragma unroll
  for (int k = 0; k < kPlanPerThread; ++k) {
    const double rv = fx_to_double(s_r[threadIdx.x * kPlanPerThread + k]);
    om[k] = rv > 0.0 ? ceil((scale == 1.0 ? rv : scale * rv) * wu) : 0.0;
    c += rv > 0.0 ? 1 : 0;
    walks += (u64)om[k];
  }
  u64 tc, tw;
  u64 e = tile_eoff[tile] + block_exclusive_scan(c, s_tmp, tc);
  u64 woff = tile_woff[tile] + block_exclusive_scan(walks, s_tmp, tw);
#pragma unroll
  for (int k = 0; k < kPlanPerThread; ++k) {
    const int lv = threadIdx.x * kPlanPerThread + k;
    const double rv = fx_to_double(s_r[lv]);
    if (rv > 0.0) {
      plan_gi[e] = ((u64)b << 32) | (uint32_t)(v0 + lv);
      plan_off[e] = woff;
      const double rw = scale == 1.0 ? rv : scale * rv;
      plan_wfx[e] = __double2ull_rn((rw / om[k]) * kFx);
      ++e;
      woff += (u64)om[k];
    }
  }
}

// The walk phase's end-point sums share memory with the push's frontier
// arrays, so they are cleared once the push is over (a kernel, so that it can
// sit in a captured graph; skipped while the push still runs there).
__global__ __launch_bounds__(256) void k_clear_walk_sums(const Ctrl* ctrl, u64* __restrict__ acc,
                                                         u64* __restrict__ cnt, u64 cap) {
  if (ctrl->skip) return;
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += stride) {
    acc[i] = 0ull;
    cnt[i] = 0ull;
  }
}

hipError_t launch_clear_walk_sums(const Ws& w, const Layout& L, hipStream_t s) {
  const u64 cap = (u64)L.cap;
  const u64 blocks = std::min<u64>((cap + 255) / 256, 8192);
  k_clear_walk_sums<<<(unsigned)std::max<u64>(blocks, 1), 256, 0, s>>>(w.ctrl, w.acc, w.cnt, cap);
  return hipGetLastError();
}

hipError_t launch_plan(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                       hipStream_t s) {
  const hipError_t e = launch_clear_walk_sums(w, L, s);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)L.tiles_per_row, (unsigned)batch);
  k_plan_count<<<grid, kPlanThreads, 0, s>>>(w.r, w.queries, w.qstats, g.info, g.n,
                                             (int)L.tiles_per_row, w.tile_cnt, w.tile_walks,
                                             w.ctrl);
  k_plan_scan<<<1, kScanThreads, 0, s>>>(w.tile_cnt, w.tile_walks, L.tiles_per_row * batch,
                                         w.tile_eoff, w.tile_woff, w.plan_off, w.ctrl);
  k_plan_write<<<grid, kPlanThreads, 0, s>>>(w.r, w.queries, g.n, (int)L.tiles_per_row,
                                             w.tile_eoff, w.tile_woff, w.plan_gi, w.plan_off,
                                             w.plan_wfx, w.ctrl);
  return hipGetLastError();
}

// Graph replays run a fixed number of push rounds; if any frontier is still
// non-empty the rest of the replay is skipped and the host finishes it.
__global__ void k_push_gate(Ctrl* ctrl, int rounds) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl->skip = ctrl->fr_cnt[rounds & 1] != 0 ? 1 : 0;
}

hipError_t launch_push_gate(const Ws& w, int rounds, hipStream_t s) {
  k_push_gate<<<1, 64, 0, s>>>(w.ctrl, rounds);
  return hipGetLastError();
}

// W per query for the current residues (no plan written): sum over v of
// ceil(r(v) * omega_unit).
__global__ __launch_bounds__(kPlanThreads) void k_count_walks(const u64* __restrict__ r,
                                                              const QueryDev* __restrict__ Q,
                                                              int n, u64* walks) {
  __shared__ u64 s_tmp[kPlanThreads / 64];
  const int b = blockIdx.y;
  const double wu = Q[b].omega_unit;
  const u64* row = r + (size_t)b * n;
  u64 acc = 0;
  for (int k = threadIdx.x; k < kPlanTile; k += kPlanThreads) {
    const int v = blockIdx.x * kPlanTile + k;
    if (v < n) {
      const u64 rfx = row[v];
      if (rfx != 0ull) acc += (u64)ceil(fx_to_double(rfx) * wu);
    }
  }
  const u64 t = block_sum(acc, s_tmp);
  if (threadIdx.x == 0 && t) atomicAdd(&walks[b], t);
}

hipError_t launch_count_walks(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                              u64* walks, hipStream_t s) {
  dim3 grid((unsigned)L.tiles_per_row, (unsigned)batch);
  k_count_walks<<<grid, kPlanThreads, 0, s>>>(w.r, w.queries, g.n, walks);
  return hipGetLastError();
}

// ---- a caller-given plan (walk phase on its own) ---------------------------
// Entries (v, omega, w) for query 0: tile sums of omega, scan, then offsets.
// Also checks the caller's nodes: ids in [0, n), strictly increasing (a walk
// from an id outside the graph would read outside the node table).
__global__ __launch_bounds__(kPlanThreads) void k_hplan_count(const int32_t* v_in,
                                                              const uint64_t* omega,
                                                              int64_t entries, int32_t n,
                                                              uint32_t* tile_cnt,
                                                              u64* tile_walks, Ctrl* ctrl) {
  __shared__ u64 s_tmp[kPlanThreads / 64];
  u64 c = 0, walks = 0;
  bool bad = false, bad_v = false;
  for (int k = 0; k < kPlanPerThread; ++k) {
    const int64_t e = (int64_t)blockIdx.x * kPlanTile + threadIdx.x * kPlanPerThread + k;
    if (e < entries) {
      const u64 o = omega[e];
      const int32_t v = v_in[e];
      bad |= (o == 0) | (o >= 4294967296ull);
      bad_v |= v < 0 || v >= n || (e > 0 && v <= v_in[e - 1]);
      ++c;
      walks += o;
    }
  }
  if (bad) atomicOr(&ctrl->error, kErrOmegaOverflow);
  if (bad_v) atomicOr(&ctrl->error, kErrBadPlan);
  const u64 tc = block_sum(c, s_tmp);
  const u64 tw = block_sum(walks, s_tmp);
  if (threadIdx.x == 0) {
    tile_cnt[blockIdx.x] = (uint32_t)tc;
    tile_walks[blockIdx.x] = tw;
  }
}

__global__ __launch_bounds__(kPlanThreads) void k_hplan_write(
    const int32_t* v, const uint64_t* omega, const double* wgt, int64_t entries,
    const u64* tile_woff, u64* plan_gi, u64* plan_off, u64* plan_wfx) {
  __shared__ u64 s_tmp[kPlanThreads / 64];
  u64 walks = 0;
  const int64_t e0 = (int64_t)blockIdx.x * kPlanTile + threadIdx.x * kPlanPerThread;
  for (int k = 0; k < kPlanPerThread; ++k)
    if (e0 + k < entries) walks += omega[e0 + k];
  u64 tw;
  u64 woff = tile_woff[blockIdx.x] + block_exclusive_scan(walks, s_tmp, tw);
  for (int k = 0; k < kPlanPerThread; ++k) {
    const int64_t e = e0 + k;
    if (e < entries) {
      plan_gi[e] = (uint32_t)v[e];
      plan_off[e] = woff;
      plan_wfx[e] = __double2ull_rn(wgt[e] * kFx);
      woff += omega[e];
    }
  }
}

hipError_t launch_walk_plan_from_host(const GraphDev& g, const Ws& w, int64_t entries,
                                      const int32_t* d_v, const uint64_t* d_omega,
                                      const double* d_w, hipStream_t s) {

  const int64_t tiles = (entries + kPlanTile - 1) / kPlanTile;
  if (tiles == 0) return hipSuccess;
  k_hplan_count<<<(unsigned)tiles, kPlanThreads, 0, s>>>(d_v, d_omega, entries, g.n,
                                                         w.tile_cnt, w.tile_walks, w.ctrl);
  k_plan_scan<<<1, kScanThreads, 0, s>>>(w.tile_cnt, w.tile_walks, tiles, w.tile_eoff,
                                         w.tile_woff, w.plan_off, w.ctrl);
  k_hplan_write<<<(unsigned)tiles, kPlanThreads, 0, s>>>(d_v, d_omega, d_w, entries,
                                                         w.tile_woff, w.plan_gi, w.plan_off,
                                                         w.plan_wfx);
  return hipGetLastError();
}

}  // namespace fora
