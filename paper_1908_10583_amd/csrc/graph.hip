// Graph ingest: the CSR checks, the per-node {row start, out-degree} table,
// the reverse CSR for pull rounds (its in-lists' order follows an atomic
// cursor and does not matter: pull sums are integers), the degree rank (a
// stable LSD radix sort), the walk records, and the FORA+ index plan; also
// a zero fill and the Philox block kernel used for RNG checks.
#include "internal.h"
#include "scan.h"

namespace fora {

__global__ void k_fill_zero(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

__global__ void k_fill_zero_bytes(unsigned char* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  // the workspace regions are 256-byte aligned; the tail is cleared bytewise
  const size_t n16 = bytes / 16;
  if (n16) {
    const int blocks = (int)std::min<size_t>((n16 + 255) / 256, 8192);
    k_fill_zero<<<blocks, 256, 0, s>>>((uint4*)p, n16);
  }
  const size_t tail = bytes - n16 * 16;
  if (tail) k_fill_zero_bytes<<<1, 64, 0, s>>>((unsigned char*)p + n16 * 16, tail);
  return hipGetLastError();
}

// Problem definition (section 2.1): out-adjacency lists; every node needs an
// out-neighbour for the walk to move and for Algorithm 1's division by d(v).
__global__ void k_check_rows(const int32_t* rowptr, int32_t n, int64_t m, int* flags,
                             int* maxdeg, int* hubs, int2* info) {
  int local_max = 0, local_hubs = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = rowptr[v], b = rowptr[v + 1];
    if (v == 0 && a != 0) atomicOr(flags, kErrGraphRowptr);
    if (v == n - 1 && (int64_t)b != m) atomicOr(flags, kErrGraphRowptr);
    if (b < a) atomicOr(flags, kErrGraphRowptr);
    if (b == a) atomicOr(flags, kErrGraphDangling);
    const int d = b - a;
    local_max = d > local_max ? d : local_max;
    local_hubs += d > kHubDeg ? 1 : 0;
    info[v] = make_int2(a, d);
  }
  atomicMax(maxdeg, local_max);
  if (local_hubs) atomicAdd(hubs, local_hubs);
}

__global__ void k_check_targets(const int32_t* colidx, int64_t m, int32_t n, int* flags) {
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t t = colidx[e];
    bad |= (t < 0) | (t >= n);
  }
  if (bad) atomicOr(flags, kErrGraphTarget);
}

hipError_t launch_graph_check(const GraphDev& g, int* d_flags, int* d_maxdeg, int* d_hubs,
                              int2* info, hipStream_t s) {
  const int blocks_n = (int)std::min<int64_t>((g.n + 255) / 256, 16384);
  k_check_rows<<<blocks_n, 256, 0, s>>>(g.rowptr, g.n, g.m, d_flags, d_maxdeg, d_hubs, info);
  if (g.m > 0) {
    const int blocks_m = (int)std::min<int64_t>((g.m + 255) / 256, 16384);
    k_check_targets<<<blocks_m, 256, 0, s>>>(g.colidx, g.m, g.n, d_flags);
  }
  return hipGetLastError();
}

__global__ void k_philox(int64_t count, const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = philox4x32_10(ctr[i], k0, k1);
}

hipError_t launch_philox(int64_t count, const uint32_t* d_ctr, uint32_t k0, uint32_t k1,
                         uint32_t* d_out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((count + 255) / 256, 16384);
  k_philox<<<blocks, 256, 0, s>>>(count, (const uint4*)d_ctr, k0, k1, (uint4*)d_out);
  return hipGetLastError();
}

}  // namespace fora

namespace fora {

// ---- reverse (in-edge) CSR, built once at ingest for pull-mode push rounds
constexpr int kScanTile = 2048;

__global__ void k_indeg(const int32_t* __restrict__ colidx, int64_t m, int32_t* indeg) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&indeg[colidx[e]], 1);
}

__global__ __launch_bounds__(256) void k_tile_sum(const int32_t* __restrict__ x, int64_t n,
                                                  uint32_t* tsum) {
  __shared__ uint32_t s_tmp[4];
  uint32_t acc = 0;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += 256)
    if (base + k < n) acc += (uint32_t)x[base + k];
  const uint32_t t = block_sum(acc, s_tmp);
  if (threadIdx.x == 0) tsum[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_tile_scan(uint32_t* tsum, int64_t ntiles) {
  __shared__ uint32_t s_tmp[16];
  uint32_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t c = i < ntiles ? tsum[i] : 0u;
    uint32_t tot;
    const uint32_t p = block_exclusive_scan(c, s_tmp, tot);
    if (i < ntiles) tsum[i] = carry + p;
    carry += tot;
  }
}

// out[i] = sum of x[0..i); each thread scans 8 consecutive values
__global__ __launch_bounds__(256) void k_tile_apply(const int32_t* __restrict__ x, int64_t n,
                                                    const uint32_t* tsum, int32_t* out,
                                                    int32_t* out2) {
  __shared__ uint32_t s_tmp[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  uint32_t v[8], loc = 0;
  for (int k = 0; k < 8; ++k) {
    v[k] = base + k < n ? (uint32_t)x[base + k] : 0u;
    loc += v[k];
  }
  uint32_t tot;
  uint32_t run = tsum[blockIdx.x] + block_exclusive_scan(loc, s_tmp, tot);
  for (int k = 0; k < 8; ++k) {
    if (base + k < n) {
      out[base + k] = (int32_t)run;
      out2[base + k] = (int32_t)run;
    }
    if (base + k == n - 1) out[n] = (int32_t)(run + v[k]);
    run += v[k];
  }
}

__global__ void k_fill_rev(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                           const int32_t* __restrict__ rank, int32_t n, int32_t* cursor,
                           int32_t* in_colidx) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int32_t pos = atomicAdd(&cursor[colidx[e]], 1);
      in_colidx[pos] = rank[v];  // in-neighbours are stored by degree rank
    }
}

__global__ void k_list_inhubs(const int32_t* __restrict__ in_rowptr, int32_t n, int32_t* list,
                              int32_t* count, int32_t cap) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    if (in_rowptr[v + 1] - in_rowptr[v] > kHubDeg) {
      const int32_t pos = atomicAdd(count, 1);
      if (pos < cap) list[pos] = (int32_t)v;
    }
}

// Builds in_rowptr[n+1] and in_colidx[m] (caller-allocated) using the
// scratch arrays cursor[n] and tsum[ceil(n / 2048)].
hipError_t launch_build_reverse(const GraphDev& g, int32_t* in_rowptr, int32_t* in_colidx,
                                int32_t* cursor, uint32_t* tsum, hipStream_t s) {
  const int64_t n = g.n, m = g.m;
  hipError_t e = launch_fill_zero(cursor, sizeof(int32_t) * (size_t)n, s);
  if (e != hipSuccess) return e;
  const int bm = (int)std::min<int64_t>((m + 255) / 256, 16384);
  const int bn = (int)std::min<int64_t>((n + 255) / 256, 16384);
  if (m > 0) k_indeg<<<bm, 256, 0, s>>>(g.colidx, m, cursor);
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  k_tile_sum<<<(unsigned)tiles, 256, 0, s>>>(cursor, n, tsum);
  k_tile_scan<<<1, 1024, 0, s>>>(tsum, tiles);
  // in_rowptr and the fill cursor both start as the exclusive prefix
  k_tile_apply<<<(unsigned)tiles, 256, 0, s>>>(cursor, n, tsum, in_rowptr, cursor);
  if (m > 0) k_fill_rev<<<bn, 256, 0, s>>>(g.rowptr, g.colidx, g.rank, g.n, cursor, in_colidx);
  return hipGetLastError();
}

// FORA+ index plan: omega_max(v) = ceil(d(v) walks_per_degree) (FP64),
// exclusive prefix in 64 bits (tile sums, one-block scan, apply).
__global__ __launch_bounds__(256) void k_index_count(const int2* __restrict__ info, int32_t n,
                                                     double wpd, u64* om, u64* plan_gi,
                                                     u64* tsum) {
  __shared__ u64 s_tmp[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  u64 acc = 0;
  for (int k = threadIdx.x; k < kScanTile; k += 256) {
    const int64_t v = base + k;
    if (v < n) {
      const u64 c = (u64)ceil((double)info[v].y * wpd);
      om[v] = c;
      plan_gi[v] = (u64)v;
      acc += c;
    }
  }
  const u64 t = block_sum(acc, s_tmp);
  if (threadIdx.x == 0) tsum[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_tile_scan64(u64* tsum, int64_t ntiles) {
  __shared__ u64 s_tmp[16];
  u64 carry = 0;
  for (int64_t base = 0; base < ntiles; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const u64 c = i < ntiles ? tsum[i] : 0ull;
    u64 tot;
    const u64 p = block_exclusive_scan(c, s_tmp, tot);
    if (i < ntiles) tsum[i] = carry + p;
    carry += tot;
  }
}

// in place: off[v] holds omega_max(v) on entry and its exclusive prefix on
// exit; off[n] = the total
__global__ __launch_bounds__(256) void k_tile_apply64(u64* off, int64_t n, const u64* tsum) {
  __shared__ u64 s_tmp[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  u64 v[8], loc = 0;
  for (int k = 0; k < 8; ++k) {
    v[k] = base + k < n ? off[base + k] : 0ull;
    loc += v[k];
  }
  u64 tot;
  u64 run = tsum[blockIdx.x] + block_exclusive_scan(loc, s_tmp, tot);
  for (int k = 0; k < 8; ++k) {
    if (base + k < n) off[base + k] = run;
    if (base + k == n - 1) off[n] = run + v[k];
    run += v[k];
  }
}

hipError_t launch_index_plan(const GraphDev& g, double walks_per_degree, u64* off, u64* plan_gi,
                             u64* scratch, hipStream_t s) {
  const int64_t n = g.n;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  k_index_count<<<(unsigned)tiles, 256, 0, s>>>(g.info, g.n, walks_per_degree, off, plan_gi,
                                                scratch);
  k_tile_scan64<<<1, 1024, 0, s>>>(scratch, tiles);
  k_tile_apply64<<<(unsigned)tiles, 256, 0, s>>>(off, n, scratch);
  return hipGetLastError();
}

// Degree rank: rank[v] = position of v when nodes are ordered by out-degree
// descending, ties by id ascending. An LSD radix sort of the keys
// (max_deg - d(v)) with the ids as values, 8-bit digits, as many passes as
// max_deg has bytes; every pass is stable, so equal degrees keep id order.
// A pass: per-tile digit histograms (digit-major, so one exclusive scan over
// them gives each (digit, tile) its output start), then a scatter in which
// each wave ranks its lanes among equal digits with eight ballots and the
// waves of a block take their places in lane, wave and round order.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;  // elements per block

__global__ void k_deg_keys(const int2* __restrict__ info, int32_t n, int32_t max_deg,
                           uint32_t* key, int32_t* id) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    key[v] = (uint32_t)(max_deg - info[v].y);
    id[v] = (int32_t)v;
  }
}

// element i of tile t sits at t * kSortTile + round * kSortThreads + thread
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const uint32_t* __restrict__ key,
                                                            int64_t n, int shift, int64_t tiles,
                                                            uint32_t* hist) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&s_h[(key[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * tiles + blockIdx.x] = s_h[threadIdx.x];
}

// Exclusive scan of `count` entries in place, one block.
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t* a, int64_t count) {
  __shared__ uint32_t s_tmp[1024 / 64];
  uint32_t carry = 0;
  for (int64_t base = 0; base < count; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < count ? a[i] : 0u;
    uint32_t tot;
    const uint32_t pre = block_exclusive_scan(v, s_tmp, tot);
    if (i < count) a[i] = carry + pre;
    carry += tot;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t* __restrict__ key_in, const int32_t* __restrict__ val_in, int64_t n, int shift,
    int64_t tiles, const uint32_t* __restrict__ start, uint32_t* key_out, int32_t* val_out) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_wcnt[kSortThreads / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  s_base[threadIdx.x] = start[(size_t)threadIdx.x * tiles + blockIdx.x];
  for (int w = 0; w < kSortThreads / 64; ++w) s_wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    const bool valid = i < n;
    const uint32_t k = valid ? key_in[i] : 0u;
    const int32_t v = valid ? val_in[i] : 0;
    const uint32_t d = (k >> shift) & 0xFFu;
    // lanes of this wave holding the same digit
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long m = __ballot(bit);
      same &= bit ? m : ~m;
    }
    const uint32_t before = (uint32_t)__popcll(same & below);
    if (valid && before == 0) s_wcnt[wave][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pos = s_base[d] + before;
      for (int w = 0; w < wave; ++w) pos += s_wcnt[w][d];
      key_out[pos] = k;
      val_out[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortThreads / 64; ++w) {
      add += s_wcnt[w][threadIdx.x];
      s_wcnt[w][threadIdx.x] = 0;
    }
    s_base[threadIdx.x] += add;
    __syncthreads();
  }
}

__global__ void k_rank_from_order(const int32_t* __restrict__ order, int32_t n, int32_t* rank) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    rank[order[i]] = (int32_t)i;
}

hipError_t degree_rank_scratch_bytes(int32_t n, size_t* bytes) {
  const int64_t tiles = ((int64_t)n + kSortTile - 1) / kSortTile;
  *bytes = 4 * sizeof(int32_t) * (size_t)n + 256 + 256 * sizeof(uint32_t) * (size_t)tiles;
  return hipSuccess;
}

hipError_t launch_degree_rank(const GraphDev& g, int32_t* rank, void* scratch,
                              size_t scratch_bytes, hipStream_t s) {
  const int64_t n = g.n;
  const int64_t tiles = (n + kSortTile - 1) / kSortTile;
  size_t need = 0;
  (void)degree_rank_scratch_bytes(g.n, &need);
  if (scratch_bytes < need) return hipErrorInvalidValue;
  uint32_t* key[2] = {(uint32_t*)scratch, (uint32_t*)scratch + n};
  int32_t* val[2] = {(int32_t*)scratch + 2 * n, (int32_t*)scratch + 3 * n};
  const size_t used = 4 * sizeof(int32_t) * (size_t)n;
  uint32_t* hist = (uint32_t*)((char*)scratch + ((used + 255) / 256) * 256);
  const int bn = (int)std::min<int64_t>((n + 255) / 256, 16384);
  k_deg_keys<<<bn, 256, 0, s>>>(g.info, g.n, g.max_deg, key[0], val[0]);
  int passes = 1;
  while (passes < 4 && ((uint32_t)g.max_deg >> (8 * passes)) != 0) ++passes;
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    k_sort_hist<<<(unsigned)tiles, kSortThreads, 0, s>>>(key[cur], n, 8 * p, tiles, hist);
    k_scan_u32<<<1, 1024, 0, s>>>(hist, 256 * tiles);
    k_sort_scatter<<<(unsigned)tiles, kSortThreads, 0, s>>>(key[cur], val[cur], n, 8 * p, tiles,
                                                            hist, key[cur ^ 1], val[cur ^ 1]);
    cur ^= 1;
  }
  k_rank_from_order<<<bn, 256, 0, s>>>(val[cur], g.n, rank);
  return hipGetLastError();
}

// Walk records (see GraphDev): record lengths in 8-byte units, their
// exclusive prefix (the record starts), then one wavefront per node fills a
// record: lane 0 the header, all lanes the neighbours' slots (record start,
// degree and, where the graph's sizes allow, id).
__global__ void k_rec_len(const int2* __restrict__ info, const int32_t* __restrict__ rank,
                          int32_t n, int32_t* len) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    len[rank[v]] = 1 + info[v].y;
}

// rec_q[v] = start[rank[v]] (start holds the record starts in rank order)
__global__ void k_rec_start(const int32_t* __restrict__ rank, int32_t n,
                            const uint32_t* __restrict__ start, uint32_t* rec_q) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    rec_q[v] = start[rank[v]];
  if (blockIdx.x == 0 && threadIdx.x == 0) rec_q[n] = start[n];
}

__global__ void k_fill_rec(const int2* __restrict__ info, const int32_t* __restrict__ colidx,
                           int32_t n, const uint32_t* __restrict__ rec_q, u64* rec,
                           int qbits, int dbits, int ids) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); v < n;
       v += waves) {
    const int2 inf = info[v];
    u64* r = rec + rec_q[v];
    if (lane == 0) r[0] = (u64)(uint32_t)inf.y | ((u64)(uint32_t)v << 32);
    const u64 dmask = (1ull << dbits) - 1;  // all ones: the degree is in the header
    for (int i = lane; i < inf.y; i += 64) {
      const int32_t u = colidx[(int64_t)inf.x + i];
      const u64 d = (u64)(uint32_t)info[u].y;
      u64 slot = (u64)rec_q[u] | ((d < dmask ? d : dmask) << qbits);
      if (ids) slot |= (u64)(uint32_t)u << (qbits + dbits);
      r[1 + i] = slot;
    }
  }
}

// tmp: 2n + 1 int32 of scratch.
hipError_t launch_build_records(const GraphDev& g, uint32_t* rec_q, u64* rec, int32_t* tmp,
                                uint32_t* tsum, hipStream_t s) {
  const int64_t n = g.n;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  const int bn = (int)std::min<int64_t>((n + 255) / 256, 16384);
  int32_t* len = tmp;            // record lengths in rank order
  int32_t* start = tmp + n;      // their exclusive prefix, n + 1 entries
  k_rec_len<<<bn, 256, 0, s>>>(g.info, g.rank, g.n, len);
  k_tile_sum<<<(unsigned)tiles, 256, 0, s>>>(len, n, tsum);
  k_tile_scan<<<1, 1024, 0, s>>>(tsum, tiles);
  k_tile_apply<<<(unsigned)tiles, 256, 0, s>>>(len, n, tsum, start, len);
  k_rec_start<<<bn, 256, 0, s>>>(g.rank, g.n, (const uint32_t*)start, rec_q);
  const int wb = (int)std::min<int64_t>((n + 3) / 4, 65536);
  k_fill_rec<<<wb, 256, 0, s>>>(g.info, g.colidx, g.n, rec_q, rec, g.slot_qbits, g.slot_dbits,
                                g.slot_ids);
  return hipGetLastError();
}

hipError_t launch_list_inhubs(const int32_t* in_rowptr, int32_t n, int32_t* list, int32_t* count,
                              int32_t cap, hipStream_t s) {
  const int bn = (int)std::min<int64_t>((n + 255) / 256, 16384);
  k_list_inhubs<<<bn, 256, 0, s>>>(in_rowptr, n, list, count, cap);
  return hipGetLastError();
}

}  // namespace fora
