// Internal declarations of the FORA HIP library (gfx950).
//
// Data layout in HBM (per call, carved from the caller's workspace):
//   ctrl      one Ctrl block: frontier counters, walk work queue, error flags
//   qstats    QueryStats[batch]: per-query counters (device side)
//   queries   QueryDev[batch]: per-query constants computed on the host
//   r         uint64[batch][n]  residue, unsigned fixed point (62 fraction bits)
//   q         float[batch][n]   reserve (FP32)
//   then one region that the push and the walk phase take in turn:
//   push:  incd      dense increments for pull rounds, [groups][n][G]
//          fr0/fr1   uint64[batch*n]   frontier entries (query << 32 | node)
//          frx       uint64[batch*n]   per-entry increment (1-alpha) x / d (fixed point)
//   walks: acc       uint64[batch][n]  walk weights, fixed point (62 fraction bits)
//          cnt       uint64[batch][n]  walk end-point counts
//          plan_*    walk plan: entry (query << 32 | node), walk offset, weight
//          pi        float[batch][n]   q + acc, the estimate (over plan_gi, after the walks)
//   tiles     per-tile counts and offsets for the plan scan
//   topk      histograms, selection state and candidates
// Graph: rowptr/colidx borrowed from the caller, plus owned tables: info[v]
// = {rowptr[v], d(v)}, the degree rank, the reverse CSR, and the walk records
// (a walk step reads one 8-byte slot of the current node's record).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "fora.h"

namespace fora {

typedef unsigned long long u64;

constexpr int kMaxRoundsLogged = 4096;
constexpr int kPlanTile = 2048;        // nodes per plan tile (256 threads x 8)
constexpr int kTopkTile = 4096;        // nodes per top-k block
constexpr int kHistBins = 2048;        // 11-bit radix digits
constexpr int kWalkChunk = 512;        // walk ids per work-queue grab
constexpr int kStatSlots = 64;         // per-query counters are spread over slots
constexpr int kHubDeg = 2048;          // frontier entries above this are split into pieces
constexpr int kHubPiece = 2048;        // edges per piece of a split entry
constexpr int kPullRatio = 16;         // default: pull a round if frontier edges * this > n + m
constexpr double kFx = 4611686018427387904.0;  // 2^62
constexpr unsigned long long kFxOne = 1ull << 62;  // 1.0 in the fixed point of residues

// Residues are unsigned fixed point with 62 fraction bits. Increments are
// rounded once, when they are formed (one FP64 value per pushed node), and
// then summed as integers, so every sum is exact and independent of the order
// in which the atomics land: a query pushes the same nodes in the same rounds
// whatever else runs beside it, and one run equals the next bit for bit.
__device__ __forceinline__ double fx_to_double(unsigned long long x) {
  return (double)x * (1.0 / kFx);
}
__device__ __forceinline__ unsigned long long fx_from_double(double x) {
  return __double2ull_rn(x * kFx);
}
// The push test r(v) > r_max d(v), with r_max d(v) the FP64 product: for an
// integer residue r_fx it holds iff r_fx > floor(r_max d(v) 2^62).
__device__ __forceinline__ unsigned long long fx_threshold(double rmax, int d) {
  const double t = (rmax * (double)d) * kFx;
  return t < 18446744073709551616.0 ? (unsigned long long)t : ~0ull;
}

// Error flags raised by kernels.
enum : int {
  kErrFrontierOverflow = 1,
  kErrOmegaOverflow = 2,
  kErrLogOverflow = 4,
  kErrGraphRowptr = 8,
  kErrGraphTarget = 16,
  kErrGraphDangling = 32,
  kErrTopk = 64,
  kErrBadPlan = 128,
  kErrBadDist = 256,  // a source distribution entry is negative or not finite
};

struct QueryDev {
  int32_t src;
  int32_t k;
  uint32_t key0, key1;  // Philox key: (source, seed)
  uint32_t t_alpha;     // stop iff first Philox word < t_alpha
  uint32_t flags;       // FORA_PRUNE_ZERO_HOP | FORA_BALANCE
  double alpha;
  double rmax;
  double omega_unit;
  double walk_cost;     // FORA_BALANCE: one walk's cost in residue increments
};

// Per-query counters, each query's spread over kStatSlots slots so that
// concurrent blocks add to different addresses; the host sums the slots.
struct StatSlot {
  u64 pushes;
  u64 edge_ops;
  u64 entries;
  u64 walks;
  u64 steps;
  u64 r_sum_fx;          // sum of the fixed-point residues after the push
  int32_t rounds;
  int32_t term_violations;
  u64 pull_rounds;
  u64 mass_fx;           // residue pushed (sum of x, fixed point), FORA_BALANCE only
  u64 balance_stopped;   // set in slot 0 by the round-boundary test
};
typedef StatSlot QueryStatsDev;

struct Ctrl {
  u64 fr_cnt[2];       // frontier sizes, double-buffered by round parity
  u64 entries;         // plan entries (all queries)
  u64 walks;           // W (all queries)
  u64 chunk_next;      // walk work queue cursor (in chunks)
  u64 log_len;         // frontier log length (push-only path)
  u64 hub_ctr[2];      // split frontier entries: (count << 40) | pieces, by round parity
  int32_t error;
  int32_t skip;        // set by the graph's gate when the push needs more rounds
  int32_t npull;       // entries of the pull list (query groups) this round
  int32_t pad2;
  u64 round_size[kMaxRoundsLogged];
};

struct GraphDev {
  int32_t n;
  int64_t m;
  const int32_t* rowptr;
  const int32_t* colidx;
  const int2* info;
  int32_t max_deg;
  int32_t n_hubs;  // nodes with out-degree above kHubDeg
  // reverse (in-edge) CSR for pull rounds
  const int32_t* in_rowptr;
  const int32_t* in_colidx;
  int32_t n_inhubs;           // nodes with in-degree above kHubDeg, ascending
  const int32_t* inhub_node;
  const u64* inhub_base;      // first piece of each, exclusive prefix
  u64 inhub_pieces;           // total pieces
  // walk records: node v's record starts at 8-byte unit rec_q[v]; unit 0
  // is the header d(v) | v << 32, then one unit per out-neighbour u in CSR
  // order holding rec_q[u] in bits [0, slot_qbits) and d(u) in the next
  // slot_dbits bits (all ones if d(u) does not fit: then it is read from u's
  // header), so a move reads the next node's record start and degree in one
  // load. With slot_ids, u itself sits in the bits above them and no header
  // is read where a walk stops; otherwise the fields are 32 bits each and a
  // walk reads its end node's id from the header.
  const u64* rec;
  const uint32_t* rec_q;
  int32_t slot_qbits;
  int32_t slot_dbits;
  int32_t slot_ids;
  // rank of each node by out-degree, descending (ties by id): the slot of v
  // in the dense pull-increment rows, and the order of the walk records, so
  // that the values read most often (those of high-degree nodes) share lines
  const int32_t* rank;
  // FORA+ walk-destination index (null if none): offsets (n + 1) and end points
  const u64* idx_off;
  const int32_t* idx_dest;
};

// Queries per unit of the dense pull increments (1, 4 or 16): one pull
// load serves that many queries; small batches take small units so that a
// single query does not read and clear sixteen queries' worth.
__host__ __device__ inline int pull_group_for(int batch) {
  return batch >= 16 ? 16 : (batch >= 4 ? 4 : 1);
}

struct Layout {
  size_t ctrl, qstats, queries, r, q, cnt, acc, pi;
  size_t fr0, fr1, frx, hub_idx, hub_base, incd, ecnt, mode, pull_list, stop;
  size_t plan_gi, plan_off, plan_wfx;
  size_t tile_cnt, tile_walks, tile_eoff, tile_woff;
  size_t hist, sel, cand_key, cand_id, cand_cnt, blk_ties;
  size_t zero_begin, zero_end;
  size_t total;
  int64_t cap;      // frontier / plan capacity (batch * n)
  int64_t hub_cap;  // split-entry capacity per round (batch * n_hubs)
  int64_t tiles_per_row, plan_tiles, topk_blocks;
};

struct Ws {
  Ctrl* ctrl;
  QueryStatsDev* qstats;
  QueryDev* queries;
  u64* r;  // fixed point, kFxOne = 1
  float* q;
  u64* cnt;
  u64* acc;
  float* pi;
  u64* fr[2];
  u64* frx;       // per-entry increment, fixed point
  u64* hub_idx;   // frontier index of each split entry
  u64* hub_base;  // first piece number of each split entry
  u64* incd;      // [ceil(batch / G)][n][G]: frontier increments by degree rank, G =
                  // pull_group_for(batch) queries per node unit, dense, for pull rounds
  u64* ecnt;      // [2][batch][kStatSlots]: frontier edges per query, by round parity
  int32_t* mode;  // [batch]: 1 if the query's current round pulls
  int32_t* pull_list;  // groups of queries with one in pull mode this round:
                       // group << 16 | mask of the pulling members
  int32_t* stop;       // [batch]: 0, or 1 + the first round the balance rule skips
  u64* plan_gi;
  u64* plan_off;
  u64* plan_wfx;
  uint32_t* tile_cnt;
  u64* tile_walks;
  u64* tile_eoff;
  u64* tile_woff;
  uint32_t* hist;      // [batch][kHistBins]
  uint32_t* sel;       // [batch][4]: prefix, remaining k, count above, pass
  uint32_t* cand_key;  // [batch][FORA_MAX_K]
  int32_t* cand_id;    // [batch][FORA_MAX_K]
  uint32_t* cand_cnt;  // [batch]
  uint32_t* blk_ties;  // [batch][topk_blocks]
};

Layout make_layout(const GraphDev& g, int32_t batch);
Ws carve(const Layout& L, void* base);

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two
// 32x32->64 multiplies; key schedule bumps by the Weyl constants.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// floor(U * d / 2^64) for U = (hi << 32) | lo and d < 2^32: the part of the
// 96-bit product above bit 64, from two 32x32->64 products.
__device__ __forceinline__ uint32_t mul_shift_index(uint32_t hi, uint32_t lo, uint32_t d) {
  const uint64_t a = (uint64_t)hi * d;
  const uint64_t b = (uint64_t)lo * d;
  return (uint32_t)((a + (b >> 32)) >> 32);
}

// ---- launchers (each enqueues on `s`; return hipError_t) -------------------
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_graph_check(const GraphDev& g, int* d_flags, int* d_maxdeg, int* d_hubs,
                              int2* info, hipStream_t s);
hipError_t launch_init_queries(const GraphDev& g, const Ws& w, int batch, hipStream_t s);
// r = sigma (double[batch][n], rounded to the fixed point), then the round-0 frontier
hipError_t launch_init_dist(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                            const double* sigma, hipStream_t s);
constexpr uint32_t kDistKey0 = 0xFFFFFFFFu;  // first walk key word of a source distribution
hipError_t launch_push_round(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                             int t, int blocks, int pull_ratio, int32_t* frontier_log,
                             int64_t log_cap, hipStream_t s);
hipError_t launch_clear_walk_sums(const Ws& w, const Layout& L, hipStream_t s);
hipError_t launch_plan(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                       hipStream_t s);
hipError_t launch_walks(const GraphDev& g, const Ws& w, int blocks, int chunk, bool agg,
                        hipStream_t s);
hipError_t launch_push_gate(const Ws& w, int rounds, hipStream_t s);
hipError_t launch_walk_plan_from_host(const GraphDev& g, const Ws& w, int64_t entries,
                                      const int32_t* d_v, const uint64_t* d_omega,
                                      const double* d_w, hipStream_t s);
hipError_t launch_topk(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                       int kmax, int32_t* d_ids, float* d_vals, hipStream_t s);
hipError_t launch_build_reverse(const GraphDev& g, int32_t* in_rowptr, int32_t* in_colidx,
                                int32_t* cursor, uint32_t* tsum, hipStream_t s);
hipError_t launch_index_walks(const GraphDev& g, const u64* plan_gi, const u64* off, Ctrl* ctrl,
                              const QueryDev* Q, QueryStatsDev* QS, int32_t* dest, int blocks,
                              int chunk, hipStream_t s);
// omega_max(v) = ceil(d(v) walks_per_degree) and its exclusive prefix into
// off[n + 1]; plan_gi[v] = v. scratch: ceil(n / 2048) u64.
hipError_t launch_index_plan(const GraphDev& g, double walks_per_degree, u64* off, u64* plan_gi,
                             u64* scratch, hipStream_t s);
hipError_t launch_topk_kth(const float* vals, int kmax, const int32_t* ks, int count, float* kth,
                           hipStream_t s);
hipError_t launch_copy_rows(const int32_t* src_ids, const float* src_vals, int kmax,
                            const int32_t* from, const int32_t* to, int count, int32_t* dst_ids,
                            float* dst_vals, hipStream_t s);
hipError_t launch_build_records(const GraphDev& g, uint32_t* rec_q, u64* rec, int32_t* tmp,
                                uint32_t* tsum, hipStream_t s);
// rank[v] from the out-degrees; scratch: 4 int32 arrays of n and sort storage
hipError_t degree_rank_scratch_bytes(int32_t n, size_t* bytes);
hipError_t launch_degree_rank(const GraphDev& g, int32_t* rank, void* scratch,
                              size_t scratch_bytes, hipStream_t s);
hipError_t launch_list_inhubs(const int32_t* in_rowptr, int32_t n, int32_t* list, int32_t* count,
                              int32_t cap, hipStream_t s);
hipError_t launch_seed_frontier(const GraphDev& g, const Ws& w, const Layout& L, int batch, int t,
                                hipStream_t s);
hipError_t launch_count_walks(const GraphDev& g, const Ws& w, const Layout& L, int batch,
                              u64* walks, hipStream_t s);
hipError_t launch_features(const GraphDev& g, int count, const int32_t* srcs, double alpha,
                           double eps, double rmax, float* out, hipStream_t s);
hipError_t launch_mlp_forward(int count, const float* x, const float* params, float* y,
                              float* acts, hipStream_t s);
hipError_t launch_mlp_backward(int count, const float* x, const float* params, const float* acts,
                               const float* y, const float* target, float* grad, float* loss,
                               float* scratch, hipStream_t s);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, hipStream_t s);
hipError_t launch_to_bf16(int count, const float* in, uint16_t* out, hipStream_t s);
hipError_t launch_mlp_forward_bf16(int count, const float* x, const uint16_t* pb, float* y,
                                   hipStream_t s);
hipError_t launch_rmax_from_output(int count, const float* y, double rmax_star, double lo,
                                   double hi, double* out, int* fallbacks, hipStream_t s);
hipError_t launch_philox(int64_t count, const uint32_t* d_ctr, uint32_t k0, uint32_t k1,
                         uint32_t* d_out, hipStream_t s);

int device_cu_count();

}  // namespace fora
