/*
 * fora.h -- C ABI of the MI355X (gfx950) implementation of FORA approximate
 * single-source Personalized PageRank (Wang et al., TODS 2019):
 * synchronous forward push to r_max, then Philox-keyed random walks from
 * every node with residue, then top-k over reserve + walk estimate.
 *
 * Conventions
 *  - Every call returns an int status (FORA_OK or a negative FORA_E_* code);
 *    fora_last_error() gives a message for the calling thread's last failure.
 *  - "d_" pointers are device (HBM) pointers, "h_" pointers host pointers.
 *  - Device memory for inputs, outputs and the per-call workspace is owned by
 *    the caller; the query calls allocate no device memory of their own (a
 *    captured HIP graph holds what the runtime gives it). The graph handle
 *    owns derived tables of about 28 n + 12 m bytes, allocated by
 *    fora_build_csr (a per-node table, the reverse graph for pull rounds, a
 *    degree ranking and the walk records) and released by fora_free_graph;
 *    fora_set_tuning may rebuild the walk records and fora_build_index
 *    allocates the index.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    The push phase checks the frontier size from the host between groups of
 *    rounds, and every query call reads its device error flags at the end, so
 *    query calls return after their work has completed.
 *  - A workspace may be used by one call at a time; calls that share a
 *    workspace must be ordered (same stream or explicit synchronisation).
 *
 * Notation (paper, notation table): n nodes, m edges, d(v) out-degree,
 * alpha stop probability, eps relative error, delta threshold, p_f failure
 * probability, r residue, q ("pi-circle") reserve, r_max residue threshold.
 */
#ifndef FORA_H_
#define FORA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FORA_OK = 0,
  FORA_E_ARG = -1,      /* an argument is out of its documented range      */
  FORA_E_GRAPH = -2,    /* the CSR graph is malformed or has a dangling node */
  FORA_E_NOMEM = -3,    /* workspace too small, or an allocation failed    */
  FORA_E_HIP = -4,      /* a HIP runtime call failed                       */
  FORA_E_OVERFLOW = -5  /* a count exceeds the widths documented below     */
};

/* Opaque handle to a validated graph. It BORROWS the caller's CSR arrays:
 * keep them alive and unchanged until fora_free_graph. */
typedef struct fora_graph fora_graph;

/* Per-query counters. Filled when a stats pointer is given. */
typedef struct fora_stats {
  int32_t rounds;          /* synchronous push rounds with a non-empty frontier */
  int32_t term_violations; /* residues above r_max*d(v) after the push (0)     */
  int64_t pushes;          /* frontier entries pushed, over all rounds         */
  int64_t edge_ops;        /* residue increments applied (sum of d over pushes)*/
  int64_t plan_entries;    /* nodes with r(v) > 0 (walk plan length)           */
  uint64_t walks;          /* W = sum over v of omega_v                        */
  uint64_t steps;          /* walk moves (edge traversals) over all walks      */
  double r_sum;            /* sum of residues after the push (the exact sum of
                              the fixed-point residues, rounded to FP64)       */
  double rmax;             /* r_max used                                       */
  double omega_unit;       /* (2 eps/3 + 2) ln(2/p_f) / (eps^2 delta)          */
  uint32_t t_alpha;        /* floor(alpha * 2^32)                              */
  float ms_push;           /* phase times from HIP events on the call's stream */
  float ms_plan;           /* (for a batch: the whole batch's phase, repeated  */
  float ms_walk;           /*  in every entry); ms_walk spans exactly the walk */
  float ms_topk;           /*  kernel launch                                   */
  uint32_t pull_rounds;    /* push rounds that ran as a pull over in-edges     */
  uint32_t balance_stopped; /* FORA_BALANCE: the rule held at the last round
                               boundary (it ended the push, or the push ended
                               there by itself)                                 */
} fora_stats;

/* One query of a batch. */
typedef struct fora_query {
  int32_t src;   /* source node, 0 <= src < n                                */
  int32_t k;     /* 1 <= k <= min(n, FORA_MAX_K)                             */
  double alpha;  /* 0 < alpha < 1                                            */
  double eps;    /* 0 < eps < 1                                              */
  double delta;  /* 0 < delta <= 1                                           */
  double pf;     /* 0 < pf < 1                                               */
  double rmax;   /* > 0: use this r_max; <= 0: eqn:rmax (section 3.2)        */
  uint64_t seed; /* low 32 bits form the second Philox key word              */
  uint32_t flags;    /* 0 (Algorithm 2) or an OR of the FORA_* flags below  */
  uint32_t reserved; /* 0                                                     */
  double walk_cost;  /* FORA_BALANCE: cost of one walk in residue increments */
} fora_query;

/* Algorithm 3 (section 4), per query:
 * FORA_PRUNE_ZERO_HOP (section 4.1): pi_hat starts at q + alpha r; from each
 *   v with residue, omega_v = ceil(r'(v) omega_unit) walks with
 *   r' = (1 - alpha) r (FP64 from the fixed-point residue), each starting with a
 *   forced move (the step-0 Philox block only picks the out-neighbour) and
 *   adding r'(v) / omega_v at its end point.
 * FORA_BALANCE (section 4.2): before each push round the push stops once its
 *   residue increments so far reach the estimated walk cost
 *   (1 - alpha * pushed mass) (1 - alpha) omega_unit walk_cost; r_max still
 *   bounds the push from below. */
#define FORA_PRUNE_ZERO_HOP 1u
#define FORA_BALANCE 2u
/* FORA+ (section 3.3): walk j of v comes from the graph's walk-destination
 * index when j < omega_max(v) (fora_build_index); walks are then keyed by
 * the index key instead of (source, seed), and later ones run live with that
 * key, so results equal running all walks with the index key. Needs an
 * index built for the query's alpha; not combined with
 * FORA_PRUNE_ZERO_HOP. */
#define FORA_USE_INDEX 4u
/* Also count the walks that end at each node, into the workspace view
 * walk_count. A diagnostic: the estimate does not use the counts. Without
 * the flag those rows stay zero and a walk's end costs one memory-side
 * atomic instead of two. */
#define FORA_WALK_COUNTS 8u

#define FORA_MAX_K 4096
#define FORA_MAX_BATCH 4096

/* Dense per-query arrays inside a workspace, for inspection. Query b's row
 * starts at b*n. Valid after a call on that workspace has completed; the
 * three walk-phase rows (walk_count, walk_weight_fx, pi_hat) share memory
 * with the push's frontier arrays, so after fora_push_only or
 * fora_push_sweep they hold no meaning (fora_walk_only leaves pi_hat so). */
typedef struct fora_views {
  uint64_t *residue_fx;       /* r(s, v), unsigned fixed point with 62
                                 fraction bits [batch][n]                     */
  float *reserve;             /* q(s, v), FP32 [batch][n]                     */
  uint64_t *walk_count;       /* walks ending at v, [batch][n]; zero unless
                                 the query set FORA_WALK_COUNTS            */
  uint64_t *walk_weight_fx;   /* sum of walk weights ending at v, unsigned
                                 fixed point with 62 fraction bits [batch][n] */
  float *pi_hat;              /* q + walk weight, FP32 [batch][n]             */
} fora_views;

/* Launch shape of the library's kernels for one graph handle. The defaults
 * suit MI355X; fora_set_tuning replaces them (for example with values an
 * autotuner measured). Not part of the method: results do not depend on it,
 * except that graph_rounds > 0 makes fora_ssppr_batch replay a captured HIP
 * graph (see there). */
typedef struct fora_tuning {
  int32_t walk_blocks_per_cu; /* persistent walk grid = CUs x this (1..32)       */
  int32_t walk_chunk;         /* walk ids per work-queue grab (64..65536, x64)   */
  int32_t push_blocks_per_cu; /* push grid = CUs x this (1..32)                  */
  int32_t graph_rounds;       /* 0: host-driven push loop; > 0: capture this
                                 many push rounds plus plan, walks and top-k in
                                 one HIP graph per (batch, kmax, buffers)        */
  int32_t pull_ratio;         /* a query's push round runs as a pull over the
                                 reverse graph when its frontier edges times
                                 this exceed n + m (0: never pull)               */
  int32_t walk_agg;           /* 1: waves sum walk end points in LDS before
                                 adding them to HBM (same results)               */
  int32_t record_ids;         /* 1 (default): a walk-record slot also holds the
                                 neighbour's id where record start, a degree
                                 field of 12 bits or more, and id fit 64 bits,
                                 so no header is read where a walk stops
                                 (degrees too wide for the field are read from
                                 the header of the node reached); 0: (start,
                                 degree) slots only; 2: ids with a 4-bit
                                 degree field (exercises the header reads).
                                 Changing it rebuilds the records (waits for
                                 the device; same results). FORA_E_NOMEM then
                                 leaves the graph as it was; FORA_E_HIP leaves
                                 it unusable (free it)                           */
} fora_tuning;

const char *fora_last_error(void);

/* Graph ingest (section 2.1: a directed graph stored as out-adjacency lists).
 * d_rowptr: int32[n+1], d_colidx: int32[m], device. Checks on the device that
 * rowptr[0] = 0, rowptr[n] = m, rowptr is non-decreasing, every target is in
 * [0, n), and every node has out-degree >= 1 (a walk must be able to move and
 * Algorithm 1 divides by |N_out(v)|). Requires 1 <= n and m < 2^31.
 * Errors: FORA_E_ARG (sizes), FORA_E_GRAPH (content), FORA_E_HIP, FORA_E_NOMEM.
 * Waits for the check to finish. */
int fora_build_csr(int32_t n, int64_t m, const int32_t *d_rowptr,
                   const int32_t *d_colidx, void *stream, fora_graph **out);
int fora_free_graph(fora_graph *g);
int fora_graph_info(const fora_graph *g, int32_t *n, int64_t *m,
                    int32_t *max_degree);
/* Read or replace the launch shape (FORA_E_ARG if a field is out of range).
 * Replacing it drops the handle's captured graphs. Not thread-safe against
 * concurrent query calls on the same handle. */
int fora_get_tuning(const fora_graph *g, fora_tuning *out);
int fora_set_tuning(fora_graph *g, const fora_tuning *t);

/* Bytes of workspace for `batch` concurrent queries (1..FORA_MAX_BATCH):
 * about 52 bytes per node and query (residue 8, reserve 4, and 40 that the
 * push's frontier arrays and the walk phase's plan and sums take in turn). */
int fora_workspace_size(const fora_graph *g, int32_t batch, size_t *bytes);
int fora_workspace_views(const fora_graph *g, int32_t batch, void *d_ws,
                         fora_views *views);

/* Whole-graph FORA (Algorithm 2) for one source, then top-k (section 5,
 * selection over the whole-graph estimate).
 *  push: synchronous Forward Push (Algorithm 1, every node over its
 *    threshold in one round) down to r_max (eqn:rmax unless opt_rmax > 0);
 *  walks: omega_v = ceil(r(v) * omega_unit) walks from each v with
 *    r(v) > 0, each ending at t adding r(v)/omega_v to pi_hat(t);
 *  top-k: ids sorted by (pi_hat descending, id ascending).
 * Output d_topk_ids int32[k], d_topk_vals float[k] (FP32 pi_hat). If fewer
 * than k nodes have pi_hat > 0 the rest are the lowest unused ids, value 0.
 * h_stats (nullable) makes the call wait and fill the counters. The query
 * flags are 0 here (no per-node walk counts); fora_ssppr_batch with a batch
 * of one takes flags.
 * Errors: FORA_E_ARG for any parameter outside the ranges of fora_query,
 * FORA_E_NOMEM if ws_bytes < fora_workspace_size(g, 1),
 * FORA_E_OVERFLOW if some omega_v >= 2^32 (the walk index j within a node
 * is a 32-bit Philox counter word), FORA_E_HIP. */
int fora_ssppr(const fora_graph *g, int32_t src, double alpha, double eps,
               double delta, double pf, int32_t k, double opt_rmax,
               uint64_t seed, void *d_ws, size_t ws_bytes,
               int32_t *d_topk_ids, float *d_topk_vals, fora_stats *h_stats,
               void *stream);

/* fora_ssppr for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc). The
 * workspace is a static device array of FORA_STATIC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends; the call
 * makes no hipMalloc or hipFree, captures no HIP graph (graph_rounds is
 * ignored) and records no events (the ms_* fields of the stats are 0). The
 * caller passes only the outputs. Every call on a device shares that
 * device's array, which keeps the last call's contents (each call clears
 * what must start at zero): calls that overlap on one device race, so order
 * them (one stream, or synchronise). The array's device address is looked
 * up on the first call on each device. Results equal fora_ssppr's bit for
 * bit. FORA_E_NOMEM if the graph needs more workspace than the array holds
 * (fora_workspace_size(g, 1) > FORA_STATIC_SCRATCH_BYTES: graphs up to
 * about 2.5 million nodes fit); other errors as fora_ssppr. */
#define FORA_STATIC_SCRATCH_BYTES (128u << 20)
int fora_ssppr_static(const fora_graph *g, int32_t src, double alpha, double eps, double delta,
                      double pf, int32_t k, double opt_rmax, uint64_t seed, int32_t *d_topk_ids,
                      float *d_topk_vals, fora_stats *h_stats, void *stream);

/* The same for `batch` queries in one launch sequence: all queries' push
 * rounds, walk plans, walks and selections run in shared kernels. Query b's
 * result is written to d_ids[b*kmax ...], d_vals[b*kmax ...]; kmax must be at
 * least every query's k. Each query's result equals what fora_ssppr returns
 * for it, bit for bit: residues are summed in fixed point, walks are keyed by
 * (source, seed, start node, walk index, step), and end-point weights are
 * summed as integers, so no result depends on the batch or on the order in
 * which the device runs the work. h_stats
 * (nullable) is an array of `batch` entries.
 * With tuning.graph_rounds = R > 0 the whole sequence (zero fill, init, R
 * push rounds, plan, walks, top-k) is captured once per (batch, kmax,
 * workspace, outputs) into a HIP graph and replayed as one launch; if some
 * query still has a frontier after R rounds, the plan, walks and top-k of
 * the replay are skipped and the call finishes them with host-driven rounds.
 * In graph mode the ms_* fields of the stats are 0. */
int fora_ssppr_batch(const fora_graph *g, int32_t batch,
                     const fora_query *h_queries, int32_t kmax, void *d_ws,
                     size_t ws_bytes, int32_t *d_ids, float *d_vals,
                     fora_stats *h_stats, void *stream);

/* FORA for source distributions (section 6.2, the extension to source
 * distributions; global PageRank, section 6.3, is sigma = (1/n, ..., 1/n)): query b's push
 * starts from r = sigma_b instead of e_s, which keeps the invariant
 * pi(sigma, t) = q(t) + sum_v r(v) pi(v, t), so walks, estimate and top-k are
 * those of fora_ssppr_batch and the eps guarantee holds for pi(sigma, .).
 * d_sigma: double[batch][n], device, caller-owned, read once; each row a
 * probability distribution (entries rounded to the fixed-point residues;
 * FORA_BALANCE assumes a row sums to 1). The queries' src fields are not
 * used; walks are keyed by (0xFFFFFFFF, seed) (the index key with
 * FORA_USE_INDEX). Same workspace, outputs and flags as fora_ssppr_batch;
 * never replayed from a captured graph (graph_rounds is ignored). Errors:
 * those of fora_ssppr_batch; FORA_E_ARG for a null d_sigma or an entry
 * outside [0, 1] or not a number (reported when the call completes). */
int fora_dist_batch(const fora_graph *g, int32_t batch, const fora_query *h_queries,
                    const double *d_sigma, int32_t kmax, void *d_ws, size_t ws_bytes,
                    int32_t *d_ids, float *d_vals, fora_stats *h_stats, void *stream);

/* ---- FORA+ walk-destination index (section 3.3) ---------------------------
 * Builds (or replaces) the graph's index: for every node v,
 * omega_max(v) = ceil(d(v) walks_per_degree) walks (eqn:index-rwnum with
 * walks_per_degree = r_max omega_unit) keyed by (key0, key1) and walk index,
 * stopping with probability alpha; their end points are stored in (v, j)
 * order. Allocates the index (8 (n + 1) + 4 sum omega_max bytes) and waits.
 * Replacing an index drops the handle's captured graphs; not thread-safe
 * against concurrent query calls on the same handle.
 * FORA_E_OVERFLOW if some omega_max(v) >= 2^32 (checked first: the old
 * index stays). Any later failure (FORA_E_NOMEM, FORA_E_HIP) leaves the
 * handle with no index. */
int fora_build_index(fora_graph *g, double alpha, double walks_per_degree, uint32_t key0,
                     uint32_t key1, void *stream);
/* The index's parameters and total end points (0 if none). */
int fora_index_info(const fora_graph *g, int64_t *total, double *alpha,
                    double *walks_per_degree, uint32_t *key0, uint32_t *key1);
/* Copies the index: d_off uint64[n + 1] and d_dest int32[total] (device). */
int fora_index_export(const fora_graph *g, uint64_t *d_off, int32_t *d_dest, void *stream);

/* ---- top-k FORA (Algorithm 5, section 5.2) ------------------------------
 * For each query, with its own k: run Algorithm 2 with eps' = eps / 2,
 * p_f' = p_f / (n max(log2(n / k), 1)) and delta = 1/k, 1/(2k), ... (while
 * above 1/n, then 1/n), r_max by eqn:rmax for those parameters unless the
 * query's rmax is set, and Philox seed (seed + iteration); stop at the first
 * iteration whose k-th largest estimate (FP32) is at least (1 + eps) delta,
 * or at delta = 1/n. The query's delta field is ignored; flags apply to every
 * iteration. Queries that stop leave the batch; the rest run the next
 * iteration together.
 * Workspace: fora_topk_workspace_size(g, batch, kmax) bytes (the batched
 * workspace plus staging rows). Outputs as fora_ssppr_batch; h_stats
 * (nullable) holds each query's last iteration; h_iterations (int32[batch],
 * nullable) the iterations run; h_delta (double[batch], nullable) the final
 * delta. Waits for completion. */
int fora_topk_workspace_size(const fora_graph *g, int32_t batch, int32_t kmax, size_t *bytes);
int fora_topk_batch(const fora_graph *g, int32_t batch, const fora_query *h_queries,
                    int32_t kmax, void *d_ws, size_t ws_bytes, int32_t *d_ids, float *d_vals,
                    fora_stats *h_stats, int32_t *h_iterations, double *h_delta, void *stream);

/* ---- step-level entry points (used to compare each phase on its own) ---- */

/* Only the push phase of fora_ssppr for one source (Algorithm 1,
 * synchronous rounds), or, with d_sigma (nullable, double[n], device) given,
 * of fora_dist_batch for that source distribution (src is then not used).
 * Results in the workspace views (row 0).
 * h_round_sizes (nullable, max_rounds entries) receives |F_t|; d_frontiers
 * (nullable, device int32, frontier_cap entries) receives the frontiers of
 * all rounds back to back, each round's set in ascending id order.
 * Waits for completion. FORA_E_OVERFLOW if max_rounds or frontier_cap is too
 * small. */
int fora_push_only(const fora_graph *g, int32_t src, double alpha, double rmax,
                   const double *d_sigma, void *d_ws, size_t ws_bytes, int32_t max_rounds,
                   int32_t *h_round_sizes, int32_t *d_frontiers,
                   int64_t frontier_cap, fora_stats *h_stats, void *stream);

/* Only the walk phase for a caller-given plan (Algorithm 2's walk loop):
 * entries (d_v[e], d_omega[e], d_w[e]) with d_v strictly increasing,
 * 1 <= d_omega[e] < 2^32, d_w[e] > 0 (FP64). Walks use Philox key
 * (key0, key1) and stop threshold floor(alpha * 2^32). Endpoint counts go to
 * the workspace view walk_count (row 0), weights to walk_weight_fx as
 * round(d_w[e] * 2^62) per walk. h_steps (nullable) receives the move count
 * and makes the call wait. At most n entries. The plan is checked on the
 * device before any walk runs: FORA_E_ARG if d_v is not strictly increasing
 * in [0, n), FORA_E_OVERFLOW for an omega outside [1, 2^32). */
int fora_walk_only(const fora_graph *g, int64_t entries, const int32_t *d_v,
                   const uint64_t *d_omega, const double *d_w, uint32_t key0,
                   uint32_t key1, double alpha, void *d_ws, size_t ws_bytes,
                   uint64_t *h_steps, void *stream);

/* The graph's degree rank (copied to d_rank, int32[n], device): rank[v] is
 * v's position when nodes are ordered by out-degree descending, ties by id
 * ascending. It orders the walk records and the pull increments. Waits. */
int fora_graph_rank(const fora_graph *g, int32_t *d_rank, void *stream);

/* Philox4x32-10 (Salmon et al., SC'11) blocks on the device: d_out[4i..4i+3]
 * = Philox(d_ctr[4i..4i+3], (key0, key1)). */
int fora_philox(int64_t count, const uint32_t *d_ctr, uint32_t key0,
                uint32_t key1, uint32_t *d_out, void *stream);

/* ---- learned r_max --------------------------------------------------------
 * A small MLP predicts y = ln(r_max / r_max*) per source from 7 features; the
 * eps guarantee (Lemma 2) holds for any r_max, so the model only moves cost
 * between the push and the walks. Parameter vector of FORA_MLP_PARAMS floats:
 * mu[7], sigma[7] (feature standardisation, not trained), W1[64][7], b1[64],
 * W2[64][64], b2[64], W3[64], b3; y = W3.gelu(W2 gelu(W1 x' + b1) + b2) + b3
 * with x' = (x - mu) / sigma and gelu(z) = z Phi(z). */
#define FORA_MLP_FEATURES 7
#define FORA_MLP_PARAMS 4751
#define FORA_MLP_ACTS 128 /* floats saved per sample by the FP32 forward pass */
/* floats of scratch for fora_mlp_backward with `count` samples */
#define FORA_MLP_SCRATCH(count) ((size_t)(count) * 129 + ((size_t)(count) + 255) / 256)

/* Features per source, float[count][7]: ln d(s); ln of the summed out-degree
 * of s's out-neighbours; the residue mass on nodes over their threshold after
 * the first synchronous push round at r_max* (0 if s is not pushed); ln n;
 * ln m; alpha; eps. d_srcs int32[count], device; an id outside [0, n) gets
 * NaN features (checked on the device), so fora_predict_rmax falls back to
 * r_max* for it. */
int fora_features(const fora_graph *g, int32_t count, const int32_t *d_srcs, double alpha,
                  double eps, double delta, double pf, float *d_features, void *stream);
/* FP32 forward; d_acts (nullable, float[count][FORA_MLP_ACTS]) keeps what the
 * backward pass needs. */
int fora_mlp_forward(int32_t count, const float *d_x, const float *d_params, float *d_y,
                     float *d_acts, void *stream);
/* Gradient of L = mean_i (y_i - t_i)^2 with respect to the trained part of
 * the parameters (d_grad, FORA_MLP_PARAMS floats; the mu/sigma entries are
 * left untouched) and L itself (d_loss, 1 float). Needs the d_acts and d_y of
 * a forward pass on the same d_x and FORA_MLP_SCRATCH(count) floats of
 * scratch. Deterministic: sums run in sample order. */
int fora_mlp_backward(int32_t count, const float *d_x, const float *d_params,
                      const float *d_acts, const float *d_y, const float *d_target,
                      float *d_grad, float *d_loss, float *d_scratch, void *stream);
/* One Adam step (bias-corrected, step >= 1) on the trained parameters. */
int fora_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, float lr,
                   float beta1, float beta2, float eps, int32_t step, void *stream);
/* Parameters rounded to BF16 (nearest even), and the BF16 forward pass
 * (weights, standardised inputs and hidden activations in BF16, sums FP32). */
int fora_mlp_to_bf16(const float *d_params, uint16_t *d_params_bf16, void *stream);
int fora_mlp_forward_bf16(int32_t count, const float *d_x, const uint16_t *d_params_bf16,
                          float *d_y, void *stream);
/* Features, BF16 forward and r_max = r_max* exp(y) for each source, where
 * r_max* is eqn:rmax for (eps, delta, pf); sources whose y is not finite or
 * lies outside [log_lo, log_hi] get r_max* (h_fallbacks, nullable, counts
 * them and makes the call wait). d_scratch: FORA_PREDICT_SCRATCH(count)
 * floats (features, outputs and a counter). d_rmax: double[count]. */
#define FORA_PREDICT_SCRATCH(count) ((size_t)(count) * 8 + 1)
int fora_predict_rmax(const fora_graph *g, int32_t count, const int32_t *d_srcs, double alpha,
                      double eps, double delta, double pf, const uint16_t *d_params_bf16,
                      double log_lo, double log_hi, float *d_scratch, double *d_rmax,
                      int32_t *h_fallbacks, void *stream);
/* Push cost at several thresholds in one pass per source: pushes to
 * r_0 = mult[0] r_max*, then lowers the threshold to mult[1] r_max* and keeps
 * pushing from the current state, and so on (mult strictly decreasing).
 * After each threshold i it records the cumulative residue increments
 * (h_edge_ops[b * nthr + i]) and the walks Algorithm 2 would then run,
 * W = sum_v ceil(r(v) omega_unit) (h_walks[b * nthr + i]). The query's rmax
 * field is ignored. Waits for completion. */
int fora_push_sweep(const fora_graph *g, int32_t batch, const fora_query *h_queries,
                    int32_t nthr, const double *h_mult, void *d_ws, size_t ws_bytes,
                    int64_t *h_edge_ops, uint64_t *h_walks, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FORA_H_ */
