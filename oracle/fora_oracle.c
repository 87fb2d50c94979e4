/*
 * fora_oracle.c -- plain, slow, single-threaded FP64 reference of FORA
 * (Wang et al., "Efficient Algorithms for Approximate Single-Source
 * Personalized PageRank Queries", TODS 2019), whole-graph variant without
 * index or optimizations (Algorithm 1 + Algorithm 2, r_max by eqn:rmax).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Readings taken where the paper leaves a choice (each is listed, with its
 * reason, in the design notes of the repository):
 *   - logarithms are natural (Lemma 2's last step needs exp(-ln(2/p_f))).
 *   - Forward Push (Algorithm 1) picks "some v" over the threshold; here every
 *     such v is pushed at once in synchronous rounds: the residues of the
 *     round's frontier are read and cleared first, then their increments are
 *     applied. Any push order keeps the invariant of eqn:layerppr.
 *   - the push test is strict, r(v) > r_max * d(v), evaluated in FP64.
 *   - Algorithm 2's omega_i = ceil(r_i * omega / r_sum) with
 *     omega = r_sum * omega_unit is evaluated as ceil(r_i * omega_unit);
 *     the per-walk increment a_i * r_sum / omega equals r_i / omega_i.
 *   - random choices come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11): one block per
 *     walk step, key = (source, seed), counter = (start node, walk index,
 *     step, 0). Word 0 decides termination (stop iff y0 < floor(alpha*2^32));
 *     words 1, 2 form a 64-bit U and the out-neighbour index is
 *     floor(U * d / 2^64) (Lemire's multiply-shift, computed with 128-bit
 *     integers here).
 *
 * Parity pins: see the tests. The Philox block function is pinned word for
 * word against rocRAND's independent implementation of Philox4x32-10 (run
 * on the host), besides the statistics of the walk distributions it drives.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 as published in SC'11: four 32-bit words, ten rounds, two  */
/* multiply-hi/lo S-boxes per round and a Weyl-sequence key schedule.        */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_MUL_A = 0xD2511F53u;
static const uint32_t PHILOX_MUL_B = 0xCD9E8D57u;
static const uint32_t PHILOX_WEYL_0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_WEYL_1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                          uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t prodA = (uint64_t)PHILOX_MUL_A * (uint64_t)x0;
    uint64_t prodB = (uint64_t)PHILOX_MUL_B * (uint64_t)x2;
    uint32_t hiA = (uint32_t)(prodA >> 32), loA = (uint32_t)prodA;
    uint32_t hiB = (uint32_t)(prodB >> 32), loB = (uint32_t)prodB;
    uint32_t y0 = hiB ^ x1 ^ k0;
    uint32_t y1 = loB;
    uint32_t y2 = hiA ^ x3 ^ k1;
    uint32_t y3 = loA;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_WEYL_0;
    k1 += PHILOX_WEYL_1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void oracle_philox_many(int64_t count, const uint32_t *ctrs /* count x 4 */,
                        const uint32_t key[2], uint32_t *outs /* count x 4 */) {
  for (int64_t i = 0; i < count; ++i)
    oracle_philox4x32_10(ctrs + 4 * i, key, outs + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Graph check (problem definition, section 2.1): CSR well formed, targets   */
/* in range, and every node has an out-neighbour (a walk must be able to     */
/* move, and Algorithm 1 divides by |N_out(v)|).                             */
/* Returns 0 if valid, -1 malformed CSR, -2 target out of range, -3 a node   */
/* with out-degree 0.                                                        */
/* ------------------------------------------------------------------------ */
int oracle_validate(int32_t n, int64_t m, const int32_t *rowptr,
                    const int32_t *colidx) {
  if (n <= 0 || m < 0 || rowptr[0] != 0 || (int64_t)rowptr[n] != m) return -1;
  for (int32_t v = 0; v < n; ++v) {
    if (rowptr[v + 1] < rowptr[v]) return -1;
    if (rowptr[v + 1] == rowptr[v]) return -3;
  }
  for (int64_t e = 0; e < m; ++e)
    if (colidx[e] < 0 || colidx[e] >= n) return -2;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Parameters (section 3.1 Algorithm 2, section 3.2 eqn:rmax and its two     */
/* cases). out = {c, L, omega_unit, r_max, T_alpha}:                         */
/*   c = 2 eps / 3 + 2, L = ln(2 / p_f), omega_unit = c L / (eps^2 delta),   */
/*   r_max = eps / sqrt(m) * sqrt(delta / (c L)); if m r_max > 1 then        */
/*   r_max = eps^2 delta / (c L); a positive override replaces r_max.       */
/*   T_alpha = floor(alpha * 2^32), the walk-stop threshold on a 32-bit word. */
/* ------------------------------------------------------------------------ */
void oracle_constants(int64_t m, double alpha, double eps, double delta,
                      double pf, double rmax_override, double out[5]) {
  double c = 2.0 * eps / 3.0 + 2.0;
  double L = log(2.0 / pf);
  double omega_unit = (c * L) / ((eps * eps) * delta);
  double rmax = eps / sqrt((double)m) * sqrt(delta / (c * L));
  if ((double)m * rmax > 1.0) rmax = (eps * eps) * delta / (c * L);
  if (rmax_override > 0.0) rmax = rmax_override;
  out[0] = c;
  out[1] = L;
  out[2] = omega_unit;
  out[3] = rmax;
  out[4] = floor(alpha * 4294967296.0);
}

/* One synchronous round over the frontier front[0 .. nf-1] (ascending):    */
/* every listed residue is read and cleared before any increment lands,      */
/* then the increments are applied node by node in CSR order. x is scratch   */
/* of nf doubles. Returns the residue mass pushed (sum of x).                */
static double push_round(const int32_t *rowptr, const int32_t *colidx, double alpha,
                         const int32_t *front, int32_t nf, double *r, double *q,
                         double *x) {
  double pushed = 0.0;
  for (int32_t i = 0; i < nf; ++i) {
    int32_t v = front[i];
    x[i] = r[v];
    r[v] = 0.0;
    q[v] += alpha * x[i];
    pushed += x[i];
  }
  for (int32_t i = 0; i < nf; ++i) {
    int32_t v = front[i];
    int32_t d = rowptr[v + 1] - rowptr[v];
    double inc = ((1.0 - alpha) * x[i]) / (double)d;
    for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) r[colidx[e]] += inc;
  }
  return pushed;
}

/* ------------------------------------------------------------------------ */
/* Forward Push (Algorithm 1) in synchronous rounds.                         */
/* Round t: F = { v ascending : r(v) > r_max * d(v) }; stop when F is empty. */
/* For v in F: x_v = r(v); r(v) = 0; q(v) += alpha x_v. Then, for v in F     */
/* ascending and u in N_out(v) in CSR order: r(u) += (1 - alpha) x_v / d(v). */
/* Outputs r (residue) and q (reserve), FP64, length n.                      */
/* round_sizes[t] = |F_t|; if frontier_log is given the frontiers are        */
/* written back to back (capacity frontier_cap entries).                     */
/* Returns the number of rounds, or -1 if max_rounds was exceeded, -2 if the */
/* frontier log overflowed.                                                  */
/* ------------------------------------------------------------------------ */
/* The push loop from a given (r, q), so that Algorithm 1 can be continued  */
/* at a lower threshold from the state another threshold left.              */
/* With walk_cost >= 0 it also applies the balance rule of Algorithm 3      */
/* (section 4.2): before each round, with FC the edge operations done so    */
/* far and r_sum = 1 - alpha * (mass pushed so far), it stops once          */
/* FC >= r_sum (1 - alpha) omega_unit walk_cost, the estimated cost of the  */
/* walks in edge-operation units. *balance_margin (if given) receives the   */
/* smallest |FC - estimate| / estimate over the tests made; *stopped is 1   */
/* if the rule held at the last boundary tested (it ended the push, or the  */
/* push ended there by itself).                                             */
static int32_t push_core(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                         double alpha, double rmax, double *r, double *q,
                         int32_t max_rounds, int32_t *round_sizes,
                         int64_t *edge_ops, int32_t *frontier_log,
                         int64_t frontier_cap, double *min_margin,
                         double omega_unit, double walk_cost, double *balance_margin,
                         int32_t *stopped) {
  int32_t *front = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  if (!front || !x) { free(front); free(x); return -3; }
  int32_t rounds = 0;
  int64_t ops = 0, logged = 0;
  double margin = INFINITY, bmargin = INFINITY, pushed = 0.0;
  if (stopped) *stopped = 0;
  for (;;) {
    int32_t nf = 0;
    for (int32_t v = 0; v < n; ++v) {
      double thr = rmax * (double)(rowptr[v + 1] - rowptr[v]);
      if (r[v] > 0.0) {
        /* relative distance of a tested residue from its threshold */
        double rel = fabs(r[v] - thr) / thr;
        if (rel < margin) margin = rel;
      }
      if (r[v] > thr) front[nf++] = v;
    }
    if (walk_cost >= 0.0) {
      /* tested at every round boundary, the last one included */
      const double r_sum = 1.0 - alpha * pushed;
      const double est = r_sum * (1.0 - alpha) * omega_unit * walk_cost;
      if (est > 0.0) {
        const double rel = fabs((double)ops - est) / est;
        if (rel < bmargin) bmargin = rel;
      }
      if ((double)ops >= est) {
        if (stopped) *stopped = 1;
        break;
      }
    }
    if (nf == 0) break;
    if (rounds == max_rounds) { rounds = -1; break; }
    if (round_sizes) round_sizes[rounds] = nf;
    if (frontier_log) {
      if (logged + nf > frontier_cap) { rounds = -2; break; }
      memcpy(frontier_log + logged, front, sizeof(int32_t) * (size_t)nf);
      logged += nf;
    }
    pushed += push_round(rowptr, colidx, alpha, front, nf, r, q, x);
    for (int32_t i = 0; i < nf; ++i) ops += rowptr[front[i] + 1] - rowptr[front[i]];
    ++rounds;
  }
  if (edge_ops) *edge_ops = ops;
  if (min_margin) *min_margin = margin;
  if (balance_margin) *balance_margin = bmargin;
  free(front);
  free(x);
  return rounds;
}

int32_t oracle_push_continue(int32_t n, const int32_t *rowptr,
                             const int32_t *colidx, double alpha, double rmax,
                             double *r, double *q, int32_t max_rounds,
                             int32_t *round_sizes, int64_t *edge_ops,
                             int32_t *frontier_log, int64_t frontier_cap,
                             double *min_margin) {
  return push_core(n, rowptr, colidx, alpha, rmax, r, q, max_rounds, round_sizes,
                   edge_ops, frontier_log, frontier_cap, min_margin, 0.0, -1.0, NULL,
                   NULL);
}

/* Algorithm 3's push: Algorithm 1 from r = e_s with the balance rule. */
int32_t oracle_push_balanced(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                             int32_t s, double alpha, double rmax, double omega_unit,
                             double walk_cost, double *r, double *q, int32_t max_rounds,
                             int32_t *round_sizes, int64_t *edge_ops,
                             int32_t *frontier_log, int64_t frontier_cap,
                             double *min_margin, double *balance_margin,
                             int32_t *stopped) {
  for (int32_t v = 0; v < n; ++v) { r[v] = 0.0; q[v] = 0.0; }
  r[s] = 1.0;
  return push_core(n, rowptr, colidx, alpha, rmax, r, q, max_rounds, round_sizes,
                   edge_ops, frontier_log, frontier_cap, min_margin, omega_unit,
                   walk_cost, balance_margin, stopped);
}

/* Algorithm 1 from r = e_s, q = 0. */
int32_t oracle_push(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                    int32_t s, double alpha, double rmax, double *r, double *q,
                    int32_t max_rounds, int32_t *round_sizes,
                    int64_t *edge_ops, int32_t *frontier_log,
                    int64_t frontier_cap, double *min_margin) {
  for (int32_t v = 0; v < n; ++v) { r[v] = 0.0; q[v] = 0.0; }
  r[s] = 1.0;
  return oracle_push_continue(n, rowptr, colidx, alpha, rmax, r, q, max_rounds,
                              round_sizes, edge_ops, frontier_log,
                              frontier_cap, min_margin);
}

/* ------------------------------------------------------------------------ */
/* Frontier replay: Algorithm 1 from the caller's (r, q) with the frontier   */
/* of every synchronous round given rather than tested. Algorithm 1 may push */
/* nodes in any order and eqn:layerppr holds for every sequence of pushes,   */
/* so replaying another run's frontiers in FP64 rebuilds the state that run  */
/* should have reached. Each round is push_round, as in the oracle's own     */
/* push. Before each round it measures how far the listed nodes are from the */
/* push test r(v) > r_max d(v) and how far the unlisted ones are over it,    */
/* both relative to the threshold; after the last round, how far any node is */
/* over it. out[0] = max listed shortfall (r_max d(v) - r(v)) / (r_max d(v)) */
/* (negative when every listed node passes), out[1] = max unlisted excess    */
/* (r(v) - r_max d(v)) / (r_max d(v)) over every round and the final state   */
/* (at most 0 when no node was left over its threshold); both start at       */
/* -infinity. frontiers holds the rounds back to back, round_sizes[t]        */
/* entries each. Returns 0, -1 if a frontier is not strictly ascending in    */
/* [0, n), -3 if out of memory.                                              */
/* ------------------------------------------------------------------------ */
int32_t oracle_push_replay(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                           double alpha, double rmax, double *r, double *q,
                           int32_t rounds, const int64_t *round_sizes,
                           const int32_t *frontiers, double out[2]) {
  char *listed = (char *)calloc((size_t)n, 1);
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  if (!listed || !x) { free(listed); free(x); return -3; }
  double shortfall = -INFINITY, excess = -INFINITY;
  int64_t off = 0;
  int32_t rc = 0;
  for (int32_t t = 0; t < rounds && rc == 0; ++t) {
    const int32_t *F = frontiers + off;
    const int64_t nf = round_sizes[t];
    for (int64_t i = 0; i < nf; ++i) {
      if (F[i] < 0 || F[i] >= n || (i > 0 && F[i] <= F[i - 1])) { rc = -1; break; }
      listed[F[i]] = 1;
    }
    if (rc != 0) break;
    for (int32_t v = 0; v < n; ++v) {
      const int32_t deg = rowptr[v + 1] - rowptr[v];
      const double thr = rmax * (double)deg;
      double rel = listed[v] ? (thr - r[v]) / thr : (r[v] - thr) / thr;
      if (listed[v]) { if (rel > shortfall) shortfall = rel; }
      else if (rel > excess) excess = rel;
    }
    push_round(rowptr, colidx, alpha, F, (int32_t)nf, r, q, x);
    for (int64_t i = 0; i < nf; ++i) listed[F[i]] = 0;
    off += nf;
  }
  if (rc == 0) {
    for (int32_t v = 0; v < n; ++v) {
      const int32_t deg = rowptr[v + 1] - rowptr[v];
      const double thr = rmax * (double)deg;
      double rel = (r[v] - thr) / thr;
      if (rel > excess) excess = rel;
    }
  }
  out[0] = shortfall;
  out[1] = excess;
  free(listed);
  free(x);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Walk plan (Algorithm 2, the loop over v_i with r(s, v_i) > 0):            */
/* omega_v = ceil(r(v) * omega_unit), weight w_v = r(v) / omega_v, for v     */
/* ascending. Writes up to n entries; returns the entry count, or -1 if some */
/* omega_v does not fit in 32 bits.                                          */
/* ------------------------------------------------------------------------ */
int64_t oracle_plan(int32_t n, const double *r, double omega_unit,
                    int32_t *pv, uint64_t *pomega, double *pw) {
  int64_t e = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (r[v] > 0.0) {
      double om = ceil(r[v] * omega_unit);
      if (om >= 4294967296.0) return -1;
      pv[e] = v;
      pomega[e] = (uint64_t)om;
      pw[e] = r[v] / om;
      ++e;
    }
  }
  return e;
}

/* ------------------------------------------------------------------------ */
/* Random walks with restart (section 2.1): from x = v, at each step stop    */
/* with probability alpha, else move to a uniformly random out-neighbour.    */
/* For plan entry (v, omega_v, w_v) and j = 0 .. omega_v - 1, the walk's end */
/* point t gets cnt[t] += 1 and acc[t] += w_v (Algorithm 2, the increment    */
/* a_i r_sum / omega). steps counts moves. If endpoints is given it receives */
/* the end point of every walk in plan order.                                */
/* ------------------------------------------------------------------------ */
/* With first_move set (Algorithm 3, zero-hop walks pruned) the step-0     */
/* block only chooses the first out-neighbour (no stop test), so every walk */
/* starts at a random out-neighbour of v; later steps are as above.         */
void oracle_walks(int32_t n, const int32_t *rowptr, const int32_t *colidx,
                  uint32_t source, uint32_t seed, uint32_t t_alpha,
                  int64_t entries, const int32_t *pv, const uint64_t *pomega,
                  const double *pw, int32_t first_move, uint64_t *cnt, double *acc,
                  uint64_t *steps, int32_t *endpoints) {
  (void)n;
  const uint32_t key[2] = {source, seed};
  uint64_t total_steps = 0, w_index = 0;
  for (int64_t e = 0; e < entries; ++e) {
    int32_t v = pv[e];
    for (uint64_t j = 0; j < pomega[e]; ++j) {
      int32_t x = v;
      uint32_t b = 0;
      for (;;) {
        uint32_t ctr[4] = {(uint32_t)v, (uint32_t)j, b, 0u};
        uint32_t y[4];
        oracle_philox4x32_10(ctr, key, y);
        if (!(first_move && b == 0) && y[0] < t_alpha) break;
        uint64_t d = (uint64_t)(rowptr[x + 1] - rowptr[x]);
        uint64_t U = ((uint64_t)y[1] << 32) | (uint64_t)y[2];
        uint64_t idx = (uint64_t)(((unsigned __int128)U * d) >> 64);
        x = colidx[rowptr[x] + (int64_t)idx];
        ++b;
      }
      cnt[x] += 1;
      acc[x] += pw[e];
      total_steps += b;
      if (endpoints) endpoints[w_index] = x;
      ++w_index;
    }
  }
  *steps = total_steps;
}

/* ------------------------------------------------------------------------ */
/* Top-k (section 5, the straightforward selection over the whole-graph      */
/* estimate): order nodes by (pi_hat descending, id ascending), take k.      */
/* ------------------------------------------------------------------------ */
static const double *g_sort_keys;
static int cmp_desc_then_id(const void *a, const void *b) {
  int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
  double x = g_sort_keys[i], y = g_sort_keys[j];
  if (x > y) return -1;
  if (x < y) return 1;
  return (i > j) - (i < j);
}

int oracle_topk(int32_t n, const double *pi, int32_t k, int32_t *ids,
                double *vals) {
  if (k < 1 || k > n) return -1;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!order) return -3;
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  g_sort_keys = pi;
  qsort(order, (size_t)n, sizeof(int32_t), cmp_desc_then_id);
  for (int32_t i = 0; i < k; ++i) {
    ids[i] = order[i];
    vals[i] = pi[order[i]];
  }
  free(order);
  return 0;
}
