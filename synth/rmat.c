/* Multithreaded R-MAT sampler and CSR builder (input generation only; holds
 * none of the PPR method's arithmetic).
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM'04): each of `samples` edges picks
 * one of four quadrants per level of the 2^scale x 2^scale adjacency matrix
 * with probabilities (a, b, c, 1-a-b-c). Self-loops and duplicates are
 * dropped, node ids are relabelled by a seeded random permutation, and every
 * node left without an out-edge gets one uniformly random non-self target.
 * Rows of the CSR are sorted by target.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA'14) evaluated at
 * counters, so every sample can be drawn by any thread in any order and the
 * graph does not depend on the thread count. Sample i, level l uses the
 * 32-bit half (l & 1) of word splitmix64(K + (16 i + l / 2) * GAMMA) with
 * K = splitmix64(seed).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ull

/* samples drawn before their table lookups, so the lookups overlap */
enum { kBlock = 512 };

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* the SplitMix64 output for state x (state already advanced by GAMMA) */
static inline uint64_t splitmix64_at(uint64_t x) { return mix64(x + GAMMA); }

typedef struct {
  uint64_t key;
  int scale;
  uint32_t t_a, t_ab, t_abc;
} Sampler;

static inline void sample_edge(const Sampler *S, uint64_t i, uint32_t *s, uint32_t *t) {
  uint32_t src = 0, dst = 0;
  uint64_t word = 0;
  for (int l = 0; l < S->scale; ++l) {
    if ((l & 1) == 0) word = splitmix64_at(S->key + (16 * i + (uint64_t)(l >> 1)) * GAMMA);
    const uint32_t u = (l & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
    const int sh = S->scale - 1 - l;
    const uint32_t down = u >= S->t_ab;                              /* quadrants c, d */
    const uint32_t right = (u >= S->t_a) ^ down ^ (u >= S->t_abc);   /* quadrants b, d */
    src |= down << sh;
    dst |= right << sh;
  }
  *s = src;
  *t = dst;
}

static int cmp_i32(const void *x, const void *y) {
  const int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

static void sort_row(int32_t *p, int64_t len) {
  if (len < 32) {
    for (int64_t i = 1; i < len; ++i) {
      const int32_t v = p[i];
      int64_t j = i - 1;
      while (j >= 0 && p[j] > v) {
        p[j + 1] = p[j];
        --j;
      }
      p[j + 1] = v;
    }
  } else {
    qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

/* Fills rowptr[n+1] (int32), deg0[n] (out-degree before the fix-up) and
 * colidx (capacity `cap` >= samples + n entries), and the edge count *m_out.
 * Returns 0, or -1 on allocation failure, -2 if m >= 2^31, -3 if cap is too
 * small, -4 for a scale outside [1, 30] or samples outside [0, 2^32). */
int synth_rmat(int scale, int64_t samples, double a, double b, double c, uint64_t seed,
               int32_t *rowptr, int32_t *deg0, int32_t *col, int64_t cap, int64_t *m_out) {
  const int64_t n = (int64_t)1 << scale;
  if (scale < 1 || scale > 30 || samples < 0 || samples >= ((int64_t)1 << 32)) return -4;
  Sampler S;
  S.key = mix64(seed + GAMMA);
  S.scale = scale;
  const double two32 = 4294967296.0;
  double ta = a * two32, tab = (a + b) * two32, tabc = (a + b + c) * two32;
  S.t_a = (uint32_t)(ta < two32 - 1 ? ta + 0.5 : two32 - 1);
  S.t_ab = (uint32_t)(tab < two32 - 1 ? tab + 0.5 : two32 - 1);
  S.t_abc = (uint32_t)(tabc < two32 - 1 ? tabc + 0.5 : two32 - 1);

  /* the relabelling permutation: Fisher-Yates on its own SplitMix64 stream */
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!perm || !off) {
    free(perm);
    free(off);
    return -1;
  }
  for (int64_t v = 0; v < n; ++v) perm[v] = (int32_t)v;
  uint64_t ps = mix64(seed ^ 0xD1B54A32D192ED03ull);
  for (int64_t v = n - 1; v > 0; --v) {
    ps += GAMMA;
    const uint64_t r = mix64(ps);
    const int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(v + 1)) >> 64);
    const int32_t tmp = perm[v];
    perm[v] = perm[j];
    perm[j] = tmp;
  }

  /* The samples are cut into P fixed parts; each part counts its edges per
   * source in a row of its own (no shared counters between threads), and in
   * the second pass scatters into its own slice of each source's row. The
   * graph depends neither on P nor on the thread count: rows are sorted
   * afterwards. */
  const int64_t P = omp_get_max_threads() > 0 ? omp_get_max_threads() : 1;
  uint32_t *cnt = (uint32_t *)calloc((size_t)(P * n), sizeof(uint32_t));
  if (!cnt) {
    free(perm);
    free(off);
    return -1;
  }
#pragma omp parallel for schedule(static, 1)
  for (int64_t p = 0; p < P; ++p) {
    uint32_t *row = cnt + p * n;
    const int64_t lo = samples * p / P, hi = samples * (p + 1) / P;
    uint32_t bs[kBlock], bt[kBlock];
    for (int64_t i0 = lo; i0 < hi; i0 += kBlock) {
      const int nb = (int)(hi - i0 < kBlock ? hi - i0 : kBlock);
      for (int k = 0; k < nb; ++k) sample_edge(&S, (uint64_t)(i0 + k), &bs[k], &bt[k]);
      for (int k = 0; k < nb; ++k)
        if (bs[k] != bt[k]) ++row[perm[bs[k]]];
    }
  }
  /* row lengths, their prefix sums, then each part's start inside each row */
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    int64_t d = 0;
    for (int64_t p = 0; p < P; ++p) d += cnt[p * n + v];
    off[v + 1] = d;
  }
  for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
  const int64_t total = off[n];
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    int64_t c = off[v];
    for (int64_t p = 0; p < P; ++p) {
      const uint32_t k = cnt[p * n + v];
      cnt[p * n + v] = (uint32_t)c;
      c += k;
    }
  }
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  if (!tmp) {
    free(perm);
    free(off);
    free(cnt);
    return -1;
  }
  /* pass 2: scatter relabelled targets into their rows */
#pragma omp parallel for schedule(static, 1)
  for (int64_t p = 0; p < P; ++p) {
    uint32_t *cur = cnt + p * n;
    const int64_t lo = samples * p / P, hi = samples * (p + 1) / P;
    uint32_t bs[kBlock], bt[kBlock];
    for (int64_t i0 = lo; i0 < hi; i0 += kBlock) {
      const int nb = (int)(hi - i0 < kBlock ? hi - i0 : kBlock);
      for (int k = 0; k < nb; ++k) sample_edge(&S, (uint64_t)(i0 + k), &bs[k], &bt[k]);
      for (int k = 0; k < nb; ++k) {
        if (bs[k] == bt[k]) continue;
        bs[k] = (uint32_t)perm[bs[k]];
        bt[k] = (uint32_t)perm[bt[k]];
      }
      for (int k = 0; k < nb; ++k)
        if (bs[k] != bt[k]) tmp[cur[bs[k]]++] = (int32_t)bt[k];
    }
  }
  free(cnt);

  /* sort and deduplicate each row; a row left empty gets one random target */
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!deg) {
    free(perm);
    free(off);
    free(tmp);
    return -1;
  }
  const uint64_t fix_key = mix64(seed ^ 0x8CB92BA72F3D8DD7ull);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int32_t *p = tmp + off[v];
    const int64_t len = off[v + 1] - off[v];
    sort_row(p, len);
    int64_t u = 0;
    for (int64_t k = 0; k < len; ++k)
      if (u == 0 || p[k] != p[u - 1]) p[u++] = p[k];
    deg0[v] = (int32_t)u;
    deg[v] = u > 0 ? u : 1;
  }
  deg[n] = 0;
  int64_t m = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = deg[v];
    deg[v] = m;
    m += d;
  }
  deg[n] = m;
  if (m >= ((int64_t)1 << 31) || m > cap) {
    free(perm);
    free(off);
    free(tmp);
    free(deg);
    return m > cap ? -3 : -2;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    const int64_t o = deg[v];
    rowptr[v] = (int32_t)o;
    if (deg0[v] > 0) {
      memcpy(col + o, tmp + off[v], sizeof(int32_t) * (size_t)deg0[v]);
    } else {
      const uint64_t r = splitmix64_at(fix_key + (uint64_t)v * GAMMA);
      int64_t t = (int64_t)(((unsigned __int128)r * (uint64_t)(n - 1)) >> 64);
      t += t >= v;
      col[o] = (int32_t)t;
    }
  }
  rowptr[n] = (int32_t)m;
  free(perm);
  free(off);
  free(tmp);
  free(deg);
  *m_out = m;
  return 0;
}
