// Estimate and top-k (section 5, selection over the whole-graph estimate).
//
// pi_hat(t) = q(t) + acc(t) * 2^-62, formed in FP64 and stored as FP32.
// Non-negative FP32 values order like their bit patterns as unsigned
// integers, so the k-th largest key K is found by radix select: three passes
// of histograms over digits [31:21], [20:10], [9:0] of the keys that share
// the digits fixed so far. Keys above K are gathered directly; of the keys
// equal to K the lowest ids are taken, in id order. The k survivors are
// sorted by (pi_hat descending, id ascending) with a bitonic sort in LDS.
#include "internal.h"
#include "scan.h"

namespace fora {

constexpr int kTopkThreads = 256;
constexpr int kTopkPerThread = kTopkTile / kTopkThreads;  // 16

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int pass) {
  return pass == 0 ? (key >> 21) : pass == 1 ? ((key >> 10) & 0x7FFu) : (key & 0x3FFu);
}
__device__ __forceinline__ bool prefix_ok(uint32_t key, int pass, uint32_t prefix) {
  return pass == 0 ? true : pass == 1 ? ((key >> 21) == prefix) : ((key >> 10) == prefix);
}

__global__ __launch_bounds__(kTopkThreads) void k_topk_hist(
    int pass, const float* __restrict__ q, const u64* __restrict__ acc,
    const u64* __restrict__ r, const QueryDev* __restrict__ Q, float* __restrict__ pi,
    int n, uint32_t* hist, const uint32_t* sel, const Ctrl* ctrl) {
  __shared__ uint32_t s_hist[kHistBins];
  if (ctrl->skip) return;
  const int b = blockIdx.y;
  for (int i = threadIdx.x; i < kHistBins; i += kTopkThreads) s_hist[i] = 0;
  __syncthreads();
  const uint32_t prefix = pass ? sel[b * 4 + 0] : 0u;
  const size_t row = (size_t)b * n;
  const int v0 = blockIdx.x * kTopkTile;
  // FORA_PRUNE_ZERO_HOP: the zero-hop walks' share alpha r(v) is added exactly
  const double zero_hop = (Q[b].flags & FORA_PRUNE_ZERO_HOP) ? Q[b].alpha : 0.0;
  for (int k = threadIdx.x; k < kTopkTile; k += kTopkThreads) {
    const int v = v0 + k;
    if (v >= n) break;
    uint32_t key;
    if (pass == 0) {
      double p = (double)q[row + v] + (double)acc[row + v] * (1.0 / kFx);
      if (zero_hop != 0.0) p += zero_hop * fx_to_double(r[row + v]);
      const float pf = (float)p;
      pi[row + v] = pf;
      key = __float_as_uint(pf);
    } else {
      key = __float_as_uint(pi[row + v]);
    }
    if (prefix_ok(key, pass, prefix)) atomicAdd(&s_hist[digit_of(key, pass)], 1u);
  }
  __syncthreads();
  uint32_t* h = hist + (size_t)b * kHistBins;
  for (int i = threadIdx.x; i < kHistBins; i += kTopkThreads)
    if (s_hist[i]) atomicAdd(&h[i], s_hist[i]);
}

// One block per query: find the digit whose bin holds the k-th largest key
// among the keys matching the prefix; clears the histogram for the next pass.
// sel[b] = {prefix, k still needed, keys above the prefix group, -}.
__global__ __launch_bounds__(kTopkThreads) void k_topk_select(int pass, uint32_t* hist,
                                                              uint32_t* sel,
                                                              const QueryDev* Q,
                                                              uint32_t* cand_cnt,
                                                              const Ctrl* ctrl) {
  __shared__ uint32_t s_tmp[kTopkThreads / 64];
  __shared__ uint32_t s_found[2];
  if (ctrl->skip) return;
  const int b = blockIdx.x;
  if (pass == 0 && threadIdx.x == 0) cand_cnt[b] = 0;  // the collect pass appends from 0
  uint32_t* h = hist + (size_t)b * kHistBins;
  const int nb = pass == 2 ? 1024 : kHistBins;
  const int per = nb / kTopkThreads;  // 8 or 4 bins per thread
  uint32_t need = pass == 0 ? (uint32_t)Q[b].k : sel[b * 4 + 1];
  uint32_t above = pass == 0 ? 0u : sel[b * 4 + 2];
  const uint32_t prefix = pass == 0 ? 0u : sel[b * 4 + 0];
  // thread i owns bins in descending order: rank i covers bins
  // [nb - (i+1)*per, nb - i*per), scanned from the top
  if (threadIdx.x == 0) {
    s_found[0] = 0;
    s_found[1] = 0;
  }
  const int hi_bin = nb - threadIdx.x * per;
  uint32_t mine = 0;
  for (int k = 1; k <= per; ++k) mine += h[hi_bin - k];
  uint32_t tot;
  const uint32_t before = block_exclusive_scan(mine, s_tmp, tot);
  if (before < need && need <= before + mine) {
    uint32_t run = before;
    for (int k = 1; k <= per; ++k) {
      const uint32_t c = h[hi_bin - k];
      if (run + c >= need) {
        s_found[0] = (uint32_t)(hi_bin - k);
        s_found[1] = run;
        break;
      }
      run += c;
    }
  }
  __syncthreads();
  const uint32_t d = s_found[0];
  const uint32_t gt = s_found[1];  // keys in higher bins of this pass
  for (int i = threadIdx.x; i < kHistBins; i += kTopkThreads) h[i] = 0;
  if (threadIdx.x == 0) {
    const int width = pass == 0 ? 11 : pass == 1 ? 11 : 10;
    sel[b * 4 + 0] = pass == 0 ? d : ((prefix << width) | d);
    sel[b * 4 + 1] = need - gt;
    sel[b * 4 + 2] = above + gt;
    sel[b * 4 + 3] = pass + 1;
  }
}

// Keys above K go straight to the candidate list; keys equal to K are counted
// per block (blocks cover consecutive id ranges).
__global__ __launch_bounds__(kTopkThreads) void k_topk_collect(
    const float* __restrict__ pi, int n, const uint32_t* sel, uint32_t* cand_key,
    int32_t* cand_id, uint32_t* cand_cnt, uint32_t* blk_ties, int topk_blocks,
    Ctrl* ctrl) {
  __shared__ uint32_t s_tmp[kTopkThreads / 64];
  if (ctrl->skip) return;
  const int b = blockIdx.y;
  const uint32_t K = sel[b * 4 + 0];
  const uint32_t above = sel[b * 4 + 2];
  const size_t row = (size_t)b * n;
  const int v0 = blockIdx.x * kTopkTile;
  uint32_t ties = 0;
  for (int k = threadIdx.x; k < kTopkTile; k += kTopkThreads) {
    const int v = v0 + k;
    if (v >= n) break;
    const uint32_t key = __float_as_uint(pi[row + v]);
    if (key > K) {
      const uint32_t slot = atomicAdd(&cand_cnt[b], 1u);
      if (slot < above && slot < FORA_MAX_K) {
        cand_key[(size_t)b * FORA_MAX_K + slot] = key;
        cand_id[(size_t)b * FORA_MAX_K + slot] = v;
      } else {
        atomicOr(&ctrl->error, kErrTopk);
      }
    } else if (key == K) {
      ++ties;
    }
  }
  const uint32_t t = block_sum(ties, s_tmp);
  if (threadIdx.x == 0) blk_ties[(size_t)b * topk_blocks + blockIdx.x] = t;
}

// One block per query: exclusive scan of the per-block tie counts.
__global__ __launch_bounds__(1024) void k_topk_tie_scan(uint32_t* blk_ties, int topk_blocks,
                                                        const Ctrl* ctrl) {
  __shared__ uint32_t s_tmp[16];
  if (ctrl->skip) return;
  uint32_t* t = blk_ties + (size_t)blockIdx.x * topk_blocks;
  uint32_t carry = 0;
  for (int base = 0; base < topk_blocks; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t c = i < topk_blocks ? t[i] : 0u;
    uint32_t tot;
    const uint32_t p = block_exclusive_scan(c, s_tmp, tot);
    if (i < topk_blocks) t[i] = carry + p;
    carry += tot;
  }
}

// Blocks whose tie prefix is below the number still needed append their
// ties in id order (each thread owns 16 consecutive ids).
__global__ __launch_bounds__(kTopkThreads) void k_topk_ties(
    const float* __restrict__ pi, int n, const uint32_t* sel, const uint32_t* blk_ties,
    int topk_blocks, uint32_t* cand_key, int32_t* cand_id, const Ctrl* ctrl) {
  __shared__ uint32_t s_tmp[kTopkThreads / 64];
  if (ctrl->skip) return;
  const int b = blockIdx.y;
  const uint32_t K = sel[b * 4 + 0];
  const uint32_t need = sel[b * 4 + 1];
  const uint32_t above = sel[b * 4 + 2];
  const uint32_t pre = blk_ties[(size_t)b * topk_blocks + blockIdx.x];
  if (pre >= need) return;  // uniform per block
  const size_t row = (size_t)b * n;
  const int v0 = blockIdx.x * kTopkTile + threadIdx.x * kTopkPerThread;
  uint32_t mine = 0;
  for (int k = 0; k < kTopkPerThread; ++k) {
    const int v = v0 + k;
    if (v < n && __float_as_uint(pi[row + v]) == K) ++mine;
  }
  uint32_t tot;
  uint32_t rank = pre + block_exclusive_scan(mine, s_tmp, tot);
  for (int k = 0; k < kTopkPerThread && rank < need; ++k) {
    const int v = v0 + k;
    if (v < n && __float_as_uint(pi[row + v]) == K) {
      const uint32_t slot = above + rank;
      if (slot < FORA_MAX_K) {
        cand_key[(size_t)b * FORA_MAX_K + slot] = K;
        cand_id[(size_t)b * FORA_MAX_K + slot] = v;
      }
      ++rank;
    }
  }
}

// One block per query: bitonic sort of the k candidates, ascending on
// ((0xFFFFFFFF - key) << 32 | id), i.e. key descending then id ascending.
__global__ __launch_bounds__(1024) void k_topk_sort(const uint32_t* cand_key,
                                                    const int32_t* cand_id,
                                                    const QueryDev* Q, int kmax,
                                                    int32_t* out_ids, float* out_vals,
                                                    const Ctrl* ctrl) {
  __shared__ u64 s[FORA_MAX_K];
  if (ctrl->skip) return;
  const int b = blockIdx.x;
  const int k = Q[b].k;
  int P = 1;
  while (P < k) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    if (i < k) {
      const uint32_t key = cand_key[(size_t)b * FORA_MAX_K + i];
      const uint32_t id = (uint32_t)cand_id[(size_t)b * FORA_MAX_K + i];
      s[i] = ((u64)(0xFFFFFFFFu - key) << 32) | id;
    } else {
      s[i] = ~0ull;
    }
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int partner = i ^ stride;
        if (partner > i) {
          const bool up = (i & size) == 0;
          const u64 a = s[i], c = s[partner];
          if ((a > c) == up) {
            s[i] = c;
            s[partner] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kmax; i += blockDim.x) {
    if (i < k) {
      const u64 e = s[i];
      out_ids[(size_t)b * kmax + i] = (int32_t)(uint32_t)e;
      out_vals[(size_t)b * kmax + i] = __uint_as_float(0xFFFFFFFFu - (uint32_t)(e >> 32));
    } else {
      out_ids[(size_t)b * kmax + i] = -1;
      out_vals[(size_t)b * kmax + i] = 0.0f;
    }
  }
}

hipError_t launch_topk(const GraphDev& g, const Ws& w, const Layout& L, int batch, int kmax,
                       int32_t* d_ids, float* d_vals, hipStream_t s) {
  dim3 grid((unsigned)L.topk_blocks, (unsigned)batch);
  for (int pass = 0; pass < 3; ++pass) {
    k_topk_hist<<<grid, kTopkThreads, 0, s>>>(pass, w.q, w.acc, w.r, w.queries, w.pi, g.n,
                                              w.hist, w.sel, w.ctrl);
    k_topk_select<<<batch, kTopkThreads, 0, s>>>(pass, w.hist, w.sel, w.queries, w.cand_cnt,
                                                 w.ctrl);
  }
  k_topk_collect<<<grid, kTopkThreads, 0, s>>>(w.pi, g.n, w.sel, w.cand_key, w.cand_id,
                                               w.cand_cnt, w.blk_ties, (int)L.topk_blocks,
                                               w.ctrl);
  k_topk_tie_scan<<<batch, 1024, 0, s>>>(w.blk_ties, (int)L.topk_blocks, w.ctrl);
  k_topk_ties<<<grid, kTopkThreads, 0, s>>>(w.pi, g.n, w.sel, w.blk_ties, (int)L.topk_blocks,
                                            w.cand_key, w.cand_id, w.ctrl);
  k_topk_sort<<<batch, 1024, 0, s>>>(w.cand_key, w.cand_id, w.queries, kmax, d_ids, d_vals,
                                     w.ctrl);
  return hipGetLastError();
}

// Top-k FORA (Algorithm 5) helpers: the k-th value of each staged row, and
// the copy of finished rows to their final places.
__global__ void k_topk_kth(const float* __restrict__ vals, int kmax, const int32_t* __restrict__ ks,
                           int count, float* kth) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) kth[i] = vals[(size_t)i * kmax + ks[i] - 1];
}

__global__ void k_copy_rows(const int32_t* __restrict__ src_ids, const float* __restrict__ src_vals,
                            int kmax, const int32_t* __restrict__ from, const int32_t* __restrict__ to,
                            int count, int32_t* dst_ids, float* dst_vals) {
  for (int r = blockIdx.x; r < count; r += gridDim.x) {
    const size_t a = (size_t)from[r] * kmax, b = (size_t)to[r] * kmax;
    for (int j = threadIdx.x; j < kmax; j += blockDim.x) {
      dst_ids[b + j] = src_ids[a + j];
      dst_vals[b + j] = src_vals[a + j];
    }
  }
}

hipError_t launch_topk_kth(const float* vals, int kmax, const int32_t* ks, int count, float* kth,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_topk_kth<<<(count + 255) / 256, 256, 0, s>>>(vals, kmax, ks, count, kth);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const int32_t* src_ids, const float* src_vals, int kmax,
                            const int32_t* from, const int32_t* to, int count, int32_t* dst_ids,
                            float* dst_vals, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_copy_rows<<<count < 1024 ? count : 1024, 256, 0, s>>>(src_ids, src_vals, kmax, from, to, count,
                                                          dst_ids, dst_vals);
  return hipGetLastError();
}

}  // namespace fora
