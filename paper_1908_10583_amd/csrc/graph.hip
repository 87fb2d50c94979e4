// Graph ingest checks, the per-node {row start, out-degree} table, a zero
// fill, and the device Philox block kernel used for RNG checks.
#include "internal.h"

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
