// sort.hip -- counting sort of the particle SoA by nearest-node cell, so that the
// particles a workgroup processes are spatially close (mesh reads and deposits then
// hit the same cache lines).  Histogram with integer atomics, two-level exclusive scan,
// scatter through per-cell cursors.  Both atomic passes aggregate over the wave: the
// lanes that share a cell take one atomic for the group, and each lane its rank in lane
// order, so particles of one wave keep their order within a cell; the order of different
// waves within a cell is not specified.  A particle-id array travels with the data so
// results can be returned in load order.
#include <math.h>

#include "gmhc_internal.h"

namespace gmhc {
namespace {

constexpr int kScanBlock = 1024;

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// ctr[key] += (number of active lanes of the wave with this key), one atomic per
// distinct key; returns the value before the group's addition plus the lane's rank
// among the group's lanes in lane order.  Called by every lane of the wave.
__device__ __forceinline__ int32_t wave_group_add(int32_t* ctr, int32_t key, bool active) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t todo = __ballot(active);
  int32_t mine = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int32_t k = __builtin_amdgcn_readlane(key, leader);
    const uint64_t grp = __ballot(key == k) & todo;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr + k, __popcll(grp));
    base = __builtin_amdgcn_readlane(base, leader);
    if ((grp >> lane) & 1ull) mine = base + __popcll(grp & ((1ull << lane) - 1ull));
    todo &= ~grp;
  }
  return mine;
}

__global__ __launch_bounds__(kBlock) void k_cell_key(SortArgs a) {
  static_assert(kBlock % 64 == 0, "whole waves");
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < a.np;
  int32_t g = 0;
  if (valid) {
    int64_t mul = 1, gg = 0;
    for (int l = 0; l < a.M.d; ++l) {
      const double xi = (a.x[l][i] - a.M.lo[l]) * a.M.inv_h[l];
      // positions are finite and inside the box; clamp anything else into range
      double r = floor(xi + 0.5);
      if (!(r > -1.0e9 && r < 1.0e9)) r = 0.0;
      gg += (int64_t)wrapi((int)r, a.M.n[l]) * mul;
      mul *= a.M.n[l];
    }
    g = (int32_t)gg;
    a.key[i] = g;
  }
  (void)wave_group_add(a.count, g, valid);
}

// exclusive scan of count[0..n) in place; block sums to bsum
__global__ __launch_bounds__(kScanBlock) void k_scan_local(int32_t* data, int64_t n, int32_t* bsum) {
  __shared__ int32_t sh[kScanBlock];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const int32_t v = (i < n) ? data[i] : 0;
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) data[i] = sh[threadIdx.x] - v;
  if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = sh[threadIdx.x];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_sums(int32_t* bsum, int64_t nb) {
  // one workgroup scans the block sums sequentially in chunks
  __shared__ int32_t sh[kScanBlock];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = (i < nb) ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
      int32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nb) bsum[i] = sh[threadIdx.x] - v + carry;
    __syncthreads();
    if (threadIdx.x == kScanBlock - 1) carry += sh[threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(int32_t* data, int64_t n, const int32_t* bsum,
                                                         int32_t* cursor) {
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i >= n) return;
  const int32_t v = data[i] + bsum[blockIdx.x];
  data[i] = v;
  cursor[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_scatter(SortArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < a.np;
  const int32_t key = valid ? a.key[i] : 0;
  const int32_t pos = wave_group_add(a.cursor, key, valid);
  if (!valid) return;
  for (int c = 0; c < a.ncomp; ++c) {
    if (a.esz[c] == 4)
      static_cast<uint32_t*>(a.dst[c])[pos] = static_cast<const uint32_t*>(a.src[c])[i];
    else
      static_cast<uint64_t*>(a.dst[c])[pos] = static_cast<const uint64_t*>(a.src[c])[i];
  }
  a.id_dst[pos] = a.id_src[i];
}

}  // namespace

size_t sort_scan_tmp_bytes(int64_t Ng) {
  const int64_t nb = (Ng + kScanBlock - 1) / kScanBlock;
  return sizeof(int32_t) * (size_t)(nb + 1);
}

hipError_t sort_by_cell(const SortArgs& a, void* scan_tmp, size_t scan_tmp_bytes, hipStream_t s) {
  if (a.np <= 0) return hipSuccess;
  const int64_t Ng = a.M.Ng;
  const int64_t nb = (Ng + kScanBlock - 1) / kScanBlock;
  if (scan_tmp_bytes < sort_scan_tmp_bytes(Ng)) return hipErrorInvalidValue;
  int32_t* bsum = static_cast<int32_t*>(scan_tmp);
  hipError_t e = hipMemsetAsync(a.count, 0, sizeof(int32_t) * (size_t)Ng, s);
  if (e != hipSuccess) return e;
  const unsigned pb = (unsigned)((a.np + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_cell_key, dim3(pb), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanBlock), 0, s, a.count, Ng, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, a.count, Ng, bsum, a.cursor);
  hipLaunchKernelGGL(k_scatter, dim3(pb), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace gmhc
