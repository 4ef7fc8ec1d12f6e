// sort.hip -- sort of the particle SoA by nearest-node cell, so that the particles a
// workgroup processes are spatially close (mesh reads and deposits then hit the same
// cache lines).  A particle-id array travels with the data so results can be returned
// in load order.  Two sorts:
//
// Stable (the deterministic mode): a least-significant-digit radix sort of (cell, index)
// pairs, then one gather of the payload.  Each digit pass counts the digits of every
// 4096-item tile, scans the counts digit-major, and scatters each tile in item order,
// so particles of one cell keep their previous order and the permutation is the same on
// every run.
//
// Counting sort: histogram with integer atomics, two-level exclusive scan, scatter
// through per-cell cursors.  Both atomic passes aggregate over the wave: the lanes that
// share a cell take one atomic for the group, and each lane its rank in lane order, so
// particles of one wave keep their order within a cell; the order of different waves
// within a cell depends on the timing of their atomics.
#include <math.h>

#include <algorithm>

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
  if (cursor) cursor[i] = v;
}

// exclusive scan of data[0..n) in place (bsum: (n + kScanBlock - 1) / kScanBlock ints)
void scan_exclusive(int32_t* data, int64_t n, int32_t* bsum, int32_t* cursor, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanBlock), 0, s, data, n, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, data, n, bsum, cursor);
}

// ---- stable radix sort of (cell, index) pairs
//
// A workgroup of four waves takes a tile of 4096 consecutive items; wave w takes items
// [1024 w, 1024 w + 1024) of the tile, 64 at a time in item order.
constexpr int kRadixWaves = kBlock / 64;
constexpr int kRadixRounds = 16;
constexpr int kRadixWaveItems = 64 * kRadixRounds;
constexpr int kRadixTile = kRadixWaves * kRadixWaveItems;
constexpr int kRadixMaxBits = 8;

// Valid lanes of the wave whose digit equals this lane's (bits-bit digits).
__device__ __forceinline__ uint64_t digit_peers(int dg, int bits, bool valid) {
  uint64_t m = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool on = ((dg >> b) & 1) != 0;
    const uint64_t set = __ballot(on);
    m &= on ? set : ~set;
  }
  return m;
}

// Per-wave digit counts of the tile into h[w][digit] (zeroed by the caller).
__device__ __forceinline__ void tile_histogram(const int32_t* key, int64_t n, int shift, int bits,
                                               volatile int32_t* h) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile + (int64_t)w * kRadixWaveItems;
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    const int dg = valid ? (key[i] >> shift) & ((1 << bits) - 1) : 0;
    const uint64_t pe = digit_peers(dg, bits, valid);
    // one lane per distinct digit adds the group's size
    if (valid && lane == __ffsll((long long)pe) - 1) h[w * 256 + dg] += __popcll(pe);
  }
}

__global__ __launch_bounds__(kBlock) void k_radix_count(const int32_t* key, int64_t n, int shift, int bits,
                                                        int32_t* counts, int64_t ntiles) {
  __shared__ int32_t h[kRadixWaves * 256];
  for (int d = threadIdx.x; d < kRadixWaves * 256; d += blockDim.x) h[d] = 0;
  __syncthreads();
  tile_histogram(key, n, shift, bits, h);
  __syncthreads();
  for (int d = threadIdx.x; d < (1 << bits); d += blockDim.x) {
    int32_t c = 0;
    for (int w = 0; w < kRadixWaves; ++w) c += h[w * 256 + d];
    counts[(int64_t)d * ntiles + blockIdx.x] = c;
  }
}

// offs: the exclusive digit-major scan of the counts, offs[d ntiles + tile] = first output
// position of digit d in this tile.  Items keep their order within a digit.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const int32_t* key_in, const int32_t* idx_in,
                                                          int32_t* key_out, int32_t* idx_out, int64_t n, int shift,
                                                          int bits, const int32_t* offs, int64_t ntiles) {
  __shared__ int32_t h[kRadixWaves * 256];
  volatile int32_t* hv = h;
  for (int d = threadIdx.x; d < kRadixWaves * 256; d += blockDim.x) h[d] = 0;
  __syncthreads();
  tile_histogram(key_in, n, shift, bits, hv);
  __syncthreads();
  // running output position of each digit for each wave: the tile's base plus the counts
  // of the earlier waves
  for (int d = threadIdx.x; d < (1 << bits); d += blockDim.x) {
    int32_t run = offs[(int64_t)d * ntiles + blockIdx.x];
    for (int w = 0; w < kRadixWaves; ++w) {
      const int32_t c = hv[w * 256 + d];
      hv[w * 256 + d] = run;
      run += c;
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t base = (int64_t)blockIdx.x * kRadixTile + (int64_t)w * kRadixWaveItems;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int r = 0; r < kRadixRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    const int32_t k = valid ? key_in[i] : 0;
    const int dg = (k >> shift) & ((1 << bits) - 1);
    const uint64_t pe = digit_peers(dg, bits, valid);
    const int32_t start = valid ? hv[w * 256 + dg] : 0;
    if (valid) {
      const int32_t pos = start + __popcll(pe & below);
      key_out[pos] = k;
      idx_out[pos] = idx_in ? idx_in[i] : (int32_t)i;
      if (lane == __ffsll((long long)pe) - 1) hv[w * 256 + dg] = start + __popcll(pe);
    }
  }
}

// Nearest-node cell of particle i, and whether its orbit x + s dt v, s in [0, 1], crosses
// a knot of the particle shape (a half-integer node offset for S_2, a node for S_1).
__device__ __forceinline__ int64_t cell_and_cross(const SortArgs& a, int64_t i, bool& cross) {
  int64_t mul = 1, gg = 0;
  cross = false;
  for (int l = 0; l < a.M.d; ++l) {
    const double xi = (a.x[l][i] - a.M.lo[l]) * a.M.inv_h[l];
    double r = floor(xi + 0.5);
    if (!(r > -1.0e9 && r < 1.0e9)) r = 0.0;
    gg += (int64_t)wrapi((int)r, a.M.n[l]) * mul;
    mul *= a.M.n[l];
    const double del = a.dt * ld_bulk(a.v[l], i, a.prec) * a.M.inv_h[l];
    const double k = a.M.shape == 1 ? floor(xi) : r - 0.5;  // knot at or below the point
    const double e = xi + del;
    cross = cross || e < k || e > k + 1.0;
  }
  return gg;
}

// Particles whose orbit crosses a knot: each workgroup adds its count to one of
// kCrossSlots counters (a.xcount[1 ..]), spread so that the atomics do not queue on one
// address; k_cross_total sums them into a.xcount[0].
constexpr int kCrossSlots = 256;
__global__ __launch_bounds__(kBlock) void k_cross_count(SortArgs a) {
  __shared__ int32_t wsum[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool cross = false;
  if (i < a.np) (void)cell_and_cross(a, i, cross);
  const uint64_t m = __ballot(cross);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / 64] = (int32_t)__popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
    if (t) atomicAdd(a.xcount + 1 + (blockIdx.x % kCrossSlots), t);
  }
}

__global__ __launch_bounds__(kCrossSlots) void k_cross_total(int32_t* xcount) {
  __shared__ int32_t sh[kCrossSlots];
  sh[threadIdx.x] = xcount[1 + threadIdx.x];
  __syncthreads();
  for (int off = kCrossSlots / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) xcount[0] = sh[0];
}

// Radix-sort key.  Where knot-crossing particles are dense (at least kDenseCross per cell
// on average), they follow all the others: key = cell + Ng (crossing) or cell, so whole
// waves walk two segments or one, and the crossing waves still hold a cell or two.  Where
// they are sparse, grouping them would spread a wave over many cells; they follow the
// others within their own cell instead: key = 2 cell + (crossing).
constexpr int kDenseCross = 16;
__global__ __launch_bounds__(kBlock) void k_cell_key_only(SortArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  bool cross = false;
  const int64_t gg = cell_and_cross(a, i, cross);
  const bool dense = (int64_t)*a.xcount >= (int64_t)kDenseCross * a.M.Ng;
  a.key[i] = (int32_t)(dense ? gg + (cross ? a.M.Ng : 0) : 2 * gg + (cross ? 1 : 0));
}

// dst[c][i] = src[c][perm[i]] for every moved array, and the particle ids likewise.
__global__ __launch_bounds__(kBlock) void k_gather(SortArgs a, const int32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  const int64_t k = perm[i];
  for (int c = 0; c < a.ncomp; ++c) {
    if (a.esz[c] == 4)
      static_cast<uint32_t*>(a.dst[c])[i] = static_cast<const uint32_t*>(a.src[c])[k];
    else
      static_cast<uint64_t*>(a.dst[c])[i] = static_cast<const uint64_t*>(a.src[c])[k];
  }
  a.id_dst[i] = a.id_src[k];
}

int key_bits(int64_t Ng) {
  int b = 0;
  while (((int64_t)1 << b) < Ng) ++b;
  return std::max(b, 1);
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

int cross_count_ints() { return 1 + kCrossSlots; }

size_t sort_scan_tmp_bytes(int64_t Ng) {
  const int64_t nb = (Ng + kScanBlock - 1) / kScanBlock;
  return sizeof(int32_t) * (size_t)(nb + 1);
}

int64_t radix_count_ints(int64_t np) {
  const int64_t ntiles = std::max<int64_t>((np + kRadixTile - 1) / kRadixTile, 1);
  const int64_t L = ((int64_t)1 << kRadixMaxBits) * ntiles;
  return L + (L + kScanBlock - 1) / kScanBlock + 1;
}

hipError_t sort_by_cell(const SortArgs& a, void* scan_tmp, size_t scan_tmp_bytes, hipStream_t s) {
  if (a.np <= 0) return hipSuccess;
  if (a.stable) {
    const unsigned pb = (unsigned)((a.np + kBlock - 1) / kBlock);
    hipError_t e = hipMemsetAsync(a.xcount, 0, sizeof(int32_t) * (1 + kCrossSlots), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cross_count, dim3(pb), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_cross_total, dim3(1), dim3(kCrossSlots), 0, s, a.xcount);
    hipLaunchKernelGGL(k_cell_key_only, dim3(pb), dim3(kBlock), 0, s, a);
    const int kb = key_bits(2 * a.M.Ng);
    const int passes = (kb + kRadixMaxBits - 1) / kRadixMaxBits;
    const int per = (kb + passes - 1) / passes;
    const int64_t ntiles = (a.np + kRadixTile - 1) / kRadixTile;
    int32_t* counts = a.rcount;
    const int32_t* kin = a.key;
    const int32_t* iin = nullptr;
    int32_t* kout = a.key2;
    int32_t* iout = a.idx;
    for (int p = 0; p < passes; ++p) {
      const int shift = p * per, bits = std::min(per, kb - shift);
      const int64_t L = ((int64_t)1 << bits) * ntiles;
      hipLaunchKernelGGL(k_radix_count, dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, a.np, shift, bits, counts,
                         ntiles);
      scan_exclusive(counts, L, counts + L, nullptr, s);
      hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)ntiles), dim3(kBlock), 0, s, kin, iin, kout, iout, a.np,
                         shift, bits, counts, ntiles);
      // ping-pong: keys between key2 and key, indices between idx and idx2
      kin = kout;
      iin = iout;
      kout = (kout == a.key2) ? a.key : a.key2;
      iout = (iout == a.idx) ? a.idx2 : a.idx;
    }
    hipLaunchKernelGGL(k_gather, dim3(pb), dim3(kBlock), 0, s, a, iin);
    return hipGetLastError();
  }
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
