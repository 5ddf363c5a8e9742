// Counting sort of the particles by mesh tile (kTileLX/LY/LZ), so that
// the deposit and the gather can stage a tile's mesh window in LDS.
//
//   1. count:   key = tile of the particle's cell; rank within the tile from
//               a wave-aggregated atomic on the tile counter (runs of equal
//               keys among consecutive lanes take one atomic for the run).
//   2. scan:    exclusive prefix sum of the tile counts (one block).
//   3. scatter: particle -> start[key] + rank in the workspace copies.
//
// The order inside a tile depends on atomic scheduling; the set of particles
// per tile does not, and no result of the step depends on the order (the
// integer deposit is order-independent and the push is per particle).
#include "internal.h"

namespace fdm {

template <bool FIXED>
__device__ __forceinline__ int cell_of(const void* pos, int64_t np, int64_t i, int d, int logn) {
  if constexpr (FIXED) {
    return (int)(static_cast<const uint32_t*>(pos)[d * np + i] >> (32 - logn));
  } else {
    const float x = static_cast<const float*>(pos)[d * np + i];
    return (int)floorf(x) & ((1 << logn) - 1);
  }
}

template <bool FIXED>
__global__ void __launch_bounds__(kBlock) k_sort_count(const void* __restrict__ pos, int64_t np,
                                                       int logn,
                                                       unsigned* __restrict__ counts,
                                                       unsigned* __restrict__ key_out,
                                                       unsigned* __restrict__ rank_out) {
  const int lane = threadIdx.x & 63;
  const int lz = tile_lz(logn);
  const int ty_n = 1 << (logn - kTileLY), tz_n = 1 << (logn - lz);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs every iteration (uniform trip count), so the
  // cross-lane operations below always see the full wave
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < np; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < np;
    unsigned key = 0xffffffffu;
    if (valid) {
      const int tx = cell_of<FIXED>(pos, np, i, 0, logn) >> kTileLX;
      const int ty = cell_of<FIXED>(pos, np, i, 1, logn) >> kTileLY;
      const int tz = cell_of<FIXED>(pos, np, i, 2, logn) >> lz;
      key = (unsigned)((tx * ty_n + ty) * tz_n + tz);
    }
    const unsigned prev = __shfl_up(key, 1, 64);
    const bool head = (lane == 0) || (prev != key);
    const unsigned long long heads = __ballot(head);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int leader = 63 - __clzll(heads & upto);
    const unsigned long long after = (lane == 63) ? 0ull : (heads & ~upto);
    const int next = after ? __ffsll((long long)after) - 1 : 64;
    unsigned run_base = 0;
    if (head && valid) run_base = atomicAdd(&counts[key], (unsigned)(next - lane));
    run_base = __shfl(run_base, leader, 64);
    if (valid) {
      key_out[i] = key;
      rank_out[i] = run_base + (unsigned)(lane - leader);
    }
  }
}

// Exclusive scan of n counts into start[0..n]; one block of kScanThreads.
constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads) k_sort_scan(const unsigned* __restrict__ counts,
                                                           int n, unsigned* __restrict__ start) {
  __shared__ unsigned part[kScanThreads];
  const int per = (n + kScanThreads - 1) / kScanThreads;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  unsigned s = 0;
  for (int k = lo; k < hi; ++k) s += counts[k];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const unsigned v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int k = lo; k < hi; ++k) {
    start[k] = run;
    run += counts[k];
  }
  if (threadIdx.x == kScanThreads - 1) start[n] = part[kScanThreads - 1];
}

template <bool FIXED, bool IDS>
__global__ void __launch_bounds__(kBlock) k_sort_scatter(
    const void* __restrict__ pos, const float* __restrict__ vel, const int* __restrict__ ids,
    int64_t np, const unsigned* __restrict__ key, const unsigned* __restrict__ rank,
    const unsigned* __restrict__ start, uint32_t* __restrict__ pos_out,
    float* __restrict__ vel_out, int* __restrict__ ids_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const int64_t dst = (int64_t)start[key[i]] + rank[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      pos_out[d * np + dst] = static_cast<const uint32_t*>(pos)[d * np + i];
      vel_out[d * np + dst] = vel[d * np + i];
    }
    if constexpr (IDS) ids_out[dst] = ids[i];
  }
}

static unsigned grid_p(int64_t np) {
  int64_t b = (np + kBlock - 1) / kBlock;
  if (b > 16384) b = 16384;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_sort_count(bool fixed, const void* pos, int64_t np, int logn,
                             unsigned* counts, unsigned* key, unsigned* rank, hipStream_t s) {
  if (fixed)
    hipLaunchKernelGGL(k_sort_count<true>, dim3(grid_p(np)), dim3(kBlock), 0, s, pos, np, logn,
                       counts, key, rank);
  else
    hipLaunchKernelGGL(k_sort_count<false>, dim3(grid_p(np)), dim3(kBlock), 0, s, pos, np, logn,
                       counts, key, rank);
  return hipGetLastError();
}

hipError_t launch_sort_scan(const unsigned* counts, int n, unsigned* start, hipStream_t s) {
  hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, s, counts, n, start);
  return hipGetLastError();
}

hipError_t launch_sort_scatter(const void* pos, const float* vel, const int* ids, int64_t np,
                               const unsigned* key, const unsigned* rank, const unsigned* start,
                               uint32_t* pos_out, float* vel_out, int* ids_out, hipStream_t s) {
  // positions are moved as 32-bit words in both forms
  if (ids)
    hipLaunchKernelGGL((k_sort_scatter<true, true>), dim3(grid_p(np)), dim3(kBlock), 0, s, pos,
                       vel, ids, np, key, rank, start, pos_out, vel_out, ids_out);
  else
    hipLaunchKernelGGL((k_sort_scatter<true, false>), dim3(grid_p(np)), dim3(kBlock), 0, s, pos,
                       vel, ids, np, key, rank, start, pos_out, vel_out, ids_out);
  return hipGetLastError();
}

}  // namespace fdm
