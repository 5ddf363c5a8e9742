// Counting sort of the particles by mesh tile (kTileLX/LY/LZ), so that
// the deposit and the gather can stage a tile's mesh window in LDS.
//
//   1. count:   key = (tile of the particle's cell, slice = block mod
//               kSlices); rank within the key from a wave-aggregated atomic
//               on its counter (runs of equal keys among consecutive lanes
//               take one atomic for the run).
//   2. scan:    exclusive prefix sums of the sliced counts, of the tile
//               counts and of the chunks per tile (one block).
//   3. scatter: particle -> slice_start[key] + rank in the workspace copies;
//               a tile's slices are adjacent, so each tile stays contiguous.
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
                                                       unsigned* __restrict__ rank_out, Batch bt) {
  {
    const int sl = bslot(bt);
    pos = poff(pos, bt, sl);
    counts = woff(counts, bt, sl);
    key_out = woff(key_out, bt, sl);
    rank_out = woff(rank_out, bt, sl);
  }
  const int lane = threadIdx.x & 63;
  const int lx = tile_lx(logn), ly = tile_ly(logn), lz = tile_lz(logn);
  const int ty_n = 1 << (logn - ly), tz_n = 1 << (logn - lz);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // every lane of a wave runs every iteration (uniform trip count), so the
  // cross-lane operations below always see the full wave
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < np; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool valid = i < np;
    unsigned key = 0xffffffffu;
    if (valid) {
      const int tx = cell_of<FIXED>(pos, np, i, 0, logn) >> lx;
      const int ty = cell_of<FIXED>(pos, np, i, 1, logn) >> ly;
      const int tz = cell_of<FIXED>(pos, np, i, 2, logn) >> lz;
      key = (unsigned)((tx * ty_n + ty) * tz_n + tz) * kSlices + (blockIdx.x % kSlices);
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

// One block scans the sliced tile counts.  Thread k owns a contiguous run
// of tiles; a tile's kSlices counters are read as four 16-byte vectors.  Two
// exclusive prefix sums come out of one pass: particles per slice (and per
// tile) and chunks per tile.
constexpr int kScanThreads = 1024;
static_assert(kSlices == 16, "the scan reads a tile's counters as four uint4");

__device__ __forceinline__ void block_scan2(unsigned& a, unsigned& b, unsigned* pa,
                                            unsigned* pb) {
  // inclusive Hillis-Steele scan of (a, b) over the block, returns exclusive
  pa[threadIdx.x] = a;
  pb[threadIdx.x] = b;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const unsigned va = (int)threadIdx.x >= off ? pa[threadIdx.x - off] : 0u;
    const unsigned vb = (int)threadIdx.x >= off ? pb[threadIdx.x - off] : 0u;
    __syncthreads();
    pa[threadIdx.x] += va;
    pb[threadIdx.x] += vb;
    __syncthreads();
  }
  a = threadIdx.x ? pa[threadIdx.x - 1] : 0u;
  b = threadIdx.x ? pb[threadIdx.x - 1] : 0u;
}

__global__ void __launch_bounds__(kScanThreads) k_sort_scan(const unsigned* __restrict__ counts,
                                                           int tiles,
                                                           unsigned* __restrict__ slice_start,
                                                           unsigned* __restrict__ tile_start,
                                                           unsigned* __restrict__ chunk_start,
                                                           Batch bt) {
  {
    const int sl = bslot(bt);
    counts = woff(counts, bt, sl);
    slice_start = woff(slice_start, bt, sl);
    tile_start = woff(tile_start, bt, sl);
    chunk_start = woff(chunk_start, bt, sl);
  }
  __shared__ unsigned pa[kScanThreads], pb[kScanThreads];
  const int per = (tiles + kScanThreads - 1) / kScanThreads;
  const int lo = threadIdx.x * per;
  const int hi = min(tiles, lo + per);
  const uint4* c4 = reinterpret_cast<const uint4*>(counts);
  unsigned sp = 0, sc = 0;
  for (int t = lo; t < hi; ++t) {
    unsigned tot = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint4 c = c4[4 * t + v];
      tot += c.x + c.y + c.z + c.w;
    }
    sp += tot;
    sc += (tot + kChunk - 1) / kChunk;
  }
  unsigned rp = sp, rc = sc;
  block_scan2(rp, rc, pa, pb);
  uint4* s4 = reinterpret_cast<uint4*>(slice_start);
  for (int t = lo; t < hi; ++t) {
    tile_start[t] = rp;
    chunk_start[t] = rc;
    unsigned tot = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint4 c = c4[4 * t + v];
      uint4 o;
      o.x = rp;
      o.y = o.x + c.x;
      o.z = o.y + c.y;
      o.w = o.z + c.z;
      rp = o.w + c.w;
      tot += c.x + c.y + c.z + c.w;
      s4[4 * t + v] = o;
    }
    rc += (tot + kChunk - 1) / kChunk;
  }
  if (threadIdx.x == kScanThreads - 1) {
    slice_start[(size_t)tiles * kSlices] = rp;
    tile_start[tiles] = rp;
    chunk_start[tiles] = rc;
  }
}

template <bool FIXED, bool IDS>
__global__ void __launch_bounds__(kBlock) k_sort_scatter(
    const void* __restrict__ pos, const float* __restrict__ vel, const int* __restrict__ ids,
    int64_t np, const unsigned* __restrict__ key, const unsigned* __restrict__ rank,
    const unsigned* __restrict__ slice_start, uint32_t* __restrict__ pos_out,
    float* __restrict__ vel_out, int* __restrict__ ids_out, Batch bt) {
  {
    const int sl = bslot(bt);
    pos = poff(pos, bt, sl);
    vel = poff(vel, bt, sl);
    key = woff(key, bt, sl);
    rank = woff(rank, bt, sl);
    slice_start = woff(slice_start, bt, sl);
    pos_out = woff(pos_out, bt, sl);
    vel_out = woff(vel_out, bt, sl);
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const int64_t dst = (int64_t)slice_start[key[i]] + rank[i];
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
                             unsigned* counts, unsigned* key, unsigned* rank, hipStream_t s,
                             const Batch& bt) {
  const dim3 g(grid_p(np), bt.count);
  if (fixed)
    hipLaunchKernelGGL(k_sort_count<true>, g, dim3(kBlock), 0, s, pos, np, logn, counts, key,
                       rank, bt);
  else
    hipLaunchKernelGGL(k_sort_count<false>, g, dim3(kBlock), 0, s, pos, np, logn, counts, key,
                       rank, bt);
  return hipGetLastError();
}

hipError_t launch_sort_scan(const unsigned* counts, int tiles, unsigned* slice_start,
                            unsigned* tile_start, unsigned* chunk_start, hipStream_t s,
                            const Batch& bt) {
  hipLaunchKernelGGL(k_sort_scan, dim3(1, bt.count), dim3(kScanThreads), 0, s, counts, tiles,
                     slice_start, tile_start, chunk_start, bt);
  return hipGetLastError();
}

hipError_t launch_sort_scatter(const void* pos, const float* vel, const int* ids, int64_t np,
                               const unsigned* key, const unsigned* rank, const unsigned* start,
                               uint32_t* pos_out, float* vel_out, int* ids_out,
                               hipStream_t s, const Batch& bt) {
  // positions are moved as 32-bit words in both forms; ids only for single runs
  const dim3 g(grid_p(np), bt.count);
  if (ids && !bt.slots)
    hipLaunchKernelGGL((k_sort_scatter<true, true>), g, dim3(kBlock), 0, s, pos, vel, ids, np,
                       key, rank, start, pos_out, vel_out, ids_out, bt);
  else
    hipLaunchKernelGGL((k_sort_scatter<true, false>), g, dim3(kBlock), 0, s, pos, vel, ids, np,
                       key, rank, start, pos_out, vel_out, ids_out, bt);
  return hipGetLastError();
}

// Copy the sorted particle copies back (batched launches; single runs use a
// device-to-device memcpy).
__global__ void __launch_bounds__(kBlock) k_sort_copy(uint32_t* __restrict__ pos,
                                                      float* __restrict__ vel,
                                                      const uint32_t* __restrict__ pos_tmp,
                                                      const float* __restrict__ vel_tmp,
                                                      int64_t n3, Batch bt) {
  const int sl = bslot(bt);
  pos = poff(pos, bt, sl);
  vel = poff(vel, bt, sl);
  pos_tmp = woff(pos_tmp, bt, sl);
  vel_tmp = woff(vel_tmp, bt, sl);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += stride) {
    pos[i] = pos_tmp[i];
    vel[i] = vel_tmp[i];
  }
}

hipError_t launch_sort_copy(uint32_t* pos, float* vel, const uint32_t* pos_tmp,
                            const float* vel_tmp, int64_t np, hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_sort_copy, dim3(grid_p(3 * np), bt.count), dim3(kBlock), 0, s, pos, vel,
                     pos_tmp, vel_tmp, 3 * np, bt);
  return hipGetLastError();
}

}  // namespace fdm
