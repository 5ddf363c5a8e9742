// Counting sort of the particles by mesh tile (kTileLX/LY/LZ), so that
// the deposit and the gather can stage a tile's mesh window in LDS.
//
//   1. count:   a block takes a contiguous range of kCountPer * kCountBlock
//               particles and counts them per tile in an LDS hash table
//               (runs of equal tiles among consecutive lanes take one LDS
//               atomic); then one device atomic per distinct tile of the
//               block reserves the block's ranks on the counter of its
//               slice (block mod kSlices).  Counters are slice-major, so the
//               slices of a tile lie in different cache lines.
//   2. scan:    exclusive prefix sums of the sliced counts, of the tile
//               counts and of the chunks per tile (reduce per block of
//               tiles, then a down-sweep that adds the block offsets).
//   3. scatter: particle -> slice_start[key] + rank in the workspace copies;
//               a tile's slices are adjacent, so each tile stays contiguous.
//
// Device atomics on one cache line serialise across the whole chip, and a
// densely populated tile holds millions of particles, so the count keeps
// them to one per (block, tile).  The order inside a tile depends on atomic
// scheduling; the set of particles per tile does not, and no result of the
// step depends on the order (the integer deposit is order-independent and
// the push is per particle).
#include "internal.h"

namespace fdm {

constexpr int kCountBlock = 256;
constexpr int kCountPer = 16;                 // particles per thread
constexpr int kHashBits = 9;
constexpr int kHash = 1 << kHashBits;        // LDS hash slots per block
constexpr int kProbe = 16;
constexpr unsigned kEmpty = 0xffffffffu;
constexpr int kScanBlock = 256;               // tiles per scan block

template <bool FIXED>
__device__ __forceinline__ int cell_of(const void* pos, int64_t np, int64_t i, int d, int logn) {
  if constexpr (FIXED) {
    return (int)(static_cast<const uint32_t*>(pos)[d * np + i] >> (32 - logn));
  } else {
    const float x = static_cast<const float*>(pos)[d * np + i];
    return (int)floorf(x) & ((1 << logn) - 1);
  }
}

// Slot of key in the block's hash table (inserted if absent), kEmpty if the
// probe sequence is full.
__device__ __forceinline__ unsigned hash_slot(unsigned* hkey, unsigned key) {
  unsigned h = (key * 2654435761u) >> (32 - kHashBits);
  for (int k = 0; k < kProbe; ++k) {
    const unsigned cur = hkey[h] == key ? key : atomicCAS(&hkey[h], kEmpty, key);
    if (cur == kEmpty || cur == key) return h;
    h = (h + 1) & (kHash - 1);
  }
  return kEmpty;
}

template <bool FIXED>
__global__ void __launch_bounds__(kCountBlock) k_sort_count(const void* __restrict__ pos,
                                                            int64_t np, int logn,
                                                            unsigned* __restrict__ counts,
                                                            int cstride,
                                                            unsigned* __restrict__ key_out,
                                                            unsigned* __restrict__ rank_out,
                                                            Batch bt) {
  {
    const int sl = bslot(bt);
    pos = poff(pos, bt, sl);
    counts = woff(counts, bt, sl);
    key_out = woff(key_out, bt, sl);
    rank_out = woff(rank_out, bt, sl);
  }
  __shared__ unsigned hkey[kHash], hcnt[kHash];
  for (int i = threadIdx.x; i < kHash; i += kCountBlock) {
    hkey[i] = kEmpty;
    hcnt[i] = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int lx = tile_lx(logn), ly = tile_ly(logn), lz = tile_lz(logn);
  const int ty_n = 1 << (logn - ly), tz_n = 1 << (logn - lz);
  const unsigned slice = blockIdx.x % kSlices;
  unsigned* cnt = counts + (size_t)slice * cstride;
  const int64_t base = (int64_t)blockIdx.x * (kCountBlock * kCountPer) + threadIdx.x;
  unsigned tkey[kCountPer], slot[kCountPer], loc[kCountPer];
  // every lane of a wave runs every iteration, so the cross-lane operations
  // always see the full wave
#pragma unroll
  for (int j = 0; j < kCountPer; ++j) {
    const int64_t i = base + (int64_t)j * kCountBlock;
    const bool valid = i < np;
    unsigned key = kEmpty;
    if (valid) {
      const int tx = cell_of<FIXED>(pos, np, i, 0, logn) >> lx;
      const int ty = cell_of<FIXED>(pos, np, i, 1, logn) >> ly;
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
    unsigned s = kEmpty, b = 0;
    if (head && valid) {
      s = hash_slot(hkey, key);
      // a full table sends the run straight to the device counter
      b = s != kEmpty ? atomicAdd(&hcnt[s], (unsigned)(next - lane))
                      : atomicAdd(&cnt[key], (unsigned)(next - lane));
    }
    s = __shfl(s, leader, 64);
    b = __shfl(b, leader, 64);
    tkey[j] = key;
    slot[j] = s;
    loc[j] = b + (unsigned)(lane - leader);
  }
  __syncthreads();
  // one device atomic per distinct tile of the block: the block's base rank
  for (int i = threadIdx.x; i < kHash; i += kCountBlock) {
    const unsigned k = hkey[i];
    if (k != kEmpty) hcnt[i] = atomicAdd(&cnt[k], hcnt[i]);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kCountPer; ++j) {
    const int64_t i = base + (int64_t)j * kCountBlock;
    if (i < np) {
      key_out[i] = tkey[j] * kSlices + slice;
      rank_out[i] = slot[j] != kEmpty ? hcnt[slot[j]] + loc[j] : loc[j];
    }
  }
}

// Exclusive block-wide prefix sums of (a, b) over kScanBlock threads; also
// returns the block totals.
__device__ __forceinline__ void block_scan2(unsigned& a, unsigned& b, unsigned& ta,
                                            unsigned& tb) {
  __shared__ unsigned wa[kScanBlock / 64], wb[kScanBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned ia = a, ib = b;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned va = __shfl_up(ia, off, 64), vb = __shfl_up(ib, off, 64);
    if (lane >= off) {
      ia += va;
      ib += vb;
    }
  }
  if (lane == 63) {
    wa[w] = ia;
    wb[w] = ib;
  }
  __syncthreads();
  unsigned pa = 0, pb = 0;
  ta = tb = 0;
#pragma unroll
  for (int k = 0; k < kScanBlock / 64; ++k) {
    if (k < w) {
      pa += wa[k];
      pb += wb[k];
    }
    ta += wa[k];
    tb += wb[k];
  }
  a = pa + ia - a;
  b = pb + ib - b;
  __syncthreads();
}

__device__ __forceinline__ unsigned tile_total(const unsigned* counts, int cstride, int t,
                                               unsigned* sl) {
  unsigned tot = 0;
#pragma unroll
  for (int s = 0; s < kSlices; ++s) {
    const unsigned c = counts[(size_t)s * cstride + t];
    if (sl) sl[s] = c;
    tot += c;
  }
  return tot;
}

// Per block of kScanBlock tiles: particle and chunk totals.
__global__ void __launch_bounds__(kScanBlock) k_sort_scan_reduce(const unsigned* __restrict__ counts,
                                                                int tiles, int cstride,
                                                                unsigned* __restrict__ sums,
                                                                Batch bt) {
  {
    const int sl = bslot(bt);
    counts = woff(counts, bt, sl);
    sums = woff(sums, bt, sl);
  }
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  unsigned a = 0, b = 0;
  if (t < tiles) {
    a = tile_total(counts, cstride, t, nullptr);
    b = (a + kChunk - 1) / kChunk;
  }
  unsigned ta, tb;
  block_scan2(a, b, ta, tb);
  if (threadIdx.x == 0) {
    sums[2 * blockIdx.x] = ta;
    sums[2 * blockIdx.x + 1] = tb;
  }
}

// Down-sweep: offsets of the earlier blocks, then per-tile prefix sums.
__global__ void __launch_bounds__(kScanBlock) k_sort_scan_down(const unsigned* __restrict__ counts,
                                                              int tiles, int cstride,
                                                              const unsigned* __restrict__ sums,
                                                              unsigned* __restrict__ slice_start,
                                                              unsigned* __restrict__ tile_start,
                                                              unsigned* __restrict__ chunk_start,
                                                              Batch bt) {
  {
    const int sl = bslot(bt);
    counts = woff(counts, bt, sl);
    sums = woff(sums, bt, sl);
    slice_start = woff(slice_start, bt, sl);
    tile_start = woff(tile_start, bt, sl);
    chunk_start = woff(chunk_start, bt, sl);
  }
  __shared__ unsigned off[2];
  if (threadIdx.x < 64) {
    unsigned pa = 0, pb = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += 64) {
      pa += sums[2 * k];
      pb += sums[2 * k + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      pa += __shfl_xor(pa, o, 64);
      pb += __shfl_xor(pb, o, 64);
    }
    if (threadIdx.x == 0) {
      off[0] = pa;
      off[1] = pb;
    }
  }
  __syncthreads();
  const int t = blockIdx.x * kScanBlock + threadIdx.x;
  unsigned c[kSlices];
  unsigned a = 0, b = 0;
  if (t < tiles) {
    a = tile_total(counts, cstride, t, c);
    b = (a + kChunk - 1) / kChunk;
  }
  unsigned ta, tb;
  block_scan2(a, b, ta, tb);
  a += off[0];
  b += off[1];
  if (t < tiles) {
    tile_start[t] = a;
    chunk_start[t] = b;
    unsigned r = a;
    uint4* s4 = reinterpret_cast<uint4*>(slice_start + (size_t)t * kSlices);
#pragma unroll
    for (int v = 0; v < kSlices / 4; ++v) {
      uint4 o;
      o.x = r;
      o.y = o.x + c[4 * v];
      o.z = o.y + c[4 * v + 1];
      o.w = o.z + c[4 * v + 2];
      r = o.w + c[4 * v + 3];
      s4[v] = o;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    slice_start[(size_t)tiles * kSlices] = off[0] + ta;
    tile_start[tiles] = off[0] + ta;
    chunk_start[tiles] = off[1] + tb;
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
  if (b > 262144) b = 262144;   // up to one particle per thread at 256^3
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_sort_count(bool fixed, const void* pos, int64_t np, int logn,
                             unsigned* counts, unsigned* key, unsigned* rank, hipStream_t s,
                             const Batch& bt) {
  const int64_t per = (int64_t)kCountBlock * kCountPer;
  const dim3 g((unsigned)(np > 0 ? (np + per - 1) / per : 1), bt.count);
  const int cs = count_stride(tile_count(logn));
  if (fixed)
    hipLaunchKernelGGL(k_sort_count<true>, g, dim3(kCountBlock), 0, s, pos, np, logn, counts, cs,
                       key, rank, bt);
  else
    hipLaunchKernelGGL(k_sort_count<false>, g, dim3(kCountBlock), 0, s, pos, np, logn, counts,
                       cs, key, rank, bt);
  return hipGetLastError();
}

hipError_t launch_sort_scan(const unsigned* counts, int tiles, unsigned* sums,
                            unsigned* slice_start, unsigned* tile_start, unsigned* chunk_start,
                            hipStream_t s, const Batch& bt) {
  const dim3 g(scan_blocks(tiles), bt.count);
  const int cs = count_stride(tiles);
  hipLaunchKernelGGL(k_sort_scan_reduce, g, dim3(kScanBlock), 0, s, counts, tiles, cs, sums, bt);
  hipLaunchKernelGGL(k_sort_scan_down, g, dim3(kScanBlock), 0, s, counts, tiles, cs, sums,
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
