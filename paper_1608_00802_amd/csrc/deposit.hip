// Cloud-in-cell mass deposit, step (i) of Sec. II A (the paper's density
// estimate Eq. (9) with the trilinear CIC kernel in place of its spline).
//
// Fixed-point form: positions are uint32 u*2^32/N, so the top log2(N) bits are
// the cell index and the low B = 32 - log2(N) bits the fraction.  Each particle
// carries exactly 2^40 integer mass units.  A corner weight is
// w_x w_y w_z / 2^(3B) of the particle: the product w_x w_y (< 2^(2B)) is
// exact in 64-bit integers, and exact in FP64 for N >= 64 (2B <= 52); the
// multiplication by w_z is one FP64 rounding (relative 2^-53 of a value of at
// most 2^40 units: at most 2^-13 units), the scale to 2^40 units is an exact
// power of two and rint gives the integer weight -- deterministic, within
// 0.5 + 2^-13 units of the exact value.  For N <= 32 (B >= 27) w_x w_y reaches
// 2^(2B) >= 2^54 and its conversion to FP64 is a second rounding of the same
// size: within 0.5 + 2^-12 units.  The corner with the largest weight takes the remainder,
// so every particle deposits exactly 2^40 units.  Integer atomics commute,
// which makes the mesh bitwise independent of particle order and scheduling.
//
// Plain FP32 form: float positions and float atomics (order-dependent in the
// last bits), kept as the comparison baseline.
#include <type_traits>

#include "cic.h"
#include "internal.h"

namespace fdm {

__global__ void __launch_bounds__(kBlock) k_fill_zero16(uint4* __restrict__ p, size_t n16,
                                                        Batch bt) {
  p = woff(p, bt, bslot(bt));
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s, const Batch& bt) {
  // callers pass 16-byte multiples of 256-byte aligned buffers
  size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  size_t blocks = (n16 + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero16, dim3((unsigned)blocks, bt.count), dim3(kBlock), 0, s,
                     (uint4*)p, n16, bt);
  return hipGetLastError();
}

template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_deposit_fixed(const uint32_t* __restrict__ px,
                                                          const uint32_t* __restrict__ py,
                                                          const uint32_t* __restrict__ pz,
                                                          int64_t np,
                                                          unsigned long long* __restrict__ mass,
                                                          Batch bt) {
  const int sl = bslot(bt);
  px = poff(px, bt, sl);
  py = poff(py, bt, sl);
  pz = poff(pz, bt, sl);
  mass = woff(mass, bt, sl);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    int ix, iy, iz;
    unsigned long long w[8];
    fixed_weights<LOGN>(px[i], py[i], pz[i], ix, iy, iz, w);
    deposit_global<LOGN>(mass, ix, iy, iz, w);
  }
}

template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_deposit_f32(const float* __restrict__ px,
                                                        const float* __restrict__ py,
                                                        const float* __restrict__ pz,
                                                        int64_t np, float* __restrict__ acc,
                                                        Batch bt) {
  const int sl = bslot(bt);
  px = poff(px, bt, sl);
  py = poff(py, bt, sl);
  pz = poff(pz, bt, sl);
  acc = woff(acc, bt, sl);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    int ix, iy, iz;
    float w[8];
    float_weights<LOGN>(px[i], py[i], pz[i], ix, iy, iz, w);
    deposit_global<LOGN>(acc, ix, iy, iz, w);
  }
}

// Tiled deposit: block b owns tile b of the particle sort and accumulates
// its particles into an LDS window of (TX+1)(TY+1)(TZ+1) cells (the tile plus
// the +1 faces CIC reaches), then adds the window to the mesh with one global
// atomic per non-zero cell.  Particles that left their tile since the sort
// deposit with global atomics directly, so the result never depends on how
// well sorted the particles are.
// Threads per block of the tiled deposit: its 34 KB window leaves room for
// four blocks per CU, so 512-thread blocks fill all 32 wave slots.
constexpr int kDepBlock = 512;

template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kDepBlock) k_deposit_tiled(const void* __restrict__ pos,
                                                          int64_t np, TileMap tm,
                                                          void* __restrict__ mass_v, Batch bt) {
  using T = typename std::conditional<FIXED, unsigned long long, float>::type;
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << tile_lx(LOGN), TY = 1 << tile_ly(LOGN), TZ = 1 << tile_lz(LOGN);
  constexpr int HD = kDepHalo;   // window: cells o - HD .. o + T + HD
  constexpr int WX = TX + 1 + 2 * HD, WY = TY + 1 + 2 * HD, WZ = TZ + 1 + 2 * HD;
  constexpr int NTY = N / TY, NTZ = N / TZ;
  __shared__ T acc[WX * WY * WZ];
  const int sl = bslot(bt);
  pos = poff(pos, bt, sl);
  T* mass = woff(static_cast<T*>(mass_v), bt, sl);
  tm.start = woff(tm.start, bt, sl);
  tm.chunk_start = woff(tm.chunk_start, bt, sl);
  int t;
  unsigned lo, hi;
  if (!chunk_of(tm, t, lo, hi)) return;
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kDepBlock) acc[c] = (T)0;
  __syncthreads();
  for (unsigned i = lo + threadIdx.x; i < hi; i += kDepBlock) {
    int ix, iy, iz;
    T w[8];
    if constexpr (FIXED) {
      const uint32_t* p = static_cast<const uint32_t*>(pos);
      fixed_weights<LOGN>(p[i], p[np + i], p[2 * np + i], ix, iy, iz, w);
    } else {
      const float* p = static_cast<const float*>(pos);
      float_weights<LOGN>(p[i], p[np + i], p[2 * np + i], ix, iy, iz, w);
    }
    const int rx = (ix - ox + HD) & MASK, ry = (iy - oy + HD) & MASK, rz = (iz - oz + HD) & MASK;
    if (rx < TX + 2 * HD && ry < TY + 2 * HD && rz < TZ + 2 * HD) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        atomicAdd(&acc[((rx + (c >> 2)) * WY + ry + ((c >> 1) & 1)) * WZ + rz + (c & 1)], w[c]);
    } else {
      deposit_global<LOGN>(mass, ix, iy, iz, w);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kDepBlock) {
    const T v = acc[c];
    if (v != (T)0) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t cell = ((size_t)((ox - HD + lx) & MASK) * N + ((oy - HD + ly) & MASK)) * N +
                          ((oz - HD + lz) & MASK);
      add_global(&mass[cell], v);
    }
  }
}

static unsigned grid_for(int64_t np) {
  int64_t b = (np + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_deposit_fixed(const uint32_t* pos, int64_t np, int logn,
                                unsigned long long* mass, hipStream_t s, const Batch& bt) {
  const unsigned g = grid_for(np);
#define L_(LN)                                                                                \
  hipLaunchKernelGGL(k_deposit_fixed<LN>, dim3(g, bt.count), dim3(kBlock), 0, s, pos, pos + np, \
                     pos + 2 * np, np, mass, bt)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_fixed_tiled(const uint32_t* pos, int64_t np, int logn,
                                      const TileMap& tm, unsigned long long* mass,
                                      hipStream_t s, const Batch& bt) {
  const dim3 g(tiled_grid(np, tm.tiles), bt.count);
#define L_(LN) \
  hipLaunchKernelGGL((k_deposit_tiled<LN, true>), g, dim3(kDepBlock), 0, s, pos, np, tm, mass, bt)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_f32_tiled(const float* pos, int64_t np, int logn, const TileMap& tm,
                                    float* acc, hipStream_t s, const Batch& bt) {
  const dim3 g(tiled_grid(np, tm.tiles), bt.count);
#define L_(LN) \
  hipLaunchKernelGGL((k_deposit_tiled<LN, false>), g, dim3(kDepBlock), 0, s, pos, np, tm, acc, bt)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_f32(const float* pos, int64_t np, int logn, float* acc,
                              hipStream_t s, const Batch& bt) {
  const unsigned g = grid_for(np);
#define L_(LN)                                                                              \
  hipLaunchKernelGGL(k_deposit_f32<LN>, dim3(g, bt.count), dim3(kBlock), 0, s, pos, pos + np, \
                     pos + 2 * np, np, acc, bt)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace fdm
