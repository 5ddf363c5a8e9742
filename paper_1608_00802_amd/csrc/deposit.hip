// Cloud-in-cell mass deposit, step (i) of Sec. II A (the paper's density
// estimate Eq. (9) with the trilinear CIC kernel in place of its spline).
//
// Fixed-point form: positions are uint32 u*2^32/N, so the top log2(N) bits are
// the cell index and the low B = 32 - log2(N) bits the fraction.  Each particle
// carries exactly 2^40 integer mass units.  A corner weight is
// w_x w_y w_z / 2^(3B) of the particle: the product w_x w_y (< 2^51) is exact
// in 64-bit integers and in FP64, the multiplication by w_z is one FP64
// rounding (relative 2^-53), the scale to 2^40 units is an exact power of two
// and rint gives the integer weight -- deterministic, within 0.5 + 2^-10 units
// of the exact value.  The corner with the largest weight takes the remainder,
// so every particle deposits exactly 2^40 units.  Integer atomics commute,
// which makes the mesh bitwise independent of particle order and scheduling.
//
// Plain FP32 form: float positions and float atomics (order-dependent in the
// last bits), kept as the comparison baseline.
#include <type_traits>

#include "internal.h"

namespace fdm {

__global__ void __launch_bounds__(kBlock) k_fill_zero16(uint4* __restrict__ p, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  // callers pass 16-byte multiples of 256-byte aligned buffers
  size_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  size_t blocks = (n16 + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero16, dim3((unsigned)blocks), dim3(kBlock), 0, s, (uint4*)p, n16);
  return hipGetLastError();
}

// Cell index and the eight integer corner weights (2^40 units per particle)
// of one fixed-point particle.  Corner c = 4 cx + 2 cy + cz.
template <int LOGN>
__device__ __forceinline__ void fixed_weights(uint32_t ux, uint32_t uy, uint32_t uz, int& ix,
                                              int& iy, int& iz, unsigned long long w[8]) {
  constexpr int B = 32 - LOGN;
  constexpr unsigned long long ONE = 1ull << B;
  const double scale = ldexp(1.0, kMassShift - 3 * B);  // 2^(40 - 3B), exact
  ix = (int)(ux >> B);
  iy = (int)(uy >> B);
  iz = (int)(uz >> B);
  const unsigned long long fx = ux & (ONE - 1), fy = uy & (ONE - 1), fz = uz & (ONE - 1);
  const unsigned long long wx[2] = {ONE - fx, fx};
  const unsigned long long wy[2] = {ONE - fy, fy};
  const unsigned long long wz[2] = {ONE - fz, fz};
  const int big = ((fx >= (ONE >> 1)) << 2) | ((fy >= (ONE >> 1)) << 1) | (fz >= (ONE >> 1));
  unsigned long long sum = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const unsigned long long wxy = wx[c >> 2] * wy[(c >> 1) & 1];
    w[c] = (unsigned long long)rint((double)wxy * (double)wz[c & 1] * scale);
    sum += (c == big) ? 0ull : w[c];
  }
  // remainder to the heaviest corner: exactly 2^40 per particle
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (c == big) w[c] = (1ull << kMassShift) - sum;
}

// Cell index and trilinear weights of one float particle.
template <int LOGN>
__device__ __forceinline__ void float_weights(float x, float y, float z, int& ix, int& iy,
                                              int& iz, float w[8]) {
  constexpr int MASK = (1 << LOGN) - 1;
  const float flx = floorf(x), fly = floorf(y), flz = floorf(z);
  const float fx = x - flx, fy = y - fly, fz = z - flz;
  ix = (int)flx & MASK;
  iy = (int)fly & MASK;
  iz = (int)flz & MASK;
  const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
#pragma unroll
  for (int c = 0; c < 8; ++c) w[c] = wx[c >> 2] * wy[(c >> 1) & 1] * wz[c & 1];
}

__device__ __forceinline__ void add_global(unsigned long long* p, unsigned long long v) {
  atomicAdd(p, v);
}
__device__ __forceinline__ void add_global(float* p, float v) { unsafeAtomicAdd(p, v); }

template <int LOGN, typename T>
__device__ __forceinline__ void deposit_global(T* __restrict__ mass, int ix, int iy, int iz,
                                               const T w[8]) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cx = (ix + (c >> 2)) & MASK;
    const int cy = (iy + ((c >> 1) & 1)) & MASK;
    const int cz = (iz + (c & 1)) & MASK;
    if (w[c] != (T)0) add_global(&mass[((size_t)cx * N + cy) * N + cz], w[c]);
  }
}

template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_deposit_fixed(const uint32_t* __restrict__ px,
                                                          const uint32_t* __restrict__ py,
                                                          const uint32_t* __restrict__ pz,
                                                          int64_t np,
                                                          unsigned long long* __restrict__ mass) {
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
                                                        int64_t np, float* __restrict__ acc) {
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
template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_deposit_tiled(const void* __restrict__ pos,
                                                          int64_t np,
                                                          const unsigned* __restrict__ start,
                                                          void* __restrict__ mass_v) {
  using T = typename std::conditional<FIXED, unsigned long long, float>::type;
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << kTileLX, TY = 1 << kTileLY, TZ = 1 << tile_lz(LOGN);
  constexpr int WX = TX + 1, WY = TY + 1, WZ = TZ + 1;
  constexpr int NTY = N / TY, NTZ = N / TZ;
  __shared__ T acc[WX * WY * WZ];
  T* mass = static_cast<T*>(mass_v);
  const int t = blockIdx.x;
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kBlock) acc[c] = (T)0;
  __syncthreads();
  const unsigned lo = start[t], hi = start[t + 1];
  for (unsigned i = lo + threadIdx.x; i < hi; i += kBlock) {
    int ix, iy, iz;
    T w[8];
    if constexpr (FIXED) {
      const uint32_t* p = static_cast<const uint32_t*>(pos);
      fixed_weights<LOGN>(p[i], p[np + i], p[2 * np + i], ix, iy, iz, w);
    } else {
      const float* p = static_cast<const float*>(pos);
      float_weights<LOGN>(p[i], p[np + i], p[2 * np + i], ix, iy, iz, w);
    }
    const int rx = (ix - ox) & MASK, ry = (iy - oy) & MASK, rz = (iz - oz) & MASK;
    if (rx < TX && ry < TY && rz < TZ) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        atomicAdd(&acc[((rx + (c >> 2)) * WY + ry + ((c >> 1) & 1)) * WZ + rz + (c & 1)], w[c]);
    } else {
      deposit_global<LOGN>(mass, ix, iy, iz, w);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kBlock) {
    const T v = acc[c];
    if (v != (T)0) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t cell = ((size_t)((ox + lx) & MASK) * N + ((oy + ly) & MASK)) * N +
                          ((oz + lz) & MASK);
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
                                unsigned long long* mass, hipStream_t s) {
  const unsigned g = grid_for(np);
#define L_(LN)                                                                           \
  hipLaunchKernelGGL(k_deposit_fixed<LN>, dim3(g), dim3(kBlock), 0, s, pos, pos + np, \
                     pos + 2 * np, np, mass)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_fixed_tiled(const uint32_t* pos, int64_t np, int logn,
                                      const unsigned* start, unsigned long long* mass,
                                      hipStream_t s) {
  const dim3 g((unsigned)tile_count(logn));
#define L_(LN) \
  hipLaunchKernelGGL((k_deposit_tiled<LN, true>), g, dim3(kBlock), 0, s, pos, np, start, mass)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_f32_tiled(const float* pos, int64_t np, int logn,
                                    const unsigned* start, float* acc, hipStream_t s) {
  const dim3 g((unsigned)tile_count(logn));
#define L_(LN) \
  hipLaunchKernelGGL((k_deposit_tiled<LN, false>), g, dim3(kBlock), 0, s, pos, np, start, acc)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_deposit_f32(const float* pos, int64_t np, int logn, float* acc,
                              hipStream_t s) {
  const unsigned g = grid_for(np);
#define L_(LN)                                                                           \
  hipLaunchKernelGGL(k_deposit_f32<LN>, dim3(g), dim3(kBlock), 0, s, pos, pos + np, \
                     pos + 2 * np, np, acc)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace fdm
