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

template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_deposit_fixed(const uint32_t* __restrict__ px,
                                                          const uint32_t* __restrict__ py,
                                                          const uint32_t* __restrict__ pz,
                                                          int64_t np,
                                                          unsigned long long* __restrict__ mass) {
  constexpr int N = 1 << LOGN;
  constexpr uint32_t MASK = N - 1;
  constexpr int B = 32 - LOGN;
  constexpr unsigned long long ONE = 1ull << B;
  // 2^(40 - 3B), exact
  const double scale = ldexp(1.0, kMassShift - 3 * B);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const uint32_t ux = px[i], uy = py[i], uz = pz[i];
    const uint32_t ix = ux >> B, iy = uy >> B, iz = uz >> B;
    const unsigned long long fx = ux & (ONE - 1), fy = uy & (ONE - 1), fz = uz & (ONE - 1);
    const unsigned long long wx[2] = {ONE - fx, fx};
    const unsigned long long wy[2] = {ONE - fy, fy};
    const unsigned long long wz[2] = {ONE - fz, fz};
    const int big = ((fx >= (ONE >> 1)) << 2) | ((fy >= (ONE >> 1)) << 1) | (fz >= (ONE >> 1));
    unsigned long long w[8];
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
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint32_t cx = (ix + (c >> 2)) & MASK;
      const uint32_t cy = (iy + ((c >> 1) & 1)) & MASK;
      const uint32_t cz = (iz + (c & 1)) & MASK;
      const size_t cell = ((size_t)cx * N + cy) * N + cz;
      if (w[c] != 0ull) atomicAdd(&mass[cell], w[c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_deposit_f32(const float* __restrict__ px,
                                                        const float* __restrict__ py,
                                                        const float* __restrict__ pz,
                                                        int64_t np, float* __restrict__ acc) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += stride) {
    const float x = px[i], y = py[i], z = pz[i];
    const float flx = floorf(x), fly = floorf(y), flz = floorf(z);
    const float fx = x - flx, fy = y - fly, fz = z - flz;
    const int ix = (int)flx & MASK, iy = (int)fly & MASK, iz = (int)flz & MASK;
    const float wx[2] = {1.0f - fx, fx}, wy[2] = {1.0f - fy, fy}, wz[2] = {1.0f - fz, fz};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = (ix + (c >> 2)) & MASK;
      const int cy = (iy + ((c >> 1) & 1)) & MASK;
      const int cz = (iz + (c & 1)) & MASK;
      const float w = wx[c >> 2] * wy[(c >> 1) & 1] * wz[c & 1];
      unsafeAtomicAdd(&acc[((size_t)cx * N + cy) * N + cz], w);
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
