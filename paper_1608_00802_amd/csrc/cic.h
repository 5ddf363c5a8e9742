// Cloud-in-cell weights and the direct (global-atomic) deposit of one
// particle, shared by the deposit kernels and the fused push-deposit.
#pragma once

#include "internal.h"

namespace fdm {

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

}  // namespace fdm
