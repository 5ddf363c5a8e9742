// Cloud-in-cell weights and the direct (global-atomic) deposit of one
// particle, shared by the deposit kernels and the fused push-deposit.
#pragma once

#include "internal.h"

namespace fdm {

// rint(a * b) for 0 <= a * b < 2^51 as an unsigned 64-bit integer: the
// product is rounded to double, then adding 2^52 (where doubles are one
// apart) rounds it to the nearest integer, ties to even, and leaves that
// integer in the low 52 bits.  Two roundings, as in rint(fl(a * b)): the
// multiply and the add must not be contracted into one fma.
__device__ __forceinline__ unsigned long long rint_mul_u64(double a, double b) {
#pragma clang fp contract(off)
  const double t = a * b;
  const double r = t + 0x1p52;
  return (unsigned long long)__double_as_longlong(r) & 0x000FFFFFFFFFFFFFull;
}

// Cell index and fraction (an integer below 2^B) of one fixed-point
// coordinate, and whether the upper cell takes the larger weight.
template <int LOGN>
__device__ __forceinline__ void axis_weights(uint32_t u, int& i, uint32_t& f, bool& up) {
  constexpr int B = 32 - LOGN;
  constexpr uint32_t ONE = 1u << B;
  i = (int)(u >> B);
  f = u & (ONE - 1u);
  up = f >= (ONE >> 1);
}

// Cell index, the eight rounded corner weights of one fixed-point particle
// in 2^40 units per particle (corner c = 4 cx + 2 cy + cz) before the
// remainder, the heaviest corner `big` and the remainder d = 2^40 - sum of
// the eight, which `big` takes so that the particle deposits exactly 2^40.
// Each weight is rint(fl(fl(wx wy) wz) 2^(40 - 3B)) of the per-axis integer
// weights (below 2^B, B = 32 - log2 N): wx wy is one rounding of the exact
// product (exact for B <= 26), and the power-of-two scale is folded into
// wz.  Each weight is within 1/2 + 2^-12 of its exact value and the exact
// values sum to 2^40, so |d| <= 4: its low 32 bits carry it.
template <int LOGN>
__device__ __forceinline__ void fixed_weights_split(uint32_t ux, uint32_t uy, uint32_t uz,
                                                    int& ix, int& iy, int& iz,
                                                    unsigned long long w[8], int& big, int& d) {
  constexpr int B = 32 - LOGN;
  constexpr uint32_t ONE = 1u << B;
  constexpr double SCALE = 1.0 / (double)(1ull << (3 * B - kMassShift));  // 2^(40 - 3B)
  uint32_t fx, fy, fz;
  bool bx, by, bz;
  axis_weights<LOGN>(ux, ix, fx, bx);
  axis_weights<LOGN>(uy, iy, fy, by);
  axis_weights<LOGN>(uz, iz, fz, bz);
  const double wx[2] = {(double)(ONE - fx), (double)fx};
  const double wy[2] = {(double)(ONE - fy), (double)fy};
  const double wz[2] = {(double)(ONE - fz) * SCALE, (double)fz * SCALE};
  big = (bx << 2) | (by << 1) | (int)bz;
  uint32_t low = 0;   // 2^40 = 0 modulo 2^32
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    w[c] = rint_mul_u64(wx[c >> 2] * wy[(c >> 1) & 1], wz[c & 1]);
    low -= (uint32_t)w[c];
  }
  d = (int)low;
}

// The eight corner weights with the remainder applied (corner c = 4 cx +
// 2 cy + cz): exactly 2^40 per particle.
template <int LOGN>
__device__ __forceinline__ void fixed_weights(uint32_t ux, uint32_t uy, uint32_t uz, int& ix,
                                              int& iy, int& iz, unsigned long long w[8]) {
  int big, d;
  fixed_weights_split<LOGN>(ux, uy, uz, ix, iy, iz, w, big, d);
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (c == big) w[c] += (unsigned long long)(long long)d;
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
