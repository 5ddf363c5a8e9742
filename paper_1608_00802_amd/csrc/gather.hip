// Force interpolation and particle push, step (iii) of Sec. II A in the
// mesh-gradient form: the acceleration -grad(phi + Q) is taken by central
// differences on the mesh and interpolated to each particle with the same
// trilinear (CIC) weights as the deposit, then the leapfrog kick (and drift)
// are applied in the same pass.
//
// The kick factors multiply the two potentials before the gradient
// (F = fg*phi + fq*Q), since gradient and interpolation are linear.  For one
// particle the central differences at its 8 CIC nodes need F on 32 nodes:
// the 2x2x2 core plus two extra planes along each axis.
//
// Drift (fixed-point form): u += rint(p * F_d * 2^B) in 64-bit integers, then
// truncated to 32 bits, which is the periodic wrap done exactly.
#include "internal.h"

namespace fdm {

enum GatherMode : int { kKick = 0, kKickDrift = 1, kForce = 2 };

template <int LOGN, bool FIXED, bool HAS_Q, int MODE>
__global__ void __launch_bounds__(kBlock) k_gather(void* __restrict__ pos,
                                                   float* __restrict__ vel,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ q, int64_t np,
                                                   GatherConst gc, float* __restrict__ acc) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int B = 32 - LOGN;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ic[3];
    float f[3];
    uint32_t u[3];
    float xf[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if constexpr (FIXED) {
        u[d] = static_cast<const uint32_t*>(pos)[d * np + p];
        ic[d] = (int)(u[d] >> B);
        f[d] = (float)(u[d] & ((1u << B) - 1u)) * (1.0f / (float)(1u << B));
      } else {
        xf[d] = static_cast<const float*>(pos)[d * np + p];
        const float fl = floorf(xf[d]);
        f[d] = xf[d] - fl;
        ic[d] = (int)fl & MASK;
      }
    }
    int ix[4], iy[4], iz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ix[k] = (ic[0] + k - 1) & MASK;
      iy[k] = (ic[1] + k - 1) & MASK;
      iz[k] = (ic[2] + k - 1) & MASK;
    }
    auto at = [&](int a, int b, int c) -> float {
      const size_t idx = ((size_t)a * N + b) * N + c;
      float v = gc.fg * phi[idx];
      if constexpr (HAS_Q) v += gc.fq * q[idx];
      return v;
    };
    // fx4[a][b][c]: x = ix[a] (a = 0..3), y = iy[1 + b], z = iz[1 + c]
    float fx4[4][2][2];
    // fy2[a][b][c]: x = ix[1 + a], y = iy[0] (b = 0) or iy[3] (b = 1), z = iz[1 + c]
    float fy2[2][2][2];
    // fz2[a][b][c]: x = ix[1 + a], y = iy[1 + b], z = iz[0] (c = 0) or iz[3] (c = 1)
    float fz2[2][2][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) fx4[a][b][c] = at(ix[a], iy[1 + b], iz[1 + c]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          fy2[a][b][c] = at(ix[1 + a], iy[3 * b], iz[1 + c]);
          fz2[a][b][c] = at(ix[1 + a], iy[1 + b], iz[3 * c]);
        }
    const float wx[2] = {1.0f - f[0], f[0]};
    const float wy[2] = {1.0f - f[1], f[1]};
    const float wz[2] = {1.0f - f[2], f[2]};
    // F on the 4-point line through each core node along each axis
    auto fyl = [&](int a, int j, int c) -> float {  // x = ix[1+a], y = iy[j], z = iz[1+c]
      return j == 0 ? fy2[a][0][c] : (j == 3 ? fy2[a][1][c] : fx4[1 + a][j - 1][c]);
    };
    auto fzl = [&](int a, int b, int k) -> float {  // x = ix[1+a], y = iy[1+b], z = iz[k]
      return k == 0 ? fz2[a][b][0] : (k == 3 ? fz2[a][b][1] : fx4[1 + a][b][k - 1]);
    };
    float g[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float w = wy[b] * wz[c];
        g[0] += w * (wx[0] * (fx4[2][b][c] - fx4[0][b][c]) + wx[1] * (fx4[3][b][c] - fx4[1][b][c]));
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float w = wx[a] * wz[c];
        g[1] += w * (wy[0] * (fyl(a, 2, c) - fyl(a, 0, c)) + wy[1] * (fyl(a, 3, c) - fyl(a, 1, c)));
      }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const float w = wx[a] * wy[b];
        g[2] += w * (wz[0] * (fzl(a, b, 2) - fzl(a, b, 0)) + wz[1] * (fzl(a, b, 3) - fzl(a, b, 1)));
      }
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] *= -0.5f;
    if constexpr (MODE == kForce) {
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[d * np + p] = g[d];
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float v = vel[d * np + p] + g[d];
        vel[d * np + p] = v;
        if constexpr (MODE == kKickDrift) {
          if constexpr (FIXED) {
            const long long inc = __double2ll_rn((double)v * gc.fd_units);
            static_cast<uint32_t*>(pos)[d * np + p] = u[d] + (uint32_t)(unsigned long long)inc;
          } else {
            float x = xf[d] + v * (float)gc.fd_units;
            x = x - (float)N * floorf(x * (1.0f / (float)N));
            if (x >= (float)N) x = 0.0f;
            static_cast<float*>(pos)[d * np + p] = x;
          }
        }
      }
    }
  }
}

static unsigned grid_particles(int64_t np) {
  int64_t b = (np + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <int LN, int MODE>
static void launch_mode(bool fixed, bool has_q, dim3 g, hipStream_t s, void* pos, float* vel,
                        const float* phi, const float* q, int64_t np, const GatherConst& gc,
                        float* acc) {
  if (fixed && has_q)
    hipLaunchKernelGGL((k_gather<LN, true, true, MODE>), g, dim3(kBlock), 0, s, pos, vel, phi, q,
                       np, gc, acc);
  else if (fixed)
    hipLaunchKernelGGL((k_gather<LN, true, false, MODE>), g, dim3(kBlock), 0, s, pos, vel, phi,
                       q, np, gc, acc);
  else if (has_q)
    hipLaunchKernelGGL((k_gather<LN, false, true, MODE>), g, dim3(kBlock), 0, s, pos, vel, phi,
                       q, np, gc, acc);
  else
    hipLaunchKernelGGL((k_gather<LN, false, false, MODE>), g, dim3(kBlock), 0, s, pos, vel, phi,
                       q, np, gc, acc);
}

hipError_t launch_gather(bool fixed, bool has_q, bool drift, int logn, void* pos, float* vel,
                         const float* phi, const float* q, int64_t np, const GatherConst& gc,
                         hipStream_t s) {
  const dim3 g(grid_particles(np));
#define L_(LN)                                                                           \
  {                                                                                      \
    if (drift)                                                                           \
      launch_mode<LN, kKickDrift>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr); \
    else                                                                                 \
      launch_mode<LN, kKick>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr);      \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_force(bool fixed, bool has_q, int logn, const void* pos, const float* phi,
                        const float* q, int64_t np, float fg, float fq, float* acc,
                        hipStream_t s) {
  const dim3 g(grid_particles(np));
  GatherConst gc;
  gc.fg = fg;
  gc.fq = fq;
  gc.fd_units = 0.0;
#define L_(LN)                                                                           \
  launch_mode<LN, kForce>(fixed, has_q, g, s, const_cast<void*>(pos), nullptr, phi, q, np, \
                          gc, acc)
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

// FP64 partial sums of |v|^2 per block.
__global__ void __launch_bounds__(kBlock) k_kinetic(const float* __restrict__ vel, int64_t np,
                                                    double* __restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double t = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    const double vx = vel[p], vy = vel[np + p], vz = vel[2 * np + p];
    t += vx * vx + vy * vy + vz * vz;
  }
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    partials[blockIdx.x] = s;
  }
}

int kinetic_blocks(int64_t np) {
  int64_t b = (np + kBlock - 1) / kBlock;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_kinetic(const float* vel, int64_t np, double* partials, int nblocks,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic, dim3(nblocks), dim3(kBlock), 0, s, vel, np, partials);
  return hipGetLastError();
}

}  // namespace fdm
