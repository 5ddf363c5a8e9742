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

// Position of particle p: integer cell and fraction along each axis.
template <int LOGN, bool FIXED>
__device__ __forceinline__ void load_cell(const void* __restrict__ pos, int64_t np, int64_t p,
                                          int ic[3], float f[3], uint32_t u[3], float xf[3]) {
  constexpr int MASK = (1 << LOGN) - 1;
  constexpr int B = 32 - LOGN;
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
}

// Interpolated -grad F at one particle.  at(a, b, c) returns F at offsets
// (a - 1, b - 1, c - 1) from the particle's base cell, a, b, c in 0..3.
template <typename At>
__device__ __forceinline__ void interp_grad(const float f[3], At&& at, float g[3]) {
  // fx4[a][b][c]: x offset a (0..3), y offset 1 + b, z offset 1 + c
  float fx4[4][2][2];
  // fy2[a][b][c]: x offset 1 + a, y offset 0 (b = 0) or 3 (b = 1), z offset 1 + c
  float fy2[2][2][2];
  // fz2[a][b][c]: x offset 1 + a, y offset 1 + b, z offset 0 (c = 0) or 3 (c = 1)
  float fz2[2][2][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) fx4[a][b][c] = at(a, 1 + b, 1 + c);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        fy2[a][b][c] = at(1 + a, 3 * b, 1 + c);
        fz2[a][b][c] = at(1 + a, 1 + b, 3 * c);
      }
  const float wx[2] = {1.0f - f[0], f[0]};
  const float wy[2] = {1.0f - f[1], f[1]};
  const float wz[2] = {1.0f - f[2], f[2]};
  auto fyl = [&](int a, int j, int c) -> float {  // x offset 1+a, y offset j, z offset 1+c
    return j == 0 ? fy2[a][0][c] : (j == 3 ? fy2[a][1][c] : fx4[1 + a][j - 1][c]);
  };
  auto fzl = [&](int a, int b, int k) -> float {  // x offset 1+a, y offset 1+b, z offset k
    return k == 0 ? fz2[a][b][0] : (k == 3 ? fz2[a][b][1] : fx4[1 + a][b][k - 1]);
  };
  g[0] = g[1] = g[2] = 0.0f;
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
}

// Apply the result for particle p: store the force, or kick (and drift).
template <int LOGN, bool FIXED, int MODE>
__device__ __forceinline__ void push(void* __restrict__ pos, float* __restrict__ vel,
                                     float* __restrict__ acc, int64_t np, int64_t p,
                                     const float g[3], const uint32_t u[3], const float xf[3],
                                     double fd_units) {
  constexpr int N = 1 << LOGN;
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
          const long long inc = __double2ll_rn((double)v * fd_units);
          static_cast<uint32_t*>(pos)[d * np + p] = u[d] + (uint32_t)(unsigned long long)inc;
        } else {
          float x = xf[d] + v * (float)fd_units;
          x = x - (float)N * floorf(x * (1.0f / (float)N));
          if (x >= (float)N) x = 0.0f;
          static_cast<float*>(pos)[d * np + p] = x;
        }
      }
    }
  }
}

template <int LOGN, bool HAS_Q>
__device__ __forceinline__ float mesh_f(const float* __restrict__ phi, const float* __restrict__ q,
                                        const GatherConst& gc, size_t idx) {
  float v = gc.fg * phi[idx];
  if constexpr (HAS_Q) v += gc.fq * q[idx];
  return v;
}

template <int LOGN, bool FIXED, bool HAS_Q, int MODE>
__global__ void __launch_bounds__(kBlock) k_gather(void* __restrict__ pos,
                                                   float* __restrict__ vel,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ q, int64_t np,
                                                   GatherConst gc, float* __restrict__ acc) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ic[3];
    float f[3], xf[3];
    uint32_t u[3];
    load_cell<LOGN, FIXED>(pos, np, p, ic, f, u, xf);
    float g[3];
    interp_grad(f, [&](int a, int b, int c) {
      const size_t idx = ((size_t)((ic[0] + a - 1) & MASK) * N + ((ic[1] + b - 1) & MASK)) * N +
                         ((ic[2] + c - 1) & MASK);
      return mesh_f<LOGN, HAS_Q>(phi, q, gc, idx);
    }, g);
    push<LOGN, FIXED, MODE>(pos, vel, acc, np, p, g, u, xf, gc.fd_units);
  }
}

// Tiled gather: block b owns tile b of the particle sort.  F = fg phi + fq Q
// is staged once for the tile's window (cells -1 .. T+1 around the tile) in
// LDS; particles still inside their tile read their 32 nodes from LDS,
// particles that left it read the mesh directly.
template <int LOGN, bool FIXED, bool HAS_Q, int MODE>
__global__ void __launch_bounds__(kBlock) k_gather_tiled(void* __restrict__ pos,
                                                         float* __restrict__ vel,
                                                         const float* __restrict__ phi,
                                                         const float* __restrict__ q, int64_t np,
                                                         const unsigned* __restrict__ start,
                                                         GatherConst gc,
                                                         float* __restrict__ acc) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << kTileLX, TY = 1 << kTileLY, TZ = 1 << tile_lz(LOGN);
  constexpr int WX = TX + 3, WY = TY + 3, WZ = TZ + 3;
  constexpr int NTY = N / TY, NTZ = N / TZ;
  __shared__ float win[WX * WY * WZ];
  const int t = blockIdx.x;
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kBlock) {
    const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
    const size_t idx = ((size_t)((ox - 1 + lx) & MASK) * N + ((oy - 1 + ly) & MASK)) * N +
                       ((oz - 1 + lz) & MASK);
    win[c] = mesh_f<LOGN, HAS_Q>(phi, q, gc, idx);
  }
  __syncthreads();
  const unsigned lo = start[t], hi = start[t + 1];
  for (unsigned p = lo + threadIdx.x; p < hi; p += kBlock) {
    int ic[3];
    float f[3], xf[3];
    uint32_t u[3];
    load_cell<LOGN, FIXED>(pos, np, p, ic, f, u, xf);
    const int rx = (ic[0] - ox) & MASK, ry = (ic[1] - oy) & MASK, rz = (ic[2] - oz) & MASK;
    float g[3];
    if (rx < TX && ry < TY && rz < TZ) {
      interp_grad(f, [&](int a, int b, int c) {
        return win[((rx + a) * WY + ry + b) * WZ + rz + c];
      }, g);
    } else {
      interp_grad(f, [&](int a, int b, int c) {
        const size_t idx = ((size_t)((ic[0] + a - 1) & MASK) * N + ((ic[1] + b - 1) & MASK)) * N +
                           ((ic[2] + c - 1) & MASK);
        return mesh_f<LOGN, HAS_Q>(phi, q, gc, idx);
      }, g);
    }
    push<LOGN, FIXED, MODE>(pos, vel, acc, np, p, g, u, xf, gc.fd_units);
  }
}

static unsigned grid_particles(int64_t np) {
  int64_t b = (np + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <int LN, int MODE>
static void launch_mode_tiled(bool fixed, bool has_q, hipStream_t s, void* pos, float* vel,
                              const float* phi, const float* q, int64_t np,
                              const unsigned* start, const GatherConst& gc, float* acc) {
  const dim3 g((unsigned)tile_count(LN));
  if (fixed && has_q)
    hipLaunchKernelGGL((k_gather_tiled<LN, true, true, MODE>), g, dim3(kBlock), 0, s, pos, vel,
                       phi, q, np, start, gc, acc);
  else if (fixed)
    hipLaunchKernelGGL((k_gather_tiled<LN, true, false, MODE>), g, dim3(kBlock), 0, s, pos, vel,
                       phi, q, np, start, gc, acc);
  else if (has_q)
    hipLaunchKernelGGL((k_gather_tiled<LN, false, true, MODE>), g, dim3(kBlock), 0, s, pos, vel,
                       phi, q, np, start, gc, acc);
  else
    hipLaunchKernelGGL((k_gather_tiled<LN, false, false, MODE>), g, dim3(kBlock), 0, s, pos, vel,
                       phi, q, np, start, gc, acc);
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
                         const unsigned* tile_start, hipStream_t s) {
  const dim3 g(grid_particles(np));
#define L_(LN)                                                                               \
  {                                                                                          \
    if (tile_start && drift)                                                                 \
      launch_mode_tiled<LN, kKickDrift>(fixed, has_q, s, pos, vel, phi, q, np, tile_start, gc, \
                                        nullptr);                                            \
    else if (tile_start)                                                                     \
      launch_mode_tiled<LN, kKick>(fixed, has_q, s, pos, vel, phi, q, np, tile_start, gc,     \
                                   nullptr);                                                 \
    else if (drift)                                                                          \
      launch_mode<LN, kKickDrift>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr);     \
    else                                                                                     \
      launch_mode<LN, kKick>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr);          \
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
