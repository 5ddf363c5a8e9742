// Grid diagnostics of a particle state (not on the step path):
//  * the bulk velocity field of Sec. II B, Eq. (17): node sums of the
//    kernel-weighted particle momenta, one Cartesian component per pass, and
//    the per-node |P|^2 / M that gives the kinetic energy of the bulk motion;
//  * the RMS relative density difference per node of two states (Sec. III,
//    the FDM run against the CDM run from the same initial conditions).
// Sums are FP64: node momenta through FP64 atomics (rounding order varies
// from run to run at the 1e-16 level), reductions in a fixed order.
#include "cic.h"

namespace fdm {

namespace {

__device__ __forceinline__ double wave_block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Node mass in particle units from the deposit's mesh.
template <bool FIXED>
__device__ __forceinline__ double node_mass(const void* __restrict__ mass, int64_t i) {
  if constexpr (FIXED)
    return (double)static_cast<const long long*>(mass)[i] * 0x1p-40;
  else
    return (double)static_cast<const float*>(mass)[i];
}

// mom[node] += W(node - q_i) * v_i for one velocity component v.  The
// weights are the mass deposit's own (integer 2^-40 units or float), so a
// node's momentum and mass sums use the same kernel values.
template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_deposit_momentum(const void* __restrict__ pos,
                                                             int64_t np,
                                                             const float* __restrict__ v,
                                                             double* __restrict__ mom) {
  static_assert(kMassShift == 40, "node_mass and the weights below assume 2^40 units");
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ix, iy, iz;
    double w[8];
    if constexpr (FIXED) {
      const uint32_t* u = static_cast<const uint32_t*>(pos);
      unsigned long long wi[8];
      fixed_weights<LOGN>(u[p], u[np + p], u[2 * np + p], ix, iy, iz, wi);
#pragma unroll
      for (int c = 0; c < 8; ++c) w[c] = (double)wi[c] * 0x1p-40;
    } else {
      const float* x = static_cast<const float*>(pos);
      float wf[8];
      float_weights<LOGN>(x[p], x[np + p], x[2 * np + p], ix, iy, iz, wf);
#pragma unroll
      for (int c = 0; c < 8; ++c) w[c] = (double)wf[c];
    }
    const double vp = (double)v[p];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = (ix + (c >> 2)) & MASK;
      const int cy = (iy + ((c >> 1) & 1)) & MASK;
      const int cz = (iz + (c & 1)) & MASK;
      if (w[c] != 0.0) unsafeAtomicAdd(&mom[((size_t)cx * N + cy) * N + cz], w[c] * vp);
    }
  }
}

// Tiled form for a sorted context: one block per chunk of a tile sums its
// particles' momenta into an FP64 LDS window (the tile plus the faces CIC
// reaches and the deposit halo), then adds the window's non-zero nodes to the
// mesh; particles outside the window add to the mesh directly.  Same-node
// additions of a dense clump then meet in LDS instead of in L2.
template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_deposit_momentum_tiled(const void* __restrict__ pos,
                                                                   int64_t np,
                                                                   const float* __restrict__ v,
                                                                   TileMap tm,
                                                                   double* __restrict__ mom) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << tile_lx(LOGN), TY = 1 << tile_ly(LOGN), TZ = 1 << tile_lz(LOGN);
  constexpr int HD = kDepHalo;
  constexpr int WX = TX + 1 + 2 * HD, WY = TY + 1 + 2 * HD, WZ = TZ + 1 + 2 * HD;
  constexpr int NTY = N / TY, NTZ = N / TZ;
  __shared__ double acc[WX * WY * WZ];
  int t;
  unsigned lo, hi;
  if (!chunk_of(tm, t, lo, hi)) return;
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kBlock) acc[c] = 0.0;
  __syncthreads();
  for (unsigned i = lo + threadIdx.x; i < hi; i += kBlock) {
    int ix, iy, iz;
    double w[8];
    if constexpr (FIXED) {
      const uint32_t* u = static_cast<const uint32_t*>(pos);
      unsigned long long wi[8];
      fixed_weights<LOGN>(u[i], u[np + i], u[2 * np + i], ix, iy, iz, wi);
#pragma unroll
      for (int c = 0; c < 8; ++c) w[c] = (double)wi[c] * 0x1p-40;
    } else {
      const float* x = static_cast<const float*>(pos);
      float wf[8];
      float_weights<LOGN>(x[i], x[np + i], x[2 * np + i], ix, iy, iz, wf);
#pragma unroll
      for (int c = 0; c < 8; ++c) w[c] = (double)wf[c];
    }
    const double vp = (double)v[i];
    const int rx = (ix - ox + HD) & MASK, ry = (iy - oy + HD) & MASK, rz = (iz - oz + HD) & MASK;
    if (rx < TX + 2 * HD && ry < TY + 2 * HD && rz < TZ + 2 * HD) {
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (w[c] != 0.0)
          unsafeAtomicAdd(&acc[((rx + (c >> 2)) * WY + ry + ((c >> 1) & 1)) * WZ + rz + (c & 1)],
                          w[c] * vp);
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int cx = (ix + (c >> 2)) & MASK;
        const int cy = (iy + ((c >> 1) & 1)) & MASK;
        const int cz = (iz + (c & 1)) & MASK;
        if (w[c] != 0.0) unsafeAtomicAdd(&mom[((size_t)cx * N + cy) * N + cz], w[c] * vp);
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kBlock) {
    const double a = acc[c];
    if (a != 0.0) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t cell = ((size_t)((ox - HD + lx) & MASK) * N + ((oy - HD + ly) & MASK)) * N +
                          ((oz - HD + lz) & MASK);
      unsafeAtomicAdd(&mom[cell], a);
    }
  }
}

// partials[b] = sum over this block's nodes with mass of mom^2 / mass.
template <bool FIXED>
__global__ void __launch_bounds__(kBlock) k_bulk_nodes(const void* __restrict__ mass,
                                                       const double* __restrict__ mom,
                                                       int64_t ncell,
                                                       double* __restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double t = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += stride) {
    const double m = node_mass<FIXED>(mass, i);
    if (m > 0.0) {
      const double pm = mom[i];
      t += pm * pm / m;
    }
  }
  t = wave_block_sum(t, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// partials[2b], [2b+1] = sum of ((a - b) / b)^2 and the count of nodes with
// b > 0.  In the fixed-point form the difference is taken on the exact
// integer masses before the one rounding to double.
template <bool FIXED>
__global__ void __launch_bounds__(kBlock) k_rel_diff_nodes(const void* __restrict__ mass_a,
                                                           const void* __restrict__ mass_b,
                                                           int64_t ncell,
                                                           double* __restrict__ partials) {
  __shared__ double red[kBlock / 64];
  double t = 0.0, cnt = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell; i += stride) {
    double r = 0.0;
    bool has = false;
    if constexpr (FIXED) {
      const long long b = static_cast<const long long*>(mass_b)[i];
      if (b > 0) {
        const long long a = static_cast<const long long*>(mass_a)[i];
        r = (double)(a - b) / (double)b;
        has = true;
      }
    } else {
      const double b = (double)static_cast<const float*>(mass_b)[i];
      if (b > 0.0) {
        r = ((double)static_cast<const float*>(mass_a)[i] - b) / b;
        has = true;
      }
    }
    if (has) {
      t += r * r;
      cnt += 1.0;
    }
  }
  t = wave_block_sum(t, red);
  cnt = wave_block_sum(cnt, red);
  if (threadIdx.x == 0) {
    partials[2 * (size_t)blockIdx.x] = t;
    partials[2 * (size_t)blockIdx.x + 1] = cnt;
  }
}

}  // namespace

int diag_blocks(int64_t n, int max_blocks) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > max_blocks) b = max_blocks;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_deposit_momentum(bool fixed, int logn, const void* pos, int64_t np,
                                   const float* v, double* mom, const TileMap* tm,
                                   hipStream_t s) {
  if (tm) {
    const dim3 g(tiled_grid(np, tm->tiles));
#define L_(LN)                                                                                \
  if (fixed)                                                                                  \
    hipLaunchKernelGGL((k_deposit_momentum_tiled<LN, true>), g, dim3(kBlock), 0, s, pos, np, v, \
                       *tm, mom);                                                             \
  else                                                                                        \
    hipLaunchKernelGGL((k_deposit_momentum_tiled<LN, false>), g, dim3(kBlock), 0, s, pos, np,   \
                       v, *tm, mom);
    FDM_LOGN_SWITCH(logn, L_)
#undef L_
    return hipGetLastError();
  }
  const unsigned g = (unsigned)diag_blocks(np, 65536);
#define L_(LN)                                                                              \
  if (fixed)                                                                                \
    hipLaunchKernelGGL((k_deposit_momentum<LN, true>), dim3(g), dim3(kBlock), 0, s, pos, np, v, \
                       mom);                                                                \
  else                                                                                      \
    hipLaunchKernelGGL((k_deposit_momentum<LN, false>), dim3(g), dim3(kBlock), 0, s, pos, np, \
                       v, mom);
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_bulk_nodes(bool fixed, const void* mass, const double* mom, int64_t ncell,
                             double* partials, int nblocks, hipStream_t s) {
  if (fixed)
    hipLaunchKernelGGL(k_bulk_nodes<true>, dim3(nblocks), dim3(kBlock), 0, s, mass, mom, ncell,
                       partials);
  else
    hipLaunchKernelGGL(k_bulk_nodes<false>, dim3(nblocks), dim3(kBlock), 0, s, mass, mom, ncell,
                       partials);
  return hipGetLastError();
}

hipError_t launch_rel_diff_nodes(bool fixed, const void* mass_a, const void* mass_b,
                                 int64_t ncell, double* partials, int nblocks, hipStream_t s) {
  if (fixed)
    hipLaunchKernelGGL(k_rel_diff_nodes<true>, dim3(nblocks), dim3(kBlock), 0, s, mass_a, mass_b,
                       ncell, partials);
  else
    hipLaunchKernelGGL(k_rel_diff_nodes<false>, dim3(nblocks), dim3(kBlock), 0, s, mass_a,
                       mass_b, ncell, partials);
  return hipGetLastError();
}

}  // namespace fdm
