// The paper's own particle-mesh coupling (Sec. II A): density on the mesh
// nodes from the cubic spline kernel of Eq. (15) with smoothing length h,
// Eq. (9), and the quantum force on each particle by the kernel gradient,
// Eq. (14): a_i = dx^3 sum_j Q_j grad W(x_j - q_i) (dx = 1 in cell units; the
// sign makes a = -grad Q, the particle derivative of the discrete K_rho).
// Every node within h of a particle is visited: for h = 3.5 cells a cube of
// 8^3 candidate nodes, about 180 of them inside the support.
//
// The density is summed in integers: each kernel value W (per unit particle
// mass, cells^-3, at most 8 / (pi h^3)) is rounded once to a multiple of 2^-40
// and added as an unsigned 64-bit integer, in the units of the
// cloud-in-cell deposit (one particle = 2^40), into the context's mass mesh.
// Integer sums commute, so the mesh is bitwise independent of particle order
// and scheduling (tiled or direct, run to run), the density contrast is
// formed from it by the exact subtraction of the mean (the forward z pass),
// and near-empty nodes keep their full relative precision (no sum starting
// from -1), which is what the FP64 path of the Q stencil reads there.
#include "internal.h"

namespace fdm {

namespace {

// Cell index and fractional offset in [0, 1) of one coordinate.
template <int LOGN, bool FIXED>
__device__ __forceinline__ void cell_frac(const void* pos, int64_t at, int& i, float& f) {
  if constexpr (FIXED) {
    constexpr int B = 32 - LOGN;
    const uint32_t u = static_cast<const uint32_t*>(pos)[at];
    i = (int)(u >> B);
    f = (float)(u & ((1u << B) - 1u)) * (1.0f / (float)(1u << B));
  } else {
    constexpr int MASK = (1 << LOGN) - 1;
    const float x = static_cast<const float*>(pos)[at];
    const float fl = floorf(x);
    i = (int)fl & MASK;
    f = x - fl;
  }
}

// W(r) / c and dW/dr / c' of Eq. (15) for q = r / h <= 1 (c = 8 / (pi h^3),
// c' = c / h).
__device__ __forceinline__ float spline_shape(float q) {
  if (q <= 0.5f) return 1.0f - 6.0f * q * q + 6.0f * q * q * q;
  const float t = 1.0f - q;
  return 2.0f * t * t * t;
}
__device__ __forceinline__ float spline_slope(float q) {
  if (q <= 0.5f) return -12.0f * q + 18.0f * q * q;
  const float t = 1.0f - q;
  return -6.0f * t * t;
}

// r from r^2 through the hardware reciprocal square root (about 1 ulp; its
// argument held normal, and r = 0 for r^2 = 0).
__device__ __forceinline__ float spline_r(float r2) {
  return r2 * __builtin_amdgcn_rsqf(fmaxf(r2, 0x1p-100f));
}

// Offsets o in [lo, hi] along one axis that may satisfy (o - f)^2 <= rem,
// rem being h^2 less the other axes' squared distances: the integers in
// [f - sqrt(rem), f + sqrt(rem)], widened to the enclosing integers, so that
// any error of the square root below one cell never drops a node (the
// hardware square root, about 1 ulp); the exact test on r^2 inside the loops
// decides, so the nodes visited are those of the full cube.
__device__ __forceinline__ void axis_span(float f, float rem, int lo, int hi, int& a, int& b) {
  const float w = __builtin_amdgcn_sqrtf(fmaxf(rem, 0.0f));
  a = max(lo, (int)floorf(f - w));
  b = min(hi, (int)ceilf(f + w));
}

// Integer units of one kernel value w (cells^-3 per unit particle mass):
// rint(w 2^40), ties to even.  w 2^40 is exact in FP64 and below 2^39
// (w <= 8 / (pi h^3) < 1/2 for h >= 2); adding 2^52, where doubles are one
// apart, rounds it and leaves the integer in the low mantissa bits.
__device__ __forceinline__ unsigned long long spline_units(float w) {
#pragma clang fp contract(off)
  const double t = (double)w * 0x1p40;
  return (unsigned long long)__double_as_longlong(t + 0x1p52) & 0x000FFFFFFFFFFFFFull;
}

template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_spline_deposit(const void* __restrict__ pos,
                                                           int64_t np, float h, float inv_h,
                                                           float coef, int lo, int hi,
                                                           unsigned long long* __restrict__ mass) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const float h2 = h * h;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ix, iy, iz;
    float fx, fy, fz;
    cell_frac<LOGN, FIXED>(pos, p, ix, fx);
    cell_frac<LOGN, FIXED>(pos, np + p, iy, fy);
    cell_frac<LOGN, FIXED>(pos, 2 * np + p, iz, fz);
    for (int ox = lo; ox <= hi; ++ox) {
      const float dx = (float)ox - fx;
      const float dx2 = dx * dx;
      if (dx2 > h2) continue;
      const size_t rx = (size_t)((ix + ox) & MASK) * N;
      int y0, y1;
      axis_span(fy, h2 - dx2, lo, hi, y0, y1);
      for (int oy = y0; oy <= y1; ++oy) {
        const float dy = (float)oy - fy;
        const float dxy2 = dx2 + dy * dy;
        if (dxy2 > h2) continue;
        const size_t rxy = (rx + ((iy + oy) & MASK)) * N;
        int z0, z1;
        axis_span(fz, h2 - dxy2, lo, hi, z0, z1);
        for (int oz = z0; oz <= z1; ++oz) {
          const float dz = (float)oz - fz;
          const float r2 = dxy2 + dz * dz;
          if (r2 > h2) continue;
          const float q = spline_r(r2) * inv_h;
          atomicAdd(&mass[rxy + ((iz + oz) & MASK)], spline_units(coef * spline_shape(q)));
        }
      }
    }
  }
}

// Tiled form for a sorted context: one block per chunk of a tile sums the
// kernel values of its particles into an LDS window covering every node the
// tile's particles reach (offsets lo .. hi from the tile), then adds the
// window's non-zero nodes to the mesh; particles that left their tile add to
// the mesh directly.  Dense clumps then meet in LDS instead of in L2.  The
// window (64-bit integers) is sized at launch to the kernel's reach, up to
// kSplineReach cells on each side.
constexpr int kSplineReach = 5;
constexpr int kSplineBlock = 512;
template <int LOGN>
__host__ __device__ constexpr int spline_tile_nodes(int span) {
  return ((1 << tile_lx(LOGN)) + span) * ((1 << tile_ly(LOGN)) + span) *
         ((1 << tile_lz(LOGN)) + span);
}
template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kSplineBlock) k_spline_deposit_tiled(
    const void* __restrict__ pos, int64_t np, TileMap tm, float h, float inv_h, float coef,
    int lo, int hi, unsigned long long* __restrict__ mass) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << tile_lx(LOGN), TY = 1 << tile_ly(LOGN), TZ = 1 << tile_lz(LOGN);
  constexpr int NTY = N / TY, NTZ = N / TZ;
  extern __shared__ unsigned long long win[];
  int t;
  unsigned p0, p1;
  if (!chunk_of(tm, t, p0, p1)) return;
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  const int WX = TX + hi - lo, WY = TY + hi - lo, WZ = TZ + hi - lo;
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kSplineBlock) win[c] = 0ull;
  __syncthreads();
  const float h2 = h * h;
  for (unsigned p = p0 + threadIdx.x; p < p1; p += kSplineBlock) {
    int ix, iy, iz;
    float fx, fy, fz;
    cell_frac<LOGN, FIXED>(pos, p, ix, fx);
    cell_frac<LOGN, FIXED>(pos, np + p, iy, fy);
    cell_frac<LOGN, FIXED>(pos, 2 * np + p, iz, fz);
    const int rx = (ix - ox) & MASK, ry = (iy - oy) & MASK, rz = (iz - oz) & MASK;
    const bool inside = rx < TX && ry < TY && rz < TZ;
    for (int a = lo; a <= hi; ++a) {
      const float dx = (float)a - fx;
      const float dx2 = dx * dx;
      if (dx2 > h2) continue;
      int b0, b1;
      axis_span(fy, h2 - dx2, lo, hi, b0, b1);
      for (int b = b0; b <= b1; ++b) {
        const float dy = (float)b - fy;
        const float dxy2 = dx2 + dy * dy;
        if (dxy2 > h2) continue;
        int c0, c1;
        axis_span(fz, h2 - dxy2, lo, hi, c0, c1);
        for (int c = c0; c <= c1; ++c) {
          const float dz = (float)c - fz;
          const float r2 = dxy2 + dz * dz;
          if (r2 > h2) continue;
          const unsigned long long w = spline_units(coef * spline_shape(spline_r(r2) * inv_h));
          if (inside)
            atomicAdd(&win[((rx + a - lo) * WY + (ry + b - lo)) * WZ + (rz + c - lo)], w);
          else
            atomicAdd(&mass[(((size_t)((ix + a) & MASK) * N) + ((iy + b) & MASK)) * N +
                            ((iz + c) & MASK)],
                      w);
        }
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < WX * WY * WZ; c += kSplineBlock) {
    const unsigned long long v = win[c];
    if (v != 0ull) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t cell = ((size_t)((ox + lo + lx) & MASK) * N + ((oy + lo + ly) & MASK)) * N +
                          ((oz + lo + lz) & MASK);
      atomicAdd(&mass[cell], v);
    }
  }
}

template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_spline_qforce(const void* __restrict__ pos,
                                                          int64_t np,
                                                          const float* __restrict__ qmesh,
                                                          float h, float inv_h, float coef,
                                                          int lo, int hi,
                                                          float* __restrict__ acc) {
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const float h2 = h * h;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ix, iy, iz;
    float fx, fy, fz;
    cell_frac<LOGN, FIXED>(pos, p, ix, fx);
    cell_frac<LOGN, FIXED>(pos, np + p, iy, fy);
    cell_frac<LOGN, FIXED>(pos, 2 * np + p, iz, fz);
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    for (int ox = lo; ox <= hi; ++ox) {
      const float dx = (float)ox - fx;
      const float dx2 = dx * dx;
      if (dx2 > h2) continue;
      const size_t rx = (size_t)((ix + ox) & MASK) * N;
      int y0, y1;
      axis_span(fy, h2 - dx2, lo, hi, y0, y1);
      for (int oy = y0; oy <= y1; ++oy) {
        const float dy = (float)oy - fy;
        const float dxy2 = dx2 + dy * dy;
        if (dxy2 > h2) continue;
        const size_t rxy = (rx + ((iy + oy) & MASK)) * N;
        int z0, z1;
        axis_span(fz, h2 - dxy2, lo, hi, z0, z1);
        for (int oz = z0; oz <= z1; ++oz) {
          const float dz = (float)oz - fz;
          const float r2 = dxy2 + dz * dz;
          if (r2 > h2 || r2 == 0.0f) continue;
          // Q_j dW/dr / r times the node offset x_j - q_i; 1/r from the
          // hardware reciprocal square root, its argument held normal (below
          // 2^-100 cell^2 the term, dW/dr / r times an offset under 2^-50,
          // vanishes either way)
          const float ri = __builtin_amdgcn_rsqf(fmaxf(r2, 0x1p-100f));
          const float g = qmesh[rxy + ((iz + oz) & MASK)] * spline_slope(r2 * ri * inv_h) * ri;
          ax = fmaf(g, dx, ax);
          ay = fmaf(g, dy, ay);
          az = fmaf(g, dz, az);
        }
      }
    }
    acc[p] = coef * ax;
    acc[np + p] = coef * ay;
    acc[2 * np + p] = coef * az;
  }
}

// Half-kick of the spline step: v += fg g_phi + fq g_q, arrays [3][np].
__global__ void __launch_bounds__(kBlock) k_spline_kick(float* __restrict__ vel,
                                                        const float* __restrict__ gphi,
                                                        const float* __restrict__ gq, int64_t n,
                                                        float fg, float fq) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    vel[i] = fmaf(fq, gq[i], fmaf(fg, gphi[i], vel[i]));
}

// Drift of the spline step: x += fd v, periodic.  Fixed point: the
// displacement rounded to the nearest unit, 32-bit wrap; float: wrapped into
// [0, N).
template <int LOGN, bool FIXED>
__global__ void __launch_bounds__(kBlock) k_spline_drift(void* __restrict__ pos,
                                                         const float* __restrict__ vel,
                                                         int64_t n, double fd) {
  constexpr int N = 1 << LOGN;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if constexpr (FIXED) {
      const double units = (double)vel[i] * fd * (double)(1ull << (32 - LOGN));
      uint32_t* u = static_cast<uint32_t*>(pos);
      u[i] += (uint32_t)(int64_t)llrint(units);
    } else {
      float* x = static_cast<float*>(pos);
      float v = fmaf((float)fd, vel[i], x[i]);
      v -= (float)N * floorf(v * (1.0f / (float)N));
      x[i] = v >= (float)N ? 0.0f : v;
    }
  }
}

unsigned spline_grid(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// Node offsets from the particle's cell that can lie within h: the node
// j = i + o is within reach when |o - f| <= h for some f in [0, 1).
void spline_range(float h, int& lo, int& hi) {
  lo = -(int)floorf(h);
  hi = (int)floorf(h) + 1;
}

}  // namespace

hipError_t launch_spline_deposit(bool fixed, int logn, const void* pos, int64_t np, float h,
                                 const TileMap* tm, unsigned long long* mass, hipStream_t s) {
  int lo, hi;
  spline_range(h, lo, hi);
  const float coef = (float)(8.0 / (M_PI * (double)h * h * h));
  // the window of a tile holds offsets lo .. hi beyond its cells
  if (tm && -lo <= kSplineReach && hi <= kSplineReach) {
    const dim3 gt(tiled_grid(np, tm->tiles));
#define T_(LN)                                                                                \
  {                                                                                           \
    /* windows above 64 KiB of LDS (h >= 3.5) need the launch limit raised */                \
    const int lds = 8 * spline_tile_nodes<LN>(hi - lo);                                       \
    const void* kf = fixed ? reinterpret_cast<const void*>(&k_spline_deposit_tiled<LN, true>)  \
                           : reinterpret_cast<const void*>(&k_spline_deposit_tiled<LN, false>); \
    const hipError_t e = hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, lds); \
    if (e != hipSuccess) return e;                                                            \
    if (fixed)                                                                                \
      hipLaunchKernelGGL((k_spline_deposit_tiled<LN, true>), gt, dim3(kSplineBlock), lds, s,  \
                         pos, np, *tm, h, 1.0f / h, coef, lo, hi, mass);                      \
    else                                                                                      \
      hipLaunchKernelGGL((k_spline_deposit_tiled<LN, false>), gt, dim3(kSplineBlock), lds, s, \
                         pos, np, *tm, h, 1.0f / h, coef, lo, hi, mass);                      \
  }
    FDM_LOGN_SWITCH(logn, T_)
#undef T_
    return hipGetLastError();
  }
  const unsigned g = spline_grid(np);
#define L_(LN)                                                                               \
  if (fixed)                                                                                 \
    hipLaunchKernelGGL((k_spline_deposit<LN, true>), dim3(g), dim3(kBlock), 0, s, pos, np, h, \
                       1.0f / h, coef, lo, hi, mass);                                        \
  else                                                                                       \
    hipLaunchKernelGGL((k_spline_deposit<LN, false>), dim3(g), dim3(kBlock), 0, s, pos, np, h, \
                       1.0f / h, coef, lo, hi, mass);
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}


hipError_t launch_spline_qforce(bool fixed, int logn, const void* pos, int64_t np,
                                const float* q, float h, float* acc, hipStream_t s) {
  int lo, hi;
  spline_range(h, lo, hi);
  const float coef = (float)(8.0 / (M_PI * (double)h * h * h * h));
  const unsigned g = spline_grid(np);
#define L_(LN)                                                                              \
  if (fixed)                                                                                \
    hipLaunchKernelGGL((k_spline_qforce<LN, true>), dim3(g), dim3(kBlock), 0, s, pos, np, q, h, \
                       1.0f / h, coef, lo, hi, acc);                                        \
  else                                                                                      \
    hipLaunchKernelGGL((k_spline_qforce<LN, false>), dim3(g), dim3(kBlock), 0, s, pos, np, q, \
                       h, 1.0f / h, coef, lo, hi, acc);
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_spline_kick(float* vel, const float* gphi, const float* gq, int64_t np,
                              float fg, float fq, hipStream_t s) {
  const int64_t n = 3 * np;
  hipLaunchKernelGGL(k_spline_kick, dim3(spline_grid(n)), dim3(kBlock), 0, s, vel, gphi, gq, n,
                     fg, fq);
  return hipGetLastError();
}

hipError_t launch_spline_drift(bool fixed, int logn, void* pos, const float* vel, int64_t np,
                               double fd, hipStream_t s) {
  const int64_t n = 3 * np;
  const unsigned g = spline_grid(n);
#define L_(LN)                                                                               \
  if (fixed)                                                                                 \
    hipLaunchKernelGGL((k_spline_drift<LN, true>), dim3(g), dim3(kBlock), 0, s, pos, vel, n, fd); \
  else                                                                                       \
    hipLaunchKernelGGL((k_spline_drift<LN, false>), dim3(g), dim3(kBlock), 0, s, pos, vel, n, fd);
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace fdm
