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
//
// With DEP the same pass also deposits each drifted particle (step (i) of
// the next step): into the LDS window of the block's tile when the particle
// is still inside it, else with direct global atomics; the window is added
// to the mass mesh at the end of the block.  The caller zeroes the mesh.
#include <type_traits>

#include "cic.h"
#include "internal.h"

namespace fdm {

// kKickCopy: kick, writing the velocities to `acc` and copying the position
// words to `pos_out` (the closing half-kick of a call whose particles ended in
// the workspace copies: kick and copy back in one pass).
enum GatherMode : int { kKick = 0, kKickDrift = 1, kForce = 2, kKickCopy = 3 };

// Position of one particle from its three 32-bit position words (fixed-point
// units, or float bits): integer cell and fraction along each axis.
template <int LOGN, bool FIXED>
__device__ __forceinline__ void decode_cell(const uint32_t raw[3], int ic[3], float f[3],
                                            uint32_t u[3], float xf[3]) {
  constexpr int MASK = (1 << LOGN) - 1;
  constexpr int B = 32 - LOGN;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (FIXED) {
      u[d] = raw[d];
      ic[d] = (int)(u[d] >> B);
      f[d] = (float)(u[d] & ((1u << B) - 1u)) * (1.0f / (float)(1u << B));
    } else {
      xf[d] = __uint_as_float(raw[d]);
      const float fl = floorf(xf[d]);
      f[d] = xf[d] - fl;
      ic[d] = (int)fl & MASK;
    }
  }
}

// Component d of particle p in a structure-of-arrays buffer of 4-byte
// words.  With a 32-bit index (p < 2^30, which the particle limit of 8 N^3
// <= 2^30 keeps) the address is a per-component base, uniform over the
// block, plus a 32-bit byte offset.
template <typename T>
__device__ __forceinline__ T& soa(T* base, int64_t np, int d, int64_t p) {
  return base[d * np + p];
}
template <typename T>
__device__ __forceinline__ T& soa(T* base, int64_t np, int d, unsigned p) {
  static_assert(sizeof(T) == 4, "4-byte words");
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return *reinterpret_cast<T*>(reinterpret_cast<B*>(base + d * np) + (p << 2));
}

// The position words and velocity of particle p.
template <typename P>
__device__ __forceinline__ void load_particle(const void* __restrict__ pos,
                                              const float* __restrict__ vel, int64_t np, P p,
                                              uint32_t raw[3], float v[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    raw[d] = soa(static_cast<const uint32_t*>(pos), np, d, p);
    v[d] = vel ? soa(vel, np, d, p) : 0.0f;
  }
}

// Interpolated -grad F at one particle.  at(a, b, c) returns F at offsets
// (a - 1, b - 1, c - 1) from the particle's base cell, a, b, c in 0..3.
// Central differences at the 8 CIC nodes use the 2x2x2 core and, per axis,
// the two planes outside it; each axis' extra nodes are consumed as soon as
// they are read, so only the core stays live.
template <typename At>
__device__ __forceinline__ void interp_grad(const float f[3], At&& at, float g[3]) {
  float core[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) core[a][b][c] = at(1 + a, 1 + b, 1 + c);
  const float wx[2] = {1.0f - f[0], f[0]};
  const float wy[2] = {1.0f - f[1], f[1]};
  const float wz[2] = {1.0f - f[2], f[2]};
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      // node x offset 0 -> difference F(+1) - F(-1) uses core[1] and the plane at offset -1
      const float lo = at(0, 1 + b, 1 + c), hi = at(3, 1 + b, 1 + c);
      gx += wy[b] * wz[c] * (wx[0] * (core[1][b][c] - lo) + wx[1] * (hi - core[0][b][c]));
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const float lo = at(1 + a, 0, 1 + c), hi = at(1 + a, 3, 1 + c);
      gy += wx[a] * wz[c] * (wy[0] * (core[a][1][c] - lo) + wy[1] * (hi - core[a][0][c]));
    }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const float lo = at(1 + a, 1 + b, 0), hi = at(1 + a, 1 + b, 3);
      gz += wx[a] * wy[b] * (wz[0] * (core[a][b][1] - lo) + wz[1] * (hi - core[a][b][0]));
    }
  g[0] = -0.5f * gx;
  g[1] = -0.5f * gy;
  g[2] = -0.5f * gz;
}

// Low 32 bits of rint(a * b), ties to even: the drift in fixed-point units,
// wrapped.  For |a * b| < 2^51 (a drift below 2^19 box lengths), adding
// 1.5 * 2^52 rounds the product to an integer and leaves it, two's
// complement, in the low mantissa bits.  No fma contraction.
__device__ __forceinline__ uint32_t rint_mul_low32(double a, double b) {
#pragma clang fp contract(off)
  const double t = a * b;
  return (uint32_t)__double_as_longlong(t + 0x1.8p52);
}

// Apply the result for particle p: store the force, or kick (and drift).
template <int LOGN, bool FIXED, int MODE, typename P>
__device__ __forceinline__ void push(void* __restrict__ pos, float* __restrict__ vel,
                                     float* __restrict__ acc, int64_t np, P p,
                                     const float g[3], const float vin[3], const uint32_t u[3],
                                     const float xf[3], double fd_units, uint32_t unew[3],
                                     float xnew[3], void* __restrict__ pos_out = nullptr) {
  constexpr int N = 1 << LOGN;
  if constexpr (MODE == kForce) {
#pragma unroll
    for (int d = 0; d < 3; ++d) soa(acc, np, d, p) = g[d];
  } else if constexpr (MODE == kKickCopy) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      soa(acc, np, d, p) = vin[d] + g[d];
      soa(static_cast<uint32_t*>(pos_out), np, d, p) = FIXED ? u[d] : __float_as_uint(xf[d]);
    }
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float v = vin[d] + g[d];
      soa(vel, np, d, p) = v;
      if constexpr (MODE == kKickDrift) {
        if constexpr (FIXED) {
          unew[d] = u[d] + rint_mul_low32((double)v, fd_units);
          soa(static_cast<uint32_t*>(pos), np, d, p) = unew[d];
        } else {
          float x = xf[d] + v * (float)fd_units;
          x = x - (float)N * floorf(x * (1.0f / (float)N));
          if (x >= (float)N) x = 0.0f;
          xnew[d] = x;
          soa(static_cast<float*>(pos), np, d, p) = x;
        }
      }
    }
  }
}

// The potential the gather differentiates at one node.  With Q it is
// F = fg phi + fq Q, with the stencil's psi rounding (fq Q added by one
// fma); without Q it is phi (or psi) itself, and fg multiplies the
// interpolated gradient instead (gradient and interpolation are linear; for
// psi, fg = 1).
template <int LOGN, bool HAS_Q>
__device__ __forceinline__ float mesh_f(const float* __restrict__ phi, const float* __restrict__ q,
                                        const GatherConst& gc, size_t idx) {
  if constexpr (HAS_Q) return fmaf(gc.fq, q[idx], gc.fg * phi[idx]);
  return phi[idx];
}

// The factor on the interpolated gradient (fg without Q, see mesh_f).
template <bool HAS_Q>
__device__ __forceinline__ void scale_grad(const GatherConst& gc, float g[3]) {
  if constexpr (!HAS_Q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] *= gc.fg;
  }
}

// mesh_f at a byte offset below 2^32 (the mesh is at most 512^3 floats).
template <bool HAS_Q>
__device__ __forceinline__ float mesh_f_at(const float* __restrict__ phi,
                                           const float* __restrict__ q, const GatherConst& gc,
                                           uint32_t off) {
  const float p = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(phi) + off);
  if constexpr (HAS_Q)
    return fmaf(gc.fq, *reinterpret_cast<const float*>(reinterpret_cast<const char*>(q) + off),
                gc.fg * p);
  return p;
}

// Weights of the drifted particle for the fused deposit.
template <int LOGN, bool FIXED, typename T>
__device__ __forceinline__ void new_weights(const uint32_t unew[3], const float xnew[3], int& ix,
                                            int& iy, int& iz, T w[8]) {
  if constexpr (FIXED)
    fixed_weights<LOGN>(unew[0], unew[1], unew[2], ix, iy, iz, w);
  else
    float_weights<LOGN>(xnew[0], xnew[1], xnew[2], ix, iy, iz, w);
}

// FP64 sum of one value per thread over the block (all threads call it);
// the wave sums go through `red` (one slot per wave).
template <int BLOCK>
__device__ __forceinline__ double block_total(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
  return t;
}

// Energy form of the kick: -grad phi and -grad Q interpolated separately
// (gp, gq); the closing half-kick of the previous step gives the momentum at
// the synchronised time (vk, whose |vk|^2 enters K), the opening half-kick of
// this step the kick applied on top of it (g).
__device__ __forceinline__ void split_kick(const GatherConst& gc, const float vin[3],
                                           const float gp[3], const float gq[3], float vk[3],
                                           float g[3], double& ksum) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vk[d] = vin[d] + fmaf(gc.fq, gq[d], gc.fg * gp[d]);
    g[d] = fmaf(gc.oq, gq[d], gc.og * gp[d]);
    ksum += (double)vk[d] * (double)vk[d];
  }
}

template <int LOGN, bool FIXED, bool HAS_Q, int MODE, bool DEP, bool EN = false>
__global__ void __launch_bounds__(kBlock) k_gather(void* __restrict__ pos,
                                                   float* __restrict__ vel,
                                                   const float* __restrict__ phi,
                                                   const float* __restrict__ q, int64_t np,
                                                   GatherConst gc, float* __restrict__ acc,
                                                   void* __restrict__ mass_v, Batch bt) {
  {
    const int sl = bslot(bt);
    pos = poff(pos, bt, sl);
    vel = poff(vel, bt, sl);
    acc = poff(acc, bt, sl);
    phi = woff(phi, bt, sl);
    q = woff(q, bt, sl);
    mass_v = woff(mass_v, bt, sl);
    if (bt.consts) {
      const SlotConst& sc = bt.consts[blockIdx.y];
      if (!gc.psi) {
        gc.fg = sc.fg;
        gc.fq = sc.fq;
      }
      gc.fd_units = sc.fd_units;
    }
  }
  using T = typename std::conditional<FIXED, unsigned long long, float>::type;
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double ksum = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
    int ic[3];
    float f[3], xf[3], vin[3];
    uint32_t u[3], raw[3];
    load_particle(pos, MODE == kForce ? nullptr : vel, np, p, raw, vin);
    decode_cell<LOGN, FIXED>(raw, ic, f, u, xf);
    auto node = [&](int a, int b, int c) {
      return ((size_t)((ic[0] + a - 1) & MASK) * N + ((ic[1] + b - 1) & MASK)) * N +
             ((ic[2] + c - 1) & MASK);
    };
    float g[3], vk[3];
    if constexpr (EN) {
      float gp[3], gq[3] = {0.0f, 0.0f, 0.0f};
      interp_grad(f, [&](int a, int b, int c) { return phi[node(a, b, c)]; }, gp);
      if constexpr (HAS_Q)
        interp_grad(f, [&](int a, int b, int c) { return q[node(a, b, c)]; }, gq);
      split_kick(gc, vin, gp, gq, vk, g, ksum);
    } else {
      interp_grad(f, [&](int a, int b, int c) {
        return mesh_f<LOGN, HAS_Q>(phi, q, gc, node(a, b, c));
      }, g);
      scale_grad<HAS_Q>(gc, g);
#pragma unroll
      for (int d = 0; d < 3; ++d) vk[d] = vin[d];
    }
    uint32_t unew[3];
    float xnew[3];
    push<LOGN, FIXED, MODE>(pos, vel, acc, np, p, g, vk, u, xf, gc.fd_units, unew, xnew, mass_v);
    if constexpr (DEP) {
      int jx, jy, jz;
      T w[8];
      new_weights<LOGN, FIXED>(unew, xnew, jx, jy, jz, w);
      deposit_global<LOGN>(static_cast<T*>(mass_v), jx, jy, jz, w);
    }
  }
  if constexpr (EN) {
    __shared__ double kred[kBlock / 64];
    const double t = block_total<kBlock>(ksum, kred);
    if (threadIdx.x == 0) gc.kpart[blockIdx.x] = t;
  }
}

// Tiled gather: block b owns tile b of the particle sort.  F = fg phi + fq Q
// is staged once for the tile's window (cells -1 .. T+1 around the tile) in
// LDS; particles still inside their tile read their 32 nodes from LDS,
// particles that left it read the mesh directly.
// WIDE: a one-cell larger gather window and a two-cell deposit halo, for
// steps whose particles have moved since the sort in a clustered state.
// Waves per SIMD that the LDS windows leave room for (three 512-thread
// blocks per CU with the narrow windows, two with the wide ones or two
// energy-form windows); the register budget is held to that.
constexpr int gather_waves(int wide, bool two_windows) { return wide || two_windows ? 4 : 6; }

template <int LOGN, bool FIXED, bool HAS_Q, int MODE, bool DEP, int WIDE = 0, bool EN = false>
__global__ void __launch_bounds__(kGatherBlock, gather_waves(WIDE, EN && HAS_Q))
    k_gather_tiled(void* __restrict__ pos,
                                                         float* __restrict__ vel,
                                                         const float* __restrict__ phi,
                                                         const float* __restrict__ q, int64_t np,
                                                         TileMap tm, GatherConst gc,
                                                         float* __restrict__ acc,
                                                         void* __restrict__ mass_v, Batch bt) {
  {
    const int sl = bslot(bt);
    pos = poff(pos, bt, sl);
    vel = poff(vel, bt, sl);
    acc = poff(acc, bt, sl);
    phi = woff(phi, bt, sl);
    q = woff(q, bt, sl);
    mass_v = woff(mass_v, bt, sl);
    tm.start = woff(tm.start, bt, sl);
    tm.chunk_start = woff(tm.chunk_start, bt, sl);
    if (bt.consts) {
      const SlotConst& sc = bt.consts[blockIdx.y];
      if (!gc.psi) {
        gc.fg = sc.fg;
        gc.fq = sc.fq;
      }
      gc.fd_units = sc.fd_units;
    }
  }
  using T = typename std::conditional<FIXED, unsigned long long, float>::type;
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int TX = 1 << tile_lx(LOGN), TY = 1 << tile_ly(LOGN), TZ = 1 << tile_lz(LOGN);
  constexpr int HG = WIDE ? 1 : kGatherHalo, HD = WIDE ? 2 : kDepHalo;
  // F window: cells o - 1 - HG .. o + T + 1 + HG; deposit window: o - HD .. o + T + HD
  constexpr int WX = TX + 3 + 2 * HG, WY = TY + 3 + 2 * HG, WZ = TZ + 3 + 2 * HG;
  constexpr int NTY = N / TY, NTZ = N / TZ;
  constexpr int DX = TX + 1 + 2 * HD, DY = TY + 1 + 2 * HD, DZ = TZ + 1 + 2 * HD;
  __shared__ float win[WX * WY * WZ];
  // energy form: win holds phi and winq holds Q (interpolated separately)
  __shared__ float winq[EN && HAS_Q ? WX * WY * WZ : 1];
  __shared__ T dacc[DEP ? DX * DY * DZ : 1];
  __shared__ unsigned n_stray;
  int t;
  unsigned lo, hi;
  if (!chunk_of(tm, t, lo, hi)) {
    if constexpr (EN)
      if (threadIdx.x == 0) gc.kpart[blockIdx.x] = 0.0;
    return;
  }
  if (threadIdx.x == 0) n_stray = 0;
  // the first particles' loads are in flight while the window is staged;
  // afterwards particle p + PF * kGatherBlock is loaded while p is processed
  constexpr int PF = kGatherPrefetch;
  uint32_t raw_n[PF][3];
  float vin_n[PF][3];
#pragma unroll
  for (int k = 0; k < PF; ++k) {
    const unsigned pk = lo + threadIdx.x + k * kGatherBlock;
    if (pk < hi) load_particle(pos, vel, np, pk, raw_n[k], vin_n[k]);
  }
  const int ox = (t / (NTY * NTZ)) * TX, oy = ((t / NTZ) % NTY) * TY, oz = (t % NTZ) * TZ;
  if constexpr (EN) {
    for (int c = threadIdx.x; c < WX * WY * WZ; c += kGatherBlock) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t idx = ((size_t)((ox - 1 - HG + lx) & MASK) * N +
                          ((oy - 1 - HG + ly) & MASK)) * N + ((oz - 1 - HG + lz) & MASK);
      win[c] = phi[idx];
      if constexpr (HAS_Q) winq[c] = q[idx];
    }
  } else if constexpr (HAS_Q) {
    for (int c = threadIdx.x; c < WX * WY * WZ; c += kGatherBlock) {
      const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
      const size_t idx = ((size_t)((ox - 1 - HG + lx) & MASK) * N +
                          ((oy - 1 - HG + ly) & MASK)) * N + ((oz - 1 - HG + lz) & MASK);
      win[c] = mesh_f<LOGN, HAS_Q>(phi, q, gc, idx);
    }
  } else {
    // all of a thread's window loads are issued before the first is used
    // (faster for the one-field window; the two-field one was slower so)
    constexpr int WN = WX * WY * WZ;
    constexpr int WPER = (WN + kGatherBlock - 1) / kGatherBlock;
    float wphi[WPER];
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int c = threadIdx.x + k * kGatherBlock;
      if (WN % kGatherBlock == 0 || c < WN) {
        const int lx = c / (WY * WZ), ly = (c / WZ) % WY, lz = c % WZ;
        const size_t idx = ((size_t)((ox - 1 - HG + lx) & MASK) * N +
                            ((oy - 1 - HG + ly) & MASK)) * N + ((oz - 1 - HG + lz) & MASK);
        wphi[k] = phi[idx];
      }
    }
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int c = threadIdx.x + k * kGatherBlock;
      if (WN % kGatherBlock == 0 || c < WN) win[c] = wphi[k];   // mesh_f without Q
    }
  }
  if constexpr (DEP)
    for (int c = threadIdx.x; c < DX * DY * DZ; c += kGatherBlock) dacc[c] = (T)0;
  __syncthreads();
  double ksum = 0.0;
  unsigned my_stray = 0;   // this thread's deposits outside the narrow window
  for (unsigned p = lo + threadIdx.x; p < hi; p += kGatherBlock) {
    int ic[3];
    float f[3], xf[3], vin[3];
    uint32_t u[3], raw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      raw[d] = raw_n[0][d];
      vin[d] = vin_n[0][d];
    }
#pragma unroll
    for (int k = 0; k + 1 < PF; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        raw_n[k][d] = raw_n[k + 1][d];
        vin_n[k][d] = vin_n[k + 1][d];
      }
    if (p + PF * kGatherBlock < hi)
      load_particle(pos, vel, np, p + PF * kGatherBlock, raw_n[PF - 1], vin_n[PF - 1]);
    decode_cell<LOGN, FIXED>(raw, ic, f, u, xf);
    const int rx = (ic[0] - ox + HG) & MASK, ry = (ic[1] - oy + HG) & MASK,
              rz = (ic[2] - oz + HG) & MASK;
    const bool in_win = rx < TX + 2 * HG && ry < TY + 2 * HG && rz < TZ + 2 * HG;
    // one base index; the 32 nodes at constant offsets from it
    const int lbase = (rx * WY + ry) * WZ + rz;
    auto lds = [&](int a, int b, int c) { return lbase + (a * WY + b) * WZ + c; };
    auto node = [&](int a, int b, int c) {
      return ((size_t)((ic[0] + a - 1) & MASK) * N + ((ic[1] + b - 1) & MASK)) * N +
             ((ic[2] + c - 1) & MASK);
    };
    float g[3], vk[3];
    if constexpr (EN) {
      float gp[3], gq[3] = {0.0f, 0.0f, 0.0f};
      if (in_win) {
        interp_grad(f, [&](int a, int b, int c) { return win[lds(a, b, c)]; }, gp);
        if constexpr (HAS_Q)
          interp_grad(f, [&](int a, int b, int c) { return winq[lds(a, b, c)]; }, gq);
      } else {
        interp_grad(f, [&](int a, int b, int c) { return phi[node(a, b, c)]; }, gp);
        if constexpr (HAS_Q)
          interp_grad(f, [&](int a, int b, int c) { return q[node(a, b, c)]; }, gq);
      }
      split_kick(gc, vin, gp, gq, vk, g, ksum);
    } else {
      if (in_win) {
        interp_grad(f, [&](int a, int b, int c) { return win[lds(a, b, c)]; }, g);
      } else {
        // byte offsets of the 4 x 4 x 4 neighbourhood from per-axis terms
        // (disjoint bit fields: one or per node)
        uint32_t bo_x[4], bo_y[4], bo_z[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          bo_x[a] = (uint32_t)((ic[0] + a - 1) & MASK) << (2 * LOGN + 2);
          bo_y[a] = (uint32_t)((ic[1] + a - 1) & MASK) << (LOGN + 2);
          bo_z[a] = (uint32_t)((ic[2] + a - 1) & MASK) << 2;
        }
        interp_grad(f, [&](int a, int b, int c) {
          return mesh_f_at<HAS_Q>(phi, q, gc, bo_x[a] | bo_y[b] | bo_z[c]);
        }, g);
      }
      scale_grad<HAS_Q>(gc, g);
#pragma unroll
      for (int d = 0; d < 3; ++d) vk[d] = vin[d];
    }
    uint32_t unew[3];
    float xnew[3];
    push<LOGN, FIXED, MODE>(pos, vel, acc, np, p, g, vk, u, xf, gc.fd_units, unew, xnew, mass_v);
    if constexpr (DEP) {
      // natural corner order (consecutive lanes of a wave add to neighbouring
      // cells together); the fixed-point remainder d goes to the heaviest
      // corner in a ninth add where it is not zero
      int jx, jy, jz, big = 0, dfix = 0;
      T w[8];
      if constexpr (FIXED)
        fixed_weights_split<LOGN>(unew[0], unew[1], unew[2], jx, jy, jz, w, big, dfix);
      else
        float_weights<LOGN>(xnew[0], xnew[1], xnew[2], jx, jy, jz, w);
      const int sx = (jx - ox + HD) & MASK, sy = (jy - oy + HD) & MASK,
                sz = (jz - oz + HD) & MASK;
      const bool inside = sx < TX + 2 * HD && sy < TY + 2 * HD && sz < TZ + 2 * HD;
      if (inside) {
        const int a0 = (sx * DY + sy) * DZ + sz;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          atomicAdd(&dacc[a0 + ((c >> 2) * DY + ((c >> 1) & 1)) * DZ + (c & 1)], w[c]);
        if constexpr (FIXED)
          if (dfix != 0)
            atomicAdd(&dacc[a0 + ((big >> 2) * DY + ((big >> 1) & 1)) * DZ + (big & 1)],
                      (T)(long long)dfix);
      } else {
        if constexpr (FIXED) {
#pragma unroll
          for (int c = 0; c < 8; ++c)
            if (c == big) w[c] += (T)(long long)dfix;
        }
        deposit_global<LOGN>(static_cast<T*>(mass_v), jx, jy, jz, w);
      }
      // count strays (always against the narrow deposit window, so that the
      // sort interval chosen from them does not depend on the window used)
      constexpr int HN = kDepHalo;
      const bool inside_n = ((jx - ox + HN) & MASK) < TX + 2 * HN &&
                            ((jy - oy + HN) & MASK) < TY + 2 * HN &&
                            ((jz - oz + HN) & MASK) < TZ + 2 * HN;
      my_stray += inside_n ? 0u : 1u;
    }
  }
  if constexpr (DEP) {
    // one LDS add per wave
    for (int off = 32; off > 0; off >>= 1) my_stray += __shfl_down(my_stray, off, 64);
    if ((threadIdx.x & 63) == 0 && my_stray) atomicAdd(&n_stray, my_stray);
  }
  if constexpr (EN) {
    __shared__ double kred[kGatherBlock / 64];
    const double kt = block_total<kGatherBlock>(ksum, kred);
    if (threadIdx.x == 0) gc.kpart[blockIdx.x] = kt;
  }
  if constexpr (DEP) {
    __syncthreads();
    T* mass = static_cast<T*>(mass_v);
    if (threadIdx.x == 0 && n_stray)
      atomicAdd(reinterpret_cast<unsigned*>(reinterpret_cast<char*>(mass_v) +
                                            8 * ((size_t)N * N * N)) +
                    (blockIdx.x % kStraySlices) * kStrayStride,
                n_stray);
    // all of a thread's window cells are read before the first atomic
    constexpr int DN = DX * DY * DZ;
    constexpr int DPER = (DN + kGatherBlock - 1) / kGatherBlock;
    T dv[DPER];
#pragma unroll
    for (int k = 0; k < DPER; ++k) {
      const int c = threadIdx.x + k * kGatherBlock;
      dv[k] = (DN % kGatherBlock == 0 || c < DN) ? dacc[c] : (T)0;
    }
#pragma unroll
    for (int k = 0; k < DPER; ++k) {
      const int c = threadIdx.x + k * kGatherBlock;
      if (dv[k] != (T)0) {
        const int lx = c / (DY * DZ), ly = (c / DZ) % DY, lz = c % DZ;
        const size_t cell = ((size_t)((ox - HD + lx) & MASK) * N + ((oy - HD + ly) & MASK)) * N +
                            ((oz - HD + lz) & MASK);
        add_global(&mass[cell], dv[k]);
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

template <int LN, int MODE, bool DEP, bool EN = false>
static void launch_mode_tiled(bool fixed, bool has_q, hipStream_t s, void* pos, float* vel,
                              const float* phi, const float* q, int64_t np, const TileMap& tm,
                              const GatherConst& gc, float* acc, void* mass, const Batch& bt) {
  const dim3 g(tiled_grid(np, tm.tiles), bt.count);
  if (fixed && has_q)
    hipLaunchKernelGGL((k_gather_tiled<LN, true, true, MODE, DEP, 0, EN>), g, dim3(kGatherBlock),
                       0, s, pos, vel, phi, q, np, tm, gc, acc, mass, bt);
  else if (fixed)
    hipLaunchKernelGGL((k_gather_tiled<LN, true, false, MODE, DEP, 0, EN>), g, dim3(kGatherBlock),
                       0, s, pos, vel, phi, q, np, tm, gc, acc, mass, bt);
  else if (has_q)
    hipLaunchKernelGGL((k_gather_tiled<LN, false, true, MODE, DEP, 0, EN>), g, dim3(kGatherBlock),
                       0, s, pos, vel, phi, q, np, tm, gc, acc, mass, bt);
  else
    hipLaunchKernelGGL((k_gather_tiled<LN, false, false, MODE, DEP, 0, EN>), g,
                       dim3(kGatherBlock), 0, s, pos, vel, phi, q, np, tm, gc, acc, mass, bt);
}

template <int LN, int MODE, bool DEP, bool EN = false>
static void launch_mode(bool fixed, bool has_q, dim3 g, hipStream_t s, void* pos, float* vel,
                        const float* phi, const float* q, int64_t np, const GatherConst& gc,
                        float* acc, void* mass, const Batch& bt) {
  g.y = bt.count;
  if (fixed && has_q)
    hipLaunchKernelGGL((k_gather<LN, true, true, MODE, DEP, EN>), g, dim3(kBlock), 0, s, pos, vel,
                       phi, q, np, gc, acc, mass, bt);
  else if (fixed)
    hipLaunchKernelGGL((k_gather<LN, true, false, MODE, DEP, EN>), g, dim3(kBlock), 0, s, pos,
                       vel, phi, q, np, gc, acc, mass, bt);
  else if (has_q)
    hipLaunchKernelGGL((k_gather<LN, false, true, MODE, DEP, EN>), g, dim3(kBlock), 0, s, pos,
                       vel, phi, q, np, gc, acc, mass, bt);
  else
    hipLaunchKernelGGL((k_gather<LN, false, false, MODE, DEP, EN>), g, dim3(kBlock), 0, s, pos,
                       vel, phi, q, np, gc, acc, mass, bt);
}

template <int LN, bool EN = false>
static void launch_wide(bool has_q, hipStream_t s, void* pos, float* vel, const float* phi,
                        const float* q, int64_t np, const TileMap& tm, const GatherConst& gc,
                        void* mass, const Batch& bt) {
  const dim3 g(tiled_grid(np, tm.tiles), bt.count);
  if (has_q)
    hipLaunchKernelGGL((k_gather_tiled<LN, true, true, kKickDrift, true, 1, EN>), g,
                       dim3(kGatherBlock), 0, s, pos, vel, phi, q, np, tm, gc, nullptr, mass, bt);
  else
    hipLaunchKernelGGL((k_gather_tiled<LN, true, false, kKickDrift, true, 1, EN>), g,
                       dim3(kGatherBlock), 0, s, pos, vel, phi, q, np, tm, gc, nullptr, mass, bt);
}

unsigned gather_blocks(int64_t np, const TileMap* tm) {
  return tm ? tiled_grid(np, tm->tiles) : grid_particles(np);
}

hipError_t launch_gather(bool fixed, bool has_q, bool drift, int logn, void* pos, float* vel,
                         const float* phi, const float* q, int64_t np, const GatherConst& gc,
                         const TileMap* tm, void* deposit_mass, hipStream_t s, const Batch& bt,
                         bool wide, void* pos_out, float* vel_out) {
  const dim3 g(grid_particles(np));
  const bool dep = drift && deposit_mass != nullptr;
  const bool copy = !drift && tm && pos_out && vel_out;
  // the energy form exists for the launches a step makes: the fused
  // gather-deposit and the closing half-kick (with or without the copy back)
  if (gc.kpart && ((drift && !dep) || bt.slots)) return hipErrorInvalidValue;
#define L_(LN, EN)                                                                               \
  {                                                                                              \
    if (copy)                                                                                    \
      launch_mode_tiled<LN, kKickCopy, false, EN>(fixed, has_q, s, pos, vel, phi, q, np, *tm,    \
                                                  gc, vel_out, pos_out, bt);                     \
    else if (tm && dep && wide && fixed)                                                         \
      launch_wide<LN, EN>(has_q, s, pos, vel, phi, q, np, *tm, gc, deposit_mass, bt);            \
    else if (tm && dep)                                                                          \
      launch_mode_tiled<LN, kKickDrift, true, EN>(fixed, has_q, s, pos, vel, phi, q, np, *tm,    \
                                                  gc, nullptr, deposit_mass, bt);                \
    else if (tm && drift)                                                                        \
      launch_mode_tiled<LN, kKickDrift, false>(fixed, has_q, s, pos, vel, phi, q, np, *tm, gc,   \
                                               nullptr, nullptr, bt);                            \
    else if (tm)                                                                                 \
      launch_mode_tiled<LN, kKick, false, EN>(fixed, has_q, s, pos, vel, phi, q, np, *tm, gc,    \
                                              nullptr, nullptr, bt);                             \
    else if (dep)                                                                                \
      launch_mode<LN, kKickDrift, true, EN>(fixed, has_q, g, s, pos, vel, phi, q, np, gc,        \
                                            nullptr, deposit_mass, bt);                          \
    else if (drift)                                                                              \
      launch_mode<LN, kKickDrift, false>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr,  \
                                         nullptr, bt);                                           \
    else                                                                                         \
      launch_mode<LN, kKick, false, EN>(fixed, has_q, g, s, pos, vel, phi, q, np, gc, nullptr,   \
                                        nullptr, bt);                                            \
  }
#define E_(LN)          \
  {                     \
    if (gc.kpart)       \
      L_(LN, true)      \
    else                \
      L_(LN, false)     \
  }
  FDM_LOGN_SWITCH(logn, E_)
#undef E_
#undef L_
  return hipGetLastError();
}

// Query the wide-window kernels once, so that their first use inside a step
// loop does not also load them (a one-time stall of tens of ms otherwise).
hipError_t preload_wide(int logn) {
  hipFuncAttributes attr;
  hipError_t e = hipSuccess;
#define L_(LN)                                                                                   \
  {                                                                                              \
    e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(                               \
                                        &k_gather_tiled<LN, true, true, kKickDrift, true, 1>));   \
    if (e == hipSuccess)                                                                         \
      e = hipFuncGetAttributes(&attr, reinterpret_cast<const void*>(                             \
                                          &k_gather_tiled<LN, true, false, kKickDrift, true, 1>)); \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return e;
}

hipError_t launch_force(bool fixed, bool has_q, int logn, const void* pos, const float* phi,
                        const float* q, int64_t np, float fg, float fq, float* acc,
                        hipStream_t s) {
  const dim3 g(grid_particles(np));
  GatherConst gc;
  gc.fg = fg;
  gc.fq = fq;
  gc.fd_units = 0.0;
#define L_(LN)                                                                            \
  launch_mode<LN, kForce, false>(fixed, has_q, g, s, const_cast<void*>(pos), nullptr, phi, q, \
                                 np, gc, acc, nullptr, Batch())
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

// FP64 partial sums of |v|^2 per block.
__global__ void __launch_bounds__(kBlock) k_kinetic(const float* __restrict__ vel, int64_t np,
                                                    double* __restrict__ partials, Batch bt) {
  {
    const int sl = bslot(bt);
    vel = poff(vel, bt, sl);
    partials = woff(partials, bt, sl);
  }
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
                          hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_kinetic, dim3(nblocks, bt.count), dim3(kBlock), 0, s, vel, np, partials,
                     bt);
  return hipGetLastError();
}

}  // namespace fdm
