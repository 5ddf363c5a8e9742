// Quantum pressure on the mesh, step (ii) of Sec. II A:
//   Q_c = -(hbar/m)^2/2 * L7[sqrt R] / sqrt R,  R = max(rho, floor),
// L7 the compact 7-point stencil; the comoving Q of Eq. (18) is Q_c / a^2.
//
// Fixed-point form ("s-form"): with rho = 1 + delta, s = sqrt R - 1 is formed
// as delta / (1 + sqrt(1 + delta)), which keeps full FP32 relative precision
// for small delta; L7[sqrt R] = L7[s] exactly since the constant cancels.
// Cells with rho below a threshold recompute sqrt R and Q in FP64 from the
// exact integer mass (the 1/sqrt(rho) division is ill-conditioned there).
// Plain FP32 form: sqrt(R) and the stencil directly in FP32.
//
// With kOutEnergy, each block also writes FP64 partial sums of delta*phi (for
// the potential energy) and of sum_d (sqrt R_{j+e_d} - sqrt R_j)^2 (gradient
// energy K_rho of Eq. (6), forward differences); a single-block kernel reduces
// the partials in a fixed order, so the totals are deterministic.  With
// kOutPsi the output is psi_g * phi + psi_q * Q instead of Q.
#include "internal.h"

namespace fdm {

// Fixed-point form: the hardware square root and reciprocal (about 1 ulp
// each; arguments stay in the normal range, r >= the density floor), which
// keep s to a few ulp relative at every delta.  Q in FP32 is ~7 us faster
// at 256^3 than with correctly rounded sqrtf and division.
__device__ __forceinline__ float sqrt_hw(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// FP64 square root and reciprocal for the near-empty path: the hardware
// single-precision estimate refined by two Newton steps in FP64 (relative
// error a few 1e-16 for the positive normal arguments used here), several
// times cheaper than the correctly rounded library forms.
__device__ __forceinline__ double sqrt_d(double r) {
  double y = (double)__builtin_amdgcn_rsqf((float)r);   // ~1/sqrt(r), single precision
  y = y * (1.5 - 0.5 * r * y * y);
  y = y * (1.5 - 0.5 * r * y * y);
  return r * y;
}
__device__ __forceinline__ double rcp_d(double x) {
  double y = (double)__builtin_amdgcn_rcpf((float)x);   // ~1/x, single precision
  y = y * (2.0 - x * y);
  y = y * (2.0 - x * y);
  return y;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  // wave64 shuffle reduction, then across the block's waves through LDS
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  __syncthreads();
  return t;
}

template <int LOGN, bool FIXED, int OUT>
__global__ void __launch_bounds__(kBlock) k_qpot(const float* __restrict__ delta,
                                                 const long long* __restrict__ mass,
                                                 const float* __restrict__ phi,
                                                 float* __restrict__ q, QConst qc,
                                                 double* __restrict__ partials, Batch bt) {
  {
    const int sl = bslot(bt);
    delta = woff(delta, bt, sl);
    mass = woff(mass, bt, sl);
    phi = woff(phi, bt, sl);
    q = woff(q, bt, sl);
    partials = woff(partials, bt, sl);
    if (bt.consts) {
      qc.coef = bt.consts[blockIdx.y].qcoef;
      qc.coef_d = bt.consts[blockIdx.y].qcoef_d;
      qc.psi_g = bt.consts[blockIdx.y].fg;
      qc.psi_q = bt.consts[blockIdx.y].fq;
    }
  }
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int iz = (int)(i & MASK);
  const int iy = (int)((i >> LOGN) & MASK);
  const int ix = (int)(i >> (2 * LOGN));
  const size_t row = i - iz;
  const size_t zp = row + ((iz + 1) & MASK), zm = row + ((iz - 1) & MASK);
  const size_t yp = ((size_t)ix * N + ((iy + 1) & MASK)) * N + iz;
  const size_t ym = ((size_t)ix * N + ((iy - 1) & MASK)) * N + iz;
  const size_t xp = ((size_t)((ix + 1) & MASK) * N + iy) * N + iz;
  const size_t xm = ((size_t)((ix - 1) & MASK) * N + iy) * N + iz;
  const float dc = delta[i];
  const float dn[6] = {delta[xp], delta[xm], delta[yp], delta[ym], delta[zp], delta[zm]};
  float sc, sn[6];
  float qv;
  if constexpr (FIXED) {
    auto sfun = [&](float d) {
      const float r = 1.0f + d;
      return (r >= qc.floor_f) ? d * rcp_hw(1.0f + sqrt_hw(r)) : qc.s_floor;
    };
    sc = sfun(dc);
#pragma unroll
    for (int k = 0; k < 6; ++k) sn[k] = sfun(dn[k]);
    const float lap = ((sn[0] + sn[1]) + (sn[2] + sn[3]) + (sn[4] + sn[5])) - 6.0f * sc;
    qv = qc.coef * lap * rcp_hw(1.0f + sc);
    if ((double)(1.0f + dc) < qc.fp64_below) {
      auto sd = [&](size_t j) {
        double r = (double)mass[j] * qc.inv_mbar;
        r = r > qc.floor_d ? r : qc.floor_d;
        return sqrt_d(r);
      };
      const double c = sd(i);
      const double lapd = ((sd(xp) + sd(xm)) + (sd(yp) + sd(ym)) + (sd(zp) + sd(zm))) - 6.0 * c;
      qv = (float)(qc.coef_d * lapd * rcp_d(c));
    }
  } else {
    auto sfun = [&](float d) {
      const float r = 1.0f + d;
      return sqrtf(r >= qc.floor_f ? r : qc.floor_f);
    };
    sc = sfun(dc);
#pragma unroll
    for (int k = 0; k < 6; ++k) sn[k] = sfun(dn[k]);
    const float lap = ((sn[0] + sn[1]) + (sn[2] + sn[3]) + (sn[4] + sn[5])) - 6.0f * sc;
    qv = qc.coef * lap / sc;
  }
  if constexpr (OUT == kOutPsi)
    q[i] = fmaf(qc.psi_q, qv, qc.psi_g * phi[i]);
  else
    q[i] = qv;
  if constexpr (OUT == kOutEnergy) {
    __shared__ double red[kBlock / 64];
    const double w = (double)dc * (double)phi[i];
    const double e0 = (double)(sn[0] - sc), e1 = (double)(sn[2] - sc), e2 = (double)(sn[4] - sc);
    const double u = e0 * e0 + e1 * e1 + e2 * e2;
    const double ws = block_sum(w, red);
    const double us = block_sum(u, red);
    if (threadIdx.x == 0) {
      partials[2 * (size_t)blockIdx.x] = ws;
      partials[2 * (size_t)blockIdx.x + 1] = us;
    }
  }
}

// Tiled version (N >= 32): a block owns a QY x QZ column of (y, z) and sweeps
// QX consecutive x-planes.  Each plane of s-values (with a one-cell y/z halo)
// is loaded once into LDS; the x-neighbours stay in registers, so delta is
// read about (QY+2)(QZ+2)/(QY QZ) times instead of once per stencil point.
// The loads of planes x + 2 and x + 3 are in flight while plane x is computed.
#ifndef FDM_QPOT_QX
#define FDM_QPOT_QX 16
#endif
#ifndef FDM_QPOT_QY
#define FDM_QPOT_QY 32   // 256^3: 51.1 us against 52.2 (16 rows) and 55.4 (8 rows)
#endif
constexpr int QY = FDM_QPOT_QY, QZ = 32;
#ifndef FDM_QPOT_QX_SMALL
#define FDM_QPOT_QX_SMALL 4
#endif
// x-planes per block: fewer on meshes up to 128^3, so that a run (or a
// batch slot) still spreads over enough blocks to fill the CUs (128^3:
// 512 blocks of 4 planes instead of 128 of 16; the extra x-halo planes are
// cache hits at these sizes)
__host__ __device__ constexpr int qpot_qx(int logn) {
  return logn <= 7 ? FDM_QPOT_QX_SMALL : FDM_QPOT_QX;
}
constexpr int kQBlock = QY * QZ;   // threads per block of the tiled stencil
#ifndef FDM_XCD_QPOT
#define FDM_XCD_QPOT 8   // a z-row of blocks per XCD at a time (256^3: 64 -> 62 us)
#endif
static_assert(kQBlock % 64 == 0 && kQBlock / 64 <= 64, "whole waves, one flag per lane");

template <bool FIXED>
__device__ __forceinline__ float s_of(float d, const QConst& qc) {
  const float r = 1.0f + d;
  if constexpr (FIXED) return (r >= qc.floor_f) ? d * rcp_hw(1.0f + sqrt_hw(r)) : qc.s_floor;
  return sqrtf(r >= qc.floor_f ? r : qc.floor_f);
}

template <int LOGN, bool FIXED, int OUT>
__global__ void __launch_bounds__(kQBlock, OUT == kOutEnergy ? 1 : 8) k_qpot_tiled(const float* __restrict__ delta,
                                                       const long long* __restrict__ mass,
                                                       const float* __restrict__ phi,
                                                       float* __restrict__ q, QConst qc,
                                                       double* __restrict__ partials, Batch bt) {
  {
    const int sl = bslot(bt);
    delta = woff(delta, bt, sl);
    mass = woff(mass, bt, sl);
    phi = woff(phi, bt, sl);
    q = woff(q, bt, sl);
    partials = woff(partials, bt, sl);
    if (bt.consts) {
      qc.coef = bt.consts[blockIdx.y].qcoef;
      qc.coef_d = bt.consts[blockIdx.y].qcoef_d;
      qc.psi_g = bt.consts[blockIdx.y].fg;
      qc.psi_q = bt.consts[blockIdx.y].fq;
    }
  }
  constexpr int N = 1 << LOGN;
  constexpr int MASK = N - 1;
  constexpr int PY = QY + 2, PZ = QZ + 2;
  constexpr int PER = (PY * PZ + kQBlock - 1) / kQBlock;   // plane values per thread
  // two plane buffers: plane x + 1 is committed to one while plane x is read
  // from the other, and planes x + 2 and x + 3 are already in flight in
  // registers
  __shared__ float pl[2][PY * PZ];
  // FP64 sqrt(R) of one plane from the exact integer mass, built only where
  // this plane or the next holds a near-empty cell, so the in-plane values of
  // a near-empty region are computed once per cell
  __shared__ double dpl[FIXED ? PY * PZ : 1];
  // per wave: whether the committed plane holds a near-empty cell (two slots,
  // alternating by plane)
  __shared__ uint32_t nflag[2][kQBlock / 64];
  const int nby = N / QY, nbz = N / QZ;
  const int b = (int)xcd_block(blockIdx.x, gridDim.x, FDM_XCD_QPOT);
  const int bz = b % nbz, by = (b / nbz) % nby, bx = b / (nbz * nby);
  constexpr int QX = qpot_qx(LOGN);
  const int y0 = by * QY, z0 = bz * QZ, x0 = bx * QX;
  const int ty = threadIdx.x / QZ, tz = threadIdx.x % QZ;
  const int y = y0 + ty, z = z0 + tz;
  const float sq_floor = sqrtf((float)qc.fp64_below) - 1.0f;
  const float near = sq_floor + 1e-6f;            // s below which a cell takes the FP64 path
  const bool use64 = FIXED && qc.fp64_below > 0.0;
  auto plane_index = [&](int x, int c) {
    const int ly = c / PZ, lz = c % PZ;
    return (size_t)(x & MASK) * N * N + (size_t)((y0 - 1 + ly) & MASK) * N +
           ((z0 - 1 + lz) & MASK);
  };
  // Two register buffers take alternate planes (even and odd offsets from
  // x0), so while plane x is computed the loads of planes x + 2 and x + 3 are
  // both in flight (twice the bytes in flight of one buffer).
  float preA[PER], preB[PER];
  auto fetch = [&](int x, float (&pre)[PER]) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = threadIdx.x + k * kQBlock;
      if (c < PY * PZ) pre[k] = delta[plane_index(x, c)];
    }
  };
  // s-values of the fetched plane into buf; records whether any is near empty
  auto commit = [&](float* buf, int slot, const float (&pre)[PER]) {
    bool any = false;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = threadIdx.x + k * kQBlock;
      if (c < PY * PZ) {
        const float sv = s_of<FIXED>(pre[k], qc);
        buf[c] = sv;
        any = any || sv < near;
      }
    }
    if (use64) {
      const bool wave_any = __any(any);
      if (threadIdx.x % 64 == 0) nflag[slot][threadIdx.x / 64] = wave_any;
    }
  };
  // after the barrier that follows commit(.., slot)
  // (lane w reads wave w's flag; one vote over the wave)
  auto plane_near = [&](int slot) {
    if (!use64) return false;
    const int lane = threadIdx.x & 63;
    const uint32_t f = lane < kQBlock / 64 ? nflag[slot][lane] : 0u;
    return (bool)__any(f != 0u);
  };
  auto sdv = [&](long long m) {
    double r = (double)m * qc.inv_mbar;
    r = r > qc.floor_d ? r : qc.floor_d;
    return sqrt_d(r);
  };
  auto sd = [&](size_t j) { return sdv(mass[j]); };
  // The integer mass of the next plane, loaded while this one is computed
  // once the next plane is known to hold a near-empty cell (block-uniform),
  // so its FP64 values do not wait for a full load latency (evolved 256^3
  // box: 119 -> 95 us; it takes the last 2 of the 64 VGPRs that two blocks
  // per CU allow, hence the launch bound of 8 waves per SIMD; the energy
  // form keeps its 80 VGPRs and one block per CU rather than spill).
  long long mpre[PER];
  bool mpre_ok = false;
  const int cc = (ty + 1) * PZ + tz + 1;
  auto inplane = [&](const float* buf) {
    return (buf[cc - PZ] + buf[cc + PZ]) + (buf[cc - 1] + buf[cc + 1]);
  };
  auto phi_at = [&](int x) { return phi[((size_t)x * N + y) * N + z]; };
  double wsum = 0.0, usum = 0.0;
  float s_prev = s_of<FIXED>(delta[((size_t)((x0 - 1) & MASK) * N + y) * N + z], qc);
  // phi of the own column, two planes ahead (psi and energy outputs), in the
  // slot of the plane's parity
  float phA = 0.0f, phB = 0.0f;
  if constexpr (OUT != kOutQ) {
    phA = phi_at(x0);
    phB = phi_at(x0 + 1);
  }
  fetch(x0, preA);
  commit(pl[0], 0, preA);
  fetch(x0 + 1, preB);
  fetch(x0 + 2, preA);
  __syncthreads();
  bool near_cur = plane_near(0);                  // plane x holds a near-empty cell
  float s_cur = pl[0][cc];
  float in_cur = inplane(pl[0]);
  float sy_cur = pl[0][cc + PZ], sz_cur = pl[0][cc + 1];
  double d_prev = 0.0;                            // FP64 sqrt(R) of plane x - 1, own column
  // plane x: its successor x + 1 sits in `nxt` (loads issued two planes ago),
  // which then takes plane x + 3; `ph` holds phi of plane x and then x + 2
  auto plane = [&](int x, float (&nxt)[PER], float& ph) {
    const int nbi = (x - x0 + 1) & 1;
    float* nb = pl[nbi];
    commit(nb, nbi, nxt);                     // plane x + 1
    if (x + 3 <= x0 + QX) fetch(x + 3, nxt);
    __syncthreads();
    const bool near_next = plane_near(nbi);
    const float s_next = nb[cc];
    const float in_next = inplane(nb);
    const float sy_next = nb[cc + PZ], sz_next = nb[cc + 1];
    // FP64 values of plane x: needed by its own near-empty cells and, as the
    // x - 1 neighbour, by those of plane x + 1 (block-uniform condition)
    double d_c = 0.0, d_ym = 0.0, d_yp = 0.0, d_zm = 0.0, d_zp = 0.0;
    if constexpr (FIXED) {
      if (near_cur || near_next) {
        if (!mpre_ok) {
#pragma unroll
          for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * kQBlock;
            if (c < PY * PZ) mpre[k] = mass[plane_index(x, c)];
          }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int c = threadIdx.x + k * kQBlock;
          if (c < PY * PZ) dpl[c] = sdv(mpre[k]);
        }
        // plane x + 1 holds a near-empty cell: its FP64 values will be built
        mpre_ok = near_next && x + 1 < x0 + QX;
        if (mpre_ok) {
#pragma unroll
          for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * kQBlock;
            if (c < PY * PZ) mpre[k] = mass[plane_index(x + 1, c)];
          }
        }
        __syncthreads();
        d_c = dpl[cc];
        d_ym = dpl[cc - PZ];
        d_yp = dpl[cc + PZ];
        d_zm = dpl[cc - 1];
        d_zp = dpl[cc + 1];
      }
    }
    const size_t i = ((size_t)x * N + y) * N + z;
    const float lap = ((s_prev + s_next) + in_cur) - 6.0f * s_cur;
    float qv;
    if constexpr (FIXED) {
      qv = qc.coef * lap * rcp_hw(1.0f + s_cur);
      if (use64 && s_cur < near) {
        // near-empty cell: sqrt(R) and Q in FP64 from the exact integer mass
        const double c0 = d_c;
        if (c0 * c0 < qc.fp64_below) {
          if (x == x0) d_prev = sd(((size_t)((x0 - 1) & MASK) * N + y) * N + z);
          const double d_next = sd(((size_t)((x + 1) & MASK) * N + y) * N + z);
          const double lapd = ((d_next + d_prev) + (d_yp + d_ym) + (d_zp + d_zm)) - 6.0 * c0;
          qv = (float)(qc.coef_d * lapd * rcp_d(c0));
        }
      }
    } else {
      qv = qc.coef * lap / s_cur;
    }
    if constexpr (OUT == kOutPsi)
      q[i] = fmaf(qc.psi_q, qv, qc.psi_g * ph);
    else
      q[i] = qv;
    if constexpr (OUT == kOutEnergy) {
      wsum += (double)delta[i] * (double)ph;
      const double e0 = (double)(s_next - s_cur), e1 = (double)(sy_cur - s_cur),
                   e2 = (double)(sz_cur - s_cur);
      usum += e0 * e0 + e1 * e1 + e2 * e2;
    }
    if constexpr (OUT != kOutQ)
      if (x + 2 < x0 + QX) ph = phi_at(x + 2);
    s_prev = s_cur;
    s_cur = s_next;
    in_cur = in_next;
    sy_cur = sy_next;
    sz_cur = sz_next;
    d_prev = d_c;
    near_cur = near_next;
  };
  static_assert(QX % 2 == 0, "planes go in pairs");
  for (int x = x0; x < x0 + QX; x += 2) {
    plane(x, preB, phA);
    plane(x + 1, preA, phB);
  }
  if constexpr (OUT == kOutEnergy) {
    __shared__ double red[kQBlock / 64];
    const double ws = block_sum(wsum, red);
    const double us = block_sum(usum, red);
    if (threadIdx.x == 0) {
      partials[2 * (size_t)blockIdx.x] = ws;
      partials[2 * (size_t)blockIdx.x + 1] = us;
    }
  }
}

int qpot_blocks(int logn) {
#ifndef FDM_QPOT_SIMPLE
  if (logn >= 5) return (int)(((size_t)1 << (3 * logn)) / ((size_t)QY * QZ * qpot_qx(logn)));
#endif
  return (int)(((size_t)1 << (3 * logn)) / kBlock);
}

hipError_t launch_qpot(int logn, bool fixed, int out, const float* delta,
                       const long long* mass, const float* phi, float* q, const QConst& qc,
                       double* partials, hipStream_t s, const Batch& bt) {
  const dim3 g((unsigned)qpot_blocks(logn), bt.count);
  if (out != kOutQ && out != kOutEnergy && out != kOutPsi) return hipErrorInvalidValue;
#define K_(KERNEL, LN, FX, TB)                                                               \
  {                                                                                          \
    if (out == kOutEnergy)                                                                   \
      hipLaunchKernelGGL((KERNEL<LN, FX, kOutEnergy>), g, dim3(TB), 0, s, delta, mass,        \
                         phi, q, qc, partials, bt);                                          \
    else if (out == kOutPsi)                                                                 \
      hipLaunchKernelGGL((KERNEL<LN, FX, kOutPsi>), g, dim3(TB), 0, s, delta, mass, phi,      \
                         q, qc, partials, bt);                                               \
    else                                                                                     \
      hipLaunchKernelGGL((KERNEL<LN, FX, kOutQ>), g, dim3(TB), 0, s, delta, mass, phi, q,     \
                         qc, partials, bt);                                                  \
  }
#ifndef FDM_QPOT_SIMPLE
  if (logn >= 5) {
#define T_(LN)                          \
  {                                     \
    if (fixed)                          \
      K_(k_qpot_tiled, LN, true, kQBlock)  \
    else                                \
      K_(k_qpot_tiled, LN, false, kQBlock) \
  }
    switch (logn) {
      case 5: T_(5); break;
      case 6: T_(6); break;
      case 7: T_(7); break;
      case 8: T_(8); break;
      case 9: T_(9); break;
      default: return hipErrorInvalidValue;
    }
#undef T_
    return hipGetLastError();
  }
#endif
#define L_(LN)                   \
  {                              \
    if (fixed)                   \
      K_(k_qpot, LN, true, kBlock)  \
    else                         \
      K_(k_qpot, LN, false, kBlock) \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
#undef K_
  return hipGetLastError();
}

// Sum ncomp interleaved components of nblocks partials, fixed order.
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partials,
                                                   int nblocks, int ncomp,
                                                   double* __restrict__ out, Batch bt) {
  {
    const int sl = bslot(bt);
    partials = woff(partials, bt, sl);
    out = woff(out, bt, sl);
  }
  __shared__ double red[kBlock];
  for (int c = 0; c < ncomp; ++c) {
    double t = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) t += partials[(size_t)b * ncomp + c];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
    __syncthreads();
  }
}

hipError_t launch_reduce(const double* partials, int nblocks, int ncomp, double* out,
                         hipStream_t s, const Batch& bt) {
  hipLaunchKernelGGL(k_reduce, dim3(1, bt.count), dim3(kBlock), 0, s, partials, nblocks, ncomp,
                     out, bt);
  return hipGetLastError();
}

// One synchronised state's energies from the stencil's interleaved
// (delta phi, gradient) block partials and the gather's |p|^2 block partials:
// each component summed in a fixed order (strided per thread, then a tree).
__global__ void __launch_bounds__(kBlock) k_energy_row(const double* __restrict__ qpart, int nq,
                                                       const double* __restrict__ kpart, int nk,
                                                       EnergyScale sc, double* __restrict__ out) {
  __shared__ double red[3][kBlock];
  double w = 0.0, u = 0.0, k = 0.0;
  for (int b = threadIdx.x; b < nq; b += kBlock) {
    w += qpart[2 * (size_t)b];
    u += qpart[2 * (size_t)b + 1];
  }
  for (int b = threadIdx.x; b < nk; b += kBlock) k += kpart[b];
  red[0][threadIdx.x] = k;
  red[1][threadIdx.x] = w;
  red[2][threadIdx.x] = u;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double K = sc.k * red[0][0], W = sc.w * red[1][0], U = sc.u * red[2][0];
    out[0] = K;
    out[1] = W;
    out[2] = U;
    out[3] = K + W + U;
  }
}

hipError_t launch_energy_row(const double* qpart, int nq, const double* kpart, int nk,
                             EnergyScale sc, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_energy_row, dim3(1), dim3(kBlock), 0, s, qpart, nq, kpart, nk, sc, out);
  return hipGetLastError();
}

}  // namespace fdm
