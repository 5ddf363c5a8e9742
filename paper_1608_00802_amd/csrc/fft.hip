// Three-dimensional real FFT Poisson solve on the periodic mesh (gravity on the
// same deposited density as the quantum pressure, Sec. II A), written as five
// streaming passes over the half-spectrum.  The spectrum is stored
// spec[kz][x][y] (kz = 0..N/2 outermost) so that every pass reads and writes
// contiguous runs:
//
//   1. z-pass  (R2C): rows along z -> length-N/2 complex FFT + real unpack;
//      the block transposes through LDS and writes spec[kz][x][y0:y0+TY].
//      Fused with forming delta from the mesh (exact integer subtract).
//   2. y-pass  : rows along y, contiguous in spec.
//   3. x-pass  : columns along x (stride N), tiles of TC consecutive y; the
//      forward FFT, the Green's function -S/K^2 (7-point Laplacian symbol,
//      zero mode removed, normalisation 2/N^3 folded in) and the inverse FFT
//      happen on one LDS tile.
//   4. y-pass  (inverse).
//   5. z-pass  (C2R): pack the Hermitian half-rows into a length-N/2 complex
//      sequence, inverse FFT, write real rows.
//
// Inside a block, each row is transformed by a Stockham autosort FFT with
// radix-4 stages (one leading radix-2 stage for odd log2 lengths): every
// thread loads its butterflies' inputs into registers, the block barriers,
// then results are written back to the same LDS rows -- one LDS buffer, two
// barriers per stage, natural order at the end.  Twiddles come from an FP64-
// built table exp(-2 pi i k / N) staged in LDS.
#include "internal.h"

namespace fdm {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// ROWS independent length-L complex FFTs on LDS rows buf[r*(L+1) + n].
// tw[k*TWS] = exp(-2 pi i k / L).  Forward: exp(-i); INV: exp(+i), no scaling.
template <int L, int ROWS, int NT, int TWS, bool INV>
__device__ __forceinline__ void fft_rows(float2* __restrict__ buf, const float2* __restrict__ tw) {
  constexpr int LP = L + 1;
  const int tid = threadIdx.x;
  int ns = 1;
  if constexpr ((ilog2c(L) & 1) != 0) {
    constexpr int NB = ROWS * (L / 2);
    constexpr int PER = (NB + NT - 1) / NT;
    float2 v[PER][2];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int t = tid + p * NT;
      if (NB % NT == 0 || t < NB) {
        const int row = t / (L / 2), j = t % (L / 2);
        v[p][0] = buf[row * LP + j];
        v[p][1] = buf[row * LP + j + L / 2];
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int t = tid + p * NT;
      if (NB % NT == 0 || t < NB) {
        const int row = t / (L / 2), j = t % (L / 2);
        buf[row * LP + 2 * j] = cadd(v[p][0], v[p][1]);
        buf[row * LP + 2 * j + 1] = csub(v[p][0], v[p][1]);
      }
    }
    __syncthreads();
    ns = 2;
  }
  int lns = (ilog2c(L) & 1);  // log2(ns)
  for (; ns < L; ns <<= 2, lns += 2) {
    constexpr int NB = ROWS * (L / 4);
    constexpr int PER = (NB + NT - 1) / NT;
    float2 v[PER][4];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int t = tid + p * NT;
      if (NB % NT == 0 || t < NB) {
        const int row = t / (L / 4), j = t % (L / 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[p][r] = buf[row * LP + j + r * (L / 4)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int t = tid + p * NT;
      if (NB % NT == 0 || t < NB) {
        const int row = t / (L / 4), j = t % (L / 4);
        const int k = j & (ns - 1);
        const int step = (k * ((L / 4) >> lns)) * TWS;
        float2 a0 = v[p][0], a1 = v[p][1], a2 = v[p][2], a3 = v[p][3];
        if (k != 0) {
          if (INV) {
            a1 = cmulc(a1, tw[step]);
            a2 = cmulc(a2, tw[2 * step]);
            a3 = cmulc(a3, tw[3 * step]);
          } else {
            a1 = cmul(a1, tw[step]);
            a2 = cmul(a2, tw[2 * step]);
            a3 = cmul(a3, tw[3 * step]);
          }
        }
        const float2 b0 = cadd(a0, a2), b1 = csub(a0, a2);
        const float2 b2 = cadd(a1, a3);
        const float2 d = csub(a1, a3);
        // forward: -i * d ; inverse: +i * d
        const float2 b3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
        const int base = ((j >> lns) << (lns + 2)) + k;
        buf[row * LP + base] = cadd(b0, b2);
        buf[row * LP + base + ns] = cadd(b1, b3);
        buf[row * LP + base + 2 * ns] = csub(b0, b2);
        buf[row * LP + base + 3 * ns] = csub(b1, b3);
      }
    }
    __syncthreads();
  }
}

#ifndef FDM_FFT_Z_ELEMS
#define FDM_FFT_Z_ELEMS 4096
#endif
#ifndef FDM_FFT_Y_ELEMS
#define FDM_FFT_Y_ELEMS 2048
#endif
#ifndef FDM_FFT_X_ELEMS
#define FDM_FFT_X_ELEMS 2048
#endif
#ifndef FDM_FFT_X_MINCOL
#define FDM_FFT_X_MINCOL 8
#endif
// Rows (complex elements / N) per block of each pass, and at least
// FDM_FFT_X_MINCOL consecutive y columns (64-byte segments) per x-pass
// block.  Small tiles leave room for four or more blocks per CU, so one
// block's transform overlaps another's loads (256^3: 30 us less per step
// than tiles twice as large).
template <int N>
struct Tiles {
  static constexpr int H = N / 2;
  static constexpr int ZE = FDM_FFT_Z_ELEMS, YE = FDM_FFT_Y_ELEMS, XE = FDM_FFT_X_ELEMS;
  static constexpr int MC = FDM_FFT_X_MINCOL;
  static constexpr int TZ = (ZE / N < N) ? ZE / N : N;   // rows per z-pass block
  static constexpr int TY = (YE / N < N) ? YE / N : N;   // rows per y-pass block
  static constexpr int TC = (XE / N >= MC) ? ((XE / N < N) ? XE / N : N) : MC;  // x-pass columns
};

// ---------------------------------------------------------------- pass 1
template <int LOGN, int SRC>
__global__ void __launch_bounds__(kBlock) k_r2c_z(const void* __restrict__ in,
                                                  float* __restrict__ delta_out,
                                                  float2* __restrict__ spec,
                                                  const float2* __restrict__ tw, DeltaConv conv,
                                                  Batch bt) {
  {
    const int sl = bslot(bt);
    in = woff(in, bt, sl);
    delta_out = woff(delta_out, bt, sl);
    spec = woff(spec, bt, sl);
  }
  constexpr int N = 1 << LOGN;
  constexpr int H = N / 2;
  constexpr int TZ = Tiles<N>::TZ;
  constexpr int LP = H + 1;
  __shared__ float2 buf[TZ * LP];
  __shared__ float2 tws[N];
  const int tid = threadIdx.x;
  const int x = blockIdx.x / (N / TZ);
  const int y0 = (blockIdx.x % (N / TZ)) * TZ;
  for (int k = tid; k < N; k += kBlock) tws[k] = tw[k];
  for (int idx = tid; idx < TZ * H; idx += kBlock) {
    const int r = idx / H, n = idx % H;
    const size_t cell = ((size_t)x * N + y0 + r) * N + 2 * n;
    float2 d;
    if constexpr (SRC == kSrcMass64) {
      const longlong2 m = *reinterpret_cast<const longlong2*>((const long long*)in + cell);
      d.x = (float)((double)(m.x - conv.mbar) / conv.dmbar);
      d.y = (float)((double)(m.y - conv.mbar) / conv.dmbar);
      *reinterpret_cast<float2*>(delta_out + cell) = d;
    } else if constexpr (SRC == kSrcAcc32) {
      const float2 a = *reinterpret_cast<const float2*>((const float*)in + cell);
      d.x = a.x * conv.acc_norm - 1.0f;
      d.y = a.y * conv.acc_norm - 1.0f;
      *reinterpret_cast<float2*>(delta_out + cell) = d;
    } else {
      d = *reinterpret_cast<const float2*>((const float*)in + cell);
    }
    buf[r * LP + n] = d;
  }
  __syncthreads();
  fft_rows<H, TZ, kBlock, 2, false>(buf, tws);
  // unpack: X_k = E + w^k O, X_{H-k} = conj(E - w^k O),
  // E = (Z_k + conj Z_{H-k})/2, O = -i (Z_k - conj Z_{H-k})/2
  for (int idx = tid; idx < TZ * (H / 2 + 1); idx += kBlock) {
    const int r = idx / (H / 2 + 1), k = idx % (H / 2 + 1);
    const float2 zk = buf[r * LP + k];
    const float2 zm = cconj(buf[r * LP + ((H - k) & (H - 1))]);
    const float2 e = cscale(cadd(zk, zm), 0.5f);
    const float2 dd = cscale(csub(zk, zm), 0.5f);
    const float2 o = make_float2(dd.y, -dd.x);
    const float2 wo = cmul(tws[k], o);
    buf[r * LP + k] = cadd(e, wo);
    if (k != H / 2) buf[r * LP + H - k] = cconj(csub(e, wo));
  }
  __syncthreads();
  for (int idx = tid; idx < (H + 1) * TZ; idx += kBlock) {
    const int kz = idx / TZ, r = idx % TZ;
    spec[((size_t)kz * N + x) * N + y0 + r] = buf[r * LP + kz];
  }
}

// ---------------------------------------------------------------- passes 2, 4
template <int LOGN, bool INV>
__global__ void __launch_bounds__(kBlock) k_fft_y(float2* __restrict__ spec,
                                                  const float2* __restrict__ tw, Batch bt) {
  spec = woff(spec, bt, bslot(bt));
  constexpr int N = 1 << LOGN;
  constexpr int TY = Tiles<N>::TY;
  constexpr int LP = N + 1;
  __shared__ float2 buf[TY * LP];
  __shared__ float2 tws[N];
  const int tid = threadIdx.x;
  const size_t row0 = (size_t)blockIdx.x * TY;
  for (int k = tid; k < N; k += kBlock) tws[k] = tw[k];
  for (int idx = tid; idx < TY * N; idx += kBlock) {
    const int r = idx / N, n = idx % N;
    buf[r * LP + n] = spec[(row0 + r) * N + n];
  }
  __syncthreads();
  fft_rows<N, TY, kBlock, 1, INV>(buf, tws);
  for (int idx = tid; idx < TY * N; idx += kBlock) {
    const int r = idx / N, n = idx % N;
    spec[(row0 + r) * N + n] = buf[r * LP + n];
  }
}

// ---------------------------------------------------------------- pass 3
template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_fft_x_green(float2* __restrict__ spec,
                                                        const float2* __restrict__ tw,
                                                        const float* __restrict__ s2,
                                                        float green_scale, Batch bt) {
  spec = woff(spec, bt, bslot(bt));
  constexpr int N = 1 << LOGN;
  constexpr int TC = Tiles<N>::TC;
  constexpr int LP = N + 1;
  __shared__ float2 buf[TC * LP];
  __shared__ float2 tws[N];
  __shared__ float s2s[N];
  const int tid = threadIdx.x;
  const int b = (int)xcd_block(blockIdx.x, gridDim.x, xcd_group(FDM_XCD_FFTX, gridDim.x));
  const int kz = b / (N / TC);
  const int y0 = (b % (N / TC)) * TC;
  for (int k = tid; k < N; k += kBlock) {
    tws[k] = tw[k];
    s2s[k] = s2[k];
  }
  for (int idx = tid; idx < N * TC; idx += kBlock) {
    const int xk = idx / TC, c = idx % TC;
    buf[c * LP + xk] = spec[((size_t)kz * N + xk) * N + y0 + c];
  }
  __syncthreads();
  fft_rows<N, TC, kBlock, 1, false>(buf, tws);
  const float s2z = s2s[kz];
  for (int idx = tid; idx < TC * N; idx += kBlock) {
    const int c = idx / N, kx = idx % N;
    const float k2 = s2s[kx] + s2s[y0 + c] + s2z;
    const float g = (k2 > 0.0f) ? green_scale / k2 : 0.0f;
    buf[c * LP + kx] = cscale(buf[c * LP + kx], g);
  }
  __syncthreads();
  fft_rows<N, TC, kBlock, 1, true>(buf, tws);
  for (int idx = tid; idx < N * TC; idx += kBlock) {
    const int xk = idx / TC, c = idx % TC;
    spec[((size_t)kz * N + xk) * N + y0 + c] = buf[c * LP + xk];
  }
}

// ---------------------------------------------------------------- pass 5
template <int LOGN>
__global__ void __launch_bounds__(kBlock) k_c2r_z(const float2* __restrict__ spec,
                                                  const float2* __restrict__ tw,
                                                  float* __restrict__ out, Batch bt) {
  {
    const int sl = bslot(bt);
    spec = woff(spec, bt, sl);
    out = woff(out, bt, sl);
  }
  constexpr int N = 1 << LOGN;
  constexpr int H = N / 2;
  constexpr int TZ = Tiles<N>::TZ;
  constexpr int LP = H + 1;
  __shared__ float2 buf[TZ * LP];
  __shared__ float2 tws[N];
  const int tid = threadIdx.x;
  const int x = blockIdx.x / (N / TZ);
  const int y0 = (blockIdx.x % (N / TZ)) * TZ;
  for (int k = tid; k < N; k += kBlock) tws[k] = tw[k];
  for (int idx = tid; idx < (H + 1) * TZ; idx += kBlock) {
    const int kz = idx / TZ, r = idx % TZ;
    buf[r * LP + kz] = spec[((size_t)kz * N + x) * N + y0 + r];
  }
  __syncthreads();
  // pack: E = (X_k + conj X_{H-k})/2, O = (X_k - conj X_{H-k}) conj(w^k)/2,
  // Z_k = E + i O, Z_{H-k} = conj(E) + i conj(O)
  for (int idx = tid; idx < TZ * (H / 2 + 1); idx += kBlock) {
    const int r = idx / (H / 2 + 1), k = idx % (H / 2 + 1);
    const float2 xk = buf[r * LP + k];
    const float2 xm = cconj(buf[r * LP + H - k]);
    const float2 e = cscale(cadd(xk, xm), 0.5f);
    const float2 o = cmulc(cscale(csub(xk, xm), 0.5f), tws[k]);
    buf[r * LP + k] = make_float2(e.x - o.y, e.y + o.x);
    if (k != 0 && k != H / 2) buf[r * LP + H - k] = make_float2(e.x + o.y, -e.y + o.x);
  }
  __syncthreads();
  fft_rows<H, TZ, kBlock, 2, true>(buf, tws);
  for (int idx = tid; idx < TZ * H; idx += kBlock) {
    const int r = idx / H, n = idx % H;
    *reinterpret_cast<float2*>(out + ((size_t)x * N + y0 + r) * N + 2 * n) = buf[r * LP + n];
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_r2c_z(int logn, int src, const void* in, float* delta_out, float2* spec,
                        const float2* tw, DeltaConv conv, hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                          \
  {                                                                                     \
    constexpr int N_ = 1 << LN;                                                         \
    dim3 g(N_ * (N_ / Tiles<N_>::TZ), bt.count);                                        \
    if (src == kSrcMass64)                                                              \
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcMass64>), g, dim3(kBlock), 0, s, in, delta_out, \
                         spec, tw, conv, bt);                                           \
    else if (src == kSrcAcc32)                                                          \
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcAcc32>), g, dim3(kBlock), 0, s, in, delta_out, \
                         spec, tw, conv, bt);                                           \
    else                                                                                \
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcDelta>), g, dim3(kBlock), 0, s, in, delta_out, \
                         spec, tw, conv, bt);                                           \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_fft_y(int logn, float2* spec, const float2* tw, bool inverse,
                        hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                    \
  {                                                                               \
    constexpr int N_ = 1 << LN;                                                   \
    dim3 g((N_ / 2 + 1) * (N_ / Tiles<N_>::TY), bt.count);                       \
    if (inverse)                                                                  \
      hipLaunchKernelGGL((k_fft_y<LN, true>), g, dim3(kBlock), 0, s, spec, tw, bt); \
    else                                                                          \
      hipLaunchKernelGGL((k_fft_y<LN, false>), g, dim3(kBlock), 0, s, spec, tw, bt); \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_fft_x_green(int logn, float2* spec, const float2* tw, const float* s2,
                              float green_scale, hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                      \
  {                                                                                 \
    constexpr int N_ = 1 << LN;                                                     \
    dim3 g((N_ / 2 + 1) * (N_ / Tiles<N_>::TC), bt.count);                          \
    hipLaunchKernelGGL((k_fft_x_green<LN>), g, dim3(kBlock), 0, s, spec, tw, s2,    \
                       green_scale, bt);                                            \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

hipError_t launch_c2r_z(int logn, const float2* spec, const float2* tw, float* out,
                        hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                  \
  {                                                                             \
    constexpr int N_ = 1 << LN;                                                 \
    dim3 g(N_ * (N_ / Tiles<N_>::TZ), bt.count);                                \
    hipLaunchKernelGGL((k_c2r_z<LN>), g, dim3(kBlock), 0, s, spec, tw, out, bt); \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace fdm
