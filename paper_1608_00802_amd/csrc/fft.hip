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
// The y and x passes split each length-N transform into two factors whose
// short DFTs run in registers, with one exchange through LDS between them
// (register FFTs below); the x pass keeps the forward result in registers
// through the Green's function into the inverse transform.  The z passes
// transform rows staged in LDS with a Stockham autosort FFT of radix-4 stages
// (one leading radix-2 stage for odd log2 lengths): every thread loads its
// butterflies' inputs into registers, the block barriers, then results are
// written back to the same LDS rows -- one LDS buffer, two barriers per
// stage, natural order at the end.  Twiddles come from an FP64-built table
// exp(-2 pi i k / N) staged in LDS.
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

#ifndef FDM_FFTZ_XG
#define FDM_FFTZ_XG 4   // 512^3 (8 rows per block): C2R 374 -> 351 us
#endif
#ifndef FDM_FFT_Z_ELEMS_512
// z-pass elements per block at N = 512: 32 rows, two whole 128-byte lines of
// the kz-major spectrum per kz (with 512 threads: C2R 263 -> 239 us against
// 16 rows, R2C unchanged; 8 rows took 352 and 482 us)
#define FDM_FFT_Z_ELEMS_512 16384
#endif
#ifndef FDM_FFT_Z_ELEMS
#define FDM_FFT_Z_ELEMS 4096
#endif
#ifndef FDM_FFTZ_BLOCK
// threads per block of the z passes (512 against 256: 256^3 R2C 64 -> 60 us,
// 512^3 R2C 439 -> 428 us and C2R 279 -> 263 us with 16 rows; 1024 threads
// with 32 rows: C2R 231 but R2C 476 us)
#define FDM_FFTZ_BLOCK 512
#endif
constexpr int kZBlock = FDM_FFTZ_BLOCK;
// Rows (complex elements / N) per block of the z passes.  Small tiles leave
// room for four or more blocks per CU, so one block's transform overlaps
// another's loads (256^3: 30 us less per step than tiles twice as large).
template <int N>
struct Tiles {
  static constexpr int ZE = (N >= 512 && FDM_FFT_Z_ELEMS_512) ? FDM_FFT_Z_ELEMS_512
                                                               : FDM_FFT_Z_ELEMS;
  static constexpr int TZ = (ZE / N < N) ? ZE / N : N;   // rows per z-pass block
  // below 16 rows a block's kz-major accesses cover part of each 128-byte
  // line: the blocks sharing a line go to one XCD together
  static constexpr int XG = TZ < 16 ? FDM_FFTZ_XG : 0;
};

// ---------------------------------------------------------------- register FFTs
// An L-point transform split as L = F1 x F2: F2 DFTs of length F1 over
// n = F2 n1 + n2, the twiddles W_L^{n2 k1}, then F1 DFTs of length F2 over
// n2, giving X[k1 + F1 k2].  Each short DFT runs in one thread's registers,
// so a transform makes one trip through LDS (the exchange between the two
// factors) instead of one per radix-4 stage.  The y and x passes use this
// form; the z passes (with their real-data packing) use fft_rows.
constexpr int kRegBlock = 128;   // threads per block of the register-FFT y passes
#ifndef FDM_FFTX_XT
#define FDM_FFTX_XT 0      // x-pass threads per block (0: 64 up to N = 256, 128 above)
#endif
#ifndef FDM_FFTX_TC
#define FDM_FFTX_TC 0      // x-pass columns per block (0: 4 up to N = 256, 8 above)
#endif
#ifndef FDM_FFTX_ORDER
#define FDM_FFTX_ORDER 0   // lanes across the block's columns (see x_item)
#endif
#ifndef FDM_FFTX_BIG
#define FDM_FFTX_BIG 64    // meshes from this size on take the 256-thread, 16-column x pass
#endif
#ifndef FDM_FFTX_PAD
#define FDM_FFTX_PAD -1    // extra float2 between the x pass's LDS columns (-1: per N)
#endif

template <int L>
struct Split {
  static constexpr int LG = ilog2c(L);
  static constexpr int R1 = 1 << ((LG + 1) / 2);   // first factor (the larger)
  static constexpr int R2 = L / R1;
};

constexpr int bitrev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

// In-register radix-2 DFT of length R (natural order in and out);
// tw[m * TS] = exp(-2 pi i m / R).  INV: exp(+i), no scaling.
template <int R, bool INV, int TS>
__device__ __forceinline__ void dft_reg(float2 (&v)[R], const float2* __restrict__ tw) {
  constexpr int B = ilog2c(R);
  float2 a[R];
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = v[bitrev_c(i, B)];
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
    for (int i = 0; i < R; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        float2 t = a[i + j + len / 2];
        const int m = j * (R / len);               // twiddle W_R^m
        if (m != 0) {
          if (4 * m == R) {
            t = INV ? make_float2(-t.y, t.x) : make_float2(t.y, -t.x);   // times +i / -i
          } else {
            const float2 w = tw[m * TS];
            t = INV ? cmulc(t, w) : cmul(t, w);
          }
        }
        a[i + j + len / 2] = csub(a[i + j], t);
        a[i + j] = cadd(a[i + j], t);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = a[i];
}

// First factor of an L-point transform for one n2: v[n1] = x[F2 n1 + n2] in,
// v[k1] = W_L^{n2 k1} * sum_n1 x[F2 n1 + n2] W_F1^{n1 k1} out.
// tw[m * TWS] = exp(-2 pi i m / L).
template <int L, int F1, bool INV, int TWS = 1>
__device__ __forceinline__ void fft_first(float2 (&v)[F1], int n2, const float2* __restrict__ tw) {
  dft_reg<F1, INV, (L / F1) * TWS>(v, tw);
#pragma unroll
  for (int k1 = 1; k1 < F1; ++k1) {
    const float2 w = tw[((n2 * k1) & (L - 1)) * TWS];
    v[k1] = INV ? cmulc(v[k1], w) : cmul(v[k1], w);
  }
}

// ---------------------------------------------------------------- pass 1
template <int LOGN, int SRC>
__global__ void __launch_bounds__(kZBlock) k_r2c_z(const void* __restrict__ in,
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
  const int zb = (int)xcd_block(blockIdx.x, gridDim.x, Tiles<N>::XG);
  const int x = zb / (N / TZ);
  const int y0 = (zb % (N / TZ)) * TZ;
  for (int k = tid; k < N; k += kZBlock) tws[k] = tw[k];
  {
    // all of a thread's loads are issued before the first is used
    constexpr int NE = TZ * H;
    constexpr int PER = (NE + kZBlock - 1) / kZBlock;
    longlong2 m[SRC == kSrcMass64 ? PER : 1];
    float2 a[SRC == kSrcMass64 ? 1 : PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * kZBlock;
      if (NE % kZBlock == 0 || idx < NE) {
        const size_t cell = ((size_t)x * N + y0 + idx / H) * N + 2 * (idx % H);
        if constexpr (SRC == kSrcMass64)
          m[k] = *reinterpret_cast<const longlong2*>((const long long*)in + cell);
        else
          a[k] = *reinterpret_cast<const float2*>((const float*)in + cell);
      }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * kZBlock;
      if (NE % kZBlock == 0 || idx < NE) {
        const int r = idx / H, n = idx % H;
        const size_t cell = ((size_t)x * N + y0 + r) * N + 2 * n;
        float2 d;
        if constexpr (SRC == kSrcMass64) {
          d.x = (float)((double)(m[k].x - conv.mbar) / conv.dmbar);
          d.y = (float)((double)(m[k].y - conv.mbar) / conv.dmbar);
          *reinterpret_cast<float2*>(delta_out + cell) = d;
        } else if constexpr (SRC == kSrcAcc32) {
          d.x = a[k].x * conv.acc_norm - 1.0f;
          d.y = a[k].y * conv.acc_norm - 1.0f;
          *reinterpret_cast<float2*>(delta_out + cell) = d;
        } else {
          d = a[k];
        }
        buf[r * LP + n] = d;
      }
    }
  }
  __syncthreads();
  fft_rows<H, TZ, kZBlock, 2, false>(buf, tws);
  // unpack: X_k = E + w^k O, X_{H-k} = conj(E - w^k O),
  // E = (Z_k + conj Z_{H-k})/2, O = -i (Z_k - conj Z_{H-k})/2
  for (int idx = tid; idx < TZ * (H / 2 + 1); idx += kZBlock) {
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
  for (int idx = tid; idx < (H + 1) * TZ; idx += kZBlock) {
    const int kz = idx / TZ, r = idx % TZ;
    spec[((size_t)kz * N + x) * N + y0 + r] = buf[r * LP + kz];
  }
}

// ---------------------------------------------------------------- passes 2-4
// Register-FFT versions of passes 2-4.  The y pass
// reads each row's F1-strided elements straight into registers and writes
// the result from registers; the x pass keeps the forward transform's output
// in registers for the Green's function and the inverse transform's first
// factor (whose inputs, X[k1 + R1 k2] for one k1, are exactly what one
// thread holds), so each transform crosses LDS once.
template <int N>
struct RegTiles {
  static constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  static constexpr int RMAX = R1 > R2 ? R1 : R2;
  static constexpr int RY0 = kRegBlock / R2;                       // y-pass rows per block
  static constexpr int RY = RY0 < N ? RY0 : N;
  // x pass: 256 threads and 16 columns from N = 64 on (whole 128-byte lines
  // per row; 256^3: 29.6 us against 37.5 with 64 threads and 4 columns and
  // 31.8 with 128 and 8; 512^3: 266 against 385 us with 128 and 8; 128^3:
  // 12.2 against 13.5 us with 64 and 4), 64 threads below; blocks that share
  // a line of a column run are grouped on one XCD
  static constexpr int XT = FDM_FFTX_XT ? FDM_FFTX_XT : (N < FDM_FFTX_BIG ? 64 : 256);  // threads
  static constexpr int TC0 =
      FDM_FFTX_TC ? FDM_FFTX_TC : (N < FDM_FFTX_BIG ? ((XT / RMAX > 4) ? XT / RMAX : 4) : 16);
  static constexpr int TC = TC0 < N ? TC0 : N;                     // x-pass columns per block
  static constexpr int XG = TC < 16 ? 16 / TC : 1;                 // XCD group
  // padding between the columns of the LDS exchange (2 entries with 16
  // columns: their 128-byte runs otherwise start in the same banks)
  static constexpr int PAD = FDM_FFTX_PAD >= 0 ? FDM_FFTX_PAD : (N >= FDM_FFTX_BIG ? 2 : 0);
};

// Work item `it` of the x pass: column c of the block's TC columns and index
// i < M along the transform.  Columns fastest across lanes: every group of
// four lanes loads one 32-byte run of a row (index fastest, with the same
// cache lines touched, took 46 instead of 38 us per pass at 256^3).
template <int TC, int M>
__device__ __forceinline__ void x_item(int it, int& c, int& i) {
  if constexpr (FDM_FFTX_ORDER != 0) {
    c = it / M;
    i = it % M;
  } else {
    c = it % TC;
    i = it / TC;
  }
}

template <int LOGN, bool INV>
__global__ void __launch_bounds__(kRegBlock) k_fft_y_reg(float2* __restrict__ spec,
                                                         const float2* __restrict__ tw,
                                                         Batch bt) {
  spec = woff(spec, bt, bslot(bt));
  constexpr int N = 1 << LOGN;
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  constexpr int RY = RegTiles<N>::RY;
  constexpr int XP = R1 + 1;                  // exchange: ex[r][n2][k1], k1 padded
  constexpr int NA = RY * R2, NB = RY * R1;   // work items of the two factors
  constexpr int PA = (NA + kRegBlock - 1) / kRegBlock, PB = (NB + kRegBlock - 1) / kRegBlock;
  __shared__ float2 ex[RY * R2 * XP];
  __shared__ float2 tws[N];
  const int tid = threadIdx.x;
  const size_t row0 = (size_t)blockIdx.x * RY;
  float2 v[PA][R1];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * kRegBlock;
    if (NA % kRegBlock == 0 || it < NA) {
      const int r = it / R2, n2 = it % R2;
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) v[p][n1] = spec[(row0 + r) * N + R2 * n1 + n2];
    }
  }
  for (int k = tid; k < N; k += kRegBlock) tws[k] = tw[k];
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * kRegBlock;
    if (NA % kRegBlock == 0 || it < NA) {
      const int r = it / R2, n2 = it % R2;
      fft_first<N, R1, INV>(v[p], n2, tws);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) ex[(r * R2 + n2) * XP + k1] = v[p][k1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int it = tid + p * kRegBlock;
    if (NB % kRegBlock == 0 || it < NB) {
      const int r = it / R1, k1 = it % R1;
      float2 u[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[n2] = ex[(r * R2 + n2) * XP + k1];
      dft_reg<R2, INV, N / R2>(u, tws);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) spec[(row0 + r) * N + k1 + R1 * k2] = u[k2];
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(RegTiles<1 << LOGN>::XT) k_fft_x_green_reg(float2* __restrict__ spec,
                                                               const float2* __restrict__ tw,
                                                               const float* __restrict__ s2,
                                                               float green_scale, Batch bt) {
  spec = woff(spec, bt, bslot(bt));
  constexpr int N = 1 << LOGN;
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  constexpr int TC = RegTiles<N>::TC;
  constexpr int XT = RegTiles<N>::XT;
  // forward exchange ex[c][n2][k1] (k1 < R1, padded), inverse ex[c][k1][k1']
  // (k1' < R2, padded); one buffer, the larger of the two
  constexpr int XF = R2 * (R1 + 1), XI = R1 * (R2 + 1);
  constexpr int XS = (XF > XI ? XF : XI) + RegTiles<N>::PAD;
  constexpr int NA = TC * R2, NB = TC * R1;   // items: first factor (R1 values) / second (R2 values)
  constexpr int PA = (NA + XT - 1) / XT, PB = (NB + XT - 1) / XT;
  __shared__ float2 ex[TC * XS];
  __shared__ float2 tws[N];
  __shared__ float s2s[N];
  const int tid = threadIdx.x;
  const int b = (int)xcd_block(blockIdx.x, gridDim.x, RegTiles<N>::XG);
  const int kz = b / (N / TC);
  const int y0 = (b % (N / TC)) * TC;
  auto at = [&](int x, int c) -> float2& { return spec[((size_t)kz * N + x) * N + y0 + c]; };
  // items of the first factor: c fastest, so a wave reads TC consecutive y
  float2 v[PA][R1];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * XT;
    if (NA % XT == 0 || it < NA) {
      int c, n2;
      x_item<TC, R2>(it, c, n2);
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) v[p][n1] = at(R2 * n1 + n2, c);
    }
  }
  for (int k = tid; k < N; k += XT) {
    tws[k] = tw[k];
    s2s[k] = s2[k];
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * XT;
    if (NA % XT == 0 || it < NA) {
      int c, n2;
      x_item<TC, R2>(it, c, n2);
      fft_first<N, R1, false>(v[p], n2, tws);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) ex[c * XS + n2 * (R1 + 1) + k1] = v[p][k1];
    }
  }
  __syncthreads();
  // second factor: item (c, k1) gets X[k1 + R1 k2], k2 < R2; times G; then
  // the inverse transform's first factor over the same values (n = R1 k2 + k1)
  float2 u[PB][R2];
  const float s2z = s2s[kz];
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int it = tid + p * XT;
    if (NB % XT == 0 || it < NB) {
      int c, k1;
      x_item<TC, R1>(it, c, k1);
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[p][n2] = ex[c * XS + n2 * (R1 + 1) + k1];
      dft_reg<R2, false, N / R2>(u[p], tws);
      const float s2yz = s2s[y0 + c] + s2z;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const float k2sum = s2s[k1 + R1 * k2] + s2yz;
        const float g = (k2sum > 0.0f) ? green_scale / k2sum : 0.0f;
        u[p][k2] = cscale(u[p][k2], g);
      }
      fft_first<N, R2, true>(u[p], k1, tws);
    }
  }
  __syncthreads();   // every read of the forward exchange is done
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int it = tid + p * XT;
    if (NB % XT == 0 || it < NB) {
      int c, k1;
      x_item<TC, R1>(it, c, k1);
#pragma unroll
      for (int j = 0; j < R2; ++j) ex[c * XS + k1 * (R2 + 1) + j] = u[p][j];
    }
  }
  __syncthreads();
  // inverse second factor: item (c, j), j < R2, over k1 < R1: x[j + R2 m]
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * XT;
    if (NA % XT == 0 || it < NA) {
      int c, j;
      x_item<TC, R2>(it, c, j);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) v[p][k1] = ex[c * XS + k1 * (R2 + 1) + j];
      dft_reg<R1, true, N / R1>(v[p], tws);
#pragma unroll
      for (int m = 0; m < R1; ++m) at(j + R2 * m, c) = v[p][m];
    }
  }
}

// ---------------------------------------------------------------- pass 5
template <int LOGN>
__global__ void __launch_bounds__(kZBlock) k_c2r_z(const float2* __restrict__ spec,
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
  const int zb = (int)xcd_block(blockIdx.x, gridDim.x, Tiles<N>::XG);
  const int x = zb / (N / TZ);
  const int y0 = (zb % (N / TZ)) * TZ;
  for (int k = tid; k < N; k += kZBlock) tws[k] = tw[k];
  {
    // all of a thread's loads are issued before the first is used
    constexpr int NE = (H + 1) * TZ;
    constexpr int PER = (NE + kZBlock - 1) / kZBlock;
    float2 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * kZBlock;
      if (NE % kZBlock == 0 || idx < NE)
        v[k] = spec[((size_t)(idx / TZ) * N + x) * N + y0 + idx % TZ];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = tid + k * kZBlock;
      if (NE % kZBlock == 0 || idx < NE) buf[(idx % TZ) * LP + idx / TZ] = v[k];
    }
  }
  __syncthreads();
  // pack: E = (X_k + conj X_{H-k})/2, O = (X_k - conj X_{H-k}) conj(w^k)/2,
  // Z_k = E + i O, Z_{H-k} = conj(E) + i conj(O)
  for (int idx = tid; idx < TZ * (H / 2 + 1); idx += kZBlock) {
    const int r = idx / (H / 2 + 1), k = idx % (H / 2 + 1);
    const float2 xk = buf[r * LP + k];
    const float2 xm = cconj(buf[r * LP + H - k]);
    const float2 e = cscale(cadd(xk, xm), 0.5f);
    const float2 o = cmulc(cscale(csub(xk, xm), 0.5f), tws[k]);
    buf[r * LP + k] = make_float2(e.x - o.y, e.y + o.x);
    if (k != 0 && k != H / 2) buf[r * LP + H - k] = make_float2(e.x + o.y, -e.y + o.x);
  }
  __syncthreads();
  fft_rows<H, TZ, kZBlock, 2, true>(buf, tws);
  for (int idx = tid; idx < TZ * H; idx += kZBlock) {
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
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcMass64>), g, dim3(kZBlock), 0, s, in, delta_out, \
                         spec, tw, conv, bt);                                           \
    else if (src == kSrcAcc32)                                                          \
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcAcc32>), g, dim3(kZBlock), 0, s, in, delta_out, \
                         spec, tw, conv, bt);                                           \
    else                                                                                \
      hipLaunchKernelGGL((k_r2c_z<LN, kSrcDelta>), g, dim3(kZBlock), 0, s, in, delta_out, \
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
    dim3 g((N_ / 2 + 1) * (N_ / RegTiles<N_>::RY), bt.count);                     \
    if (inverse)                                                                  \
      hipLaunchKernelGGL((k_fft_y_reg<LN, true>), g, dim3(kRegBlock), 0, s, spec, tw, bt); \
    else                                                                          \
      hipLaunchKernelGGL((k_fft_y_reg<LN, false>), g, dim3(kRegBlock), 0, s, spec, tw, bt); \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

// Power spectrum pass: the forward x transform of the x pass, then |X|^2 of
// every mode binned by its integer mode number |m| into shells
// [b - 1/2, b + 1/2), b = 1..nb, in FP64 LDS bins; each block writes its nb
// (sum, weight) pairs to partials[block][2 (nb + 1)] with plain stores.  The
// spectrum holds kz = 0..N/2 only: modes with 0 < kz < N/2 stand for their
// conjugates too (weight 2).
template <int LOGN>
__global__ void __launch_bounds__(RegTiles<1 << LOGN>::XT) k_fft_x_power_reg(
    const float2* __restrict__ spec, const float2* __restrict__ tw, int nb,
    double* __restrict__ partials) {
  constexpr int N = 1 << LOGN;
  constexpr int R1 = Split<N>::R1, R2 = Split<N>::R2;
  constexpr int TC = RegTiles<N>::TC;
  constexpr int XT = RegTiles<N>::XT;
  constexpr int XF = R2 * (R1 + 1);
  constexpr int NA = TC * R2, NB = TC * R1;
  constexpr int PA = (NA + XT - 1) / XT, PB = (NB + XT - 1) / XT;
  __shared__ float2 ex[TC * XF];
  __shared__ float2 tws[N];
  __shared__ double bins[2 * (N / 2 + 1)];
  const int tid = threadIdx.x;
  // the blocks that share a 128-byte line of a column run on one XCD, as in
  // the Poisson x pass (one L2 fetch of each line instead of one per block)
  const int b = (int)xcd_block(blockIdx.x, gridDim.x, RegTiles<N>::XG);
  const int kz = b / (N / TC);
  const int y0 = (b % (N / TC)) * TC;
  auto at = [&](int x, int c) -> float2 { return spec[((size_t)kz * N + x) * N + y0 + c]; };
  float2 v[PA][R1];
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * XT;
    if (NA % XT == 0 || it < NA) {
      int c, n2;
      x_item<TC, R2>(it, c, n2);
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) v[p][n1] = at(R2 * n1 + n2, c);
    }
  }
  for (int k = tid; k < N; k += XT) tws[k] = tw[k];
  for (int k = tid; k < 2 * (N / 2 + 1); k += XT) bins[k] = 0.0;
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PA; ++p) {
    const int it = tid + p * XT;
    if (NA % XT == 0 || it < NA) {
      int c, n2;
      x_item<TC, R2>(it, c, n2);
      fft_first<N, R1, false>(v[p], n2, tws);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) ex[c * XF + n2 * (R1 + 1) + k1] = v[p][k1];
    }
  }
  __syncthreads();
  const double wz = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
#pragma unroll
  for (int p = 0; p < PB; ++p) {
    const int it = tid + p * XT;
    if (NB % XT == 0 || it < NB) {
      int c, k1;
      x_item<TC, R1>(it, c, k1);
      float2 u[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) u[n2] = ex[c * XF + n2 * (R1 + 1) + k1];
      dft_reg<R2, false, N / R2>(u, tws);
      const int ky = y0 + c;
      const int my = ky <= N / 2 ? ky : ky - N;
      const int myz = my * my + kz * kz;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int kx = k1 + R1 * k2;
        const int mx = kx <= N / 2 ? kx : kx - N;
        const int m2 = mx * mx + myz;
        // shell index: the integer bin with (2 bin - 1)^2 <= 4 m2 < (2 bin + 1)^2
        int bin = (int)(sqrtf((float)m2) + 0.5f);
        if ((2 * bin + 1) * (2 * bin + 1) <= 4 * m2) ++bin;
        if (bin > 0 && (2 * bin - 1) * (2 * bin - 1) > 4 * m2) --bin;
        if (bin >= 1 && bin <= nb) {
          const double re = (double)u[k2].x, im = (double)u[k2].y;
          atomicAdd(&bins[2 * bin], wz * (re * re + im * im));
          atomicAdd(&bins[2 * bin + 1], wz);
        }
      }
    }
  }
  __syncthreads();
  double* out = partials + (size_t)b * 2 * (nb + 1);
  for (int k = tid; k < 2 * (nb + 1); k += XT) out[k] = bins[k];
}

// out[j] = sum over blocks of partials[block][j], j < ncomp: one block per j.
__global__ void __launch_bounds__(kBlock) k_sum_columns(const double* __restrict__ partials,
                                                        int nblocks, int ncomp,
                                                        double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int j = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) t += partials[(size_t)b * ncomp + j];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

hipError_t launch_fft_x_green(int logn, float2* spec, const float2* tw, const float* s2,
                              float green_scale, hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                      \
  {                                                                                 \
    constexpr int N_ = 1 << LN;                                                     \
    dim3 g((N_ / 2 + 1) * (N_ / RegTiles<N_>::TC), bt.count);                       \
    hipLaunchKernelGGL((k_fft_x_green_reg<LN>), g, dim3(RegTiles<N_>::XT), 0, s, spec, tw, s2, \
                       green_scale, bt);                                            \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

int power_blocks(int logn) {
  switch (logn) {
#define B_(LN) \
    case LN: return ((1 << LN) / 2 + 1) * ((1 << LN) / RegTiles<(1 << LN)>::TC);
    B_(4) B_(5) B_(6) B_(7) B_(8) B_(9)
#undef B_
    default: return 0;
  }
}

hipError_t launch_fft_x_power(int logn, const float2* spec, const float2* tw, int nb,
                              double* partials, double* out, hipStream_t s) {
  if (nb < 1 || nb > (1 << logn) / 2) return hipErrorInvalidValue;
#define L_(LN)                                                                      \
  {                                                                                 \
    constexpr int N_ = 1 << LN;                                                     \
    dim3 g((N_ / 2 + 1) * (N_ / RegTiles<N_>::TC));                                 \
    hipLaunchKernelGGL((k_fft_x_power_reg<LN>), g, dim3(RegTiles<N_>::XT), 0, s, spec, tw, nb, \
                       partials);                                                   \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  const int ncomp = 2 * (nb + 1);
  hipLaunchKernelGGL(k_sum_columns, dim3(ncomp), dim3(kBlock), 0, s, partials,
                     power_blocks(logn), ncomp, out);
  return hipGetLastError();
}

hipError_t launch_c2r_z(int logn, const float2* spec, const float2* tw, float* out,
                        hipStream_t s, const Batch& bt) {
#define L_(LN)                                                                  \
  {                                                                             \
    constexpr int N_ = 1 << LN;                                                 \
    dim3 g(N_ * (N_ / Tiles<N_>::TZ), bt.count);                                \
    hipLaunchKernelGGL((k_c2r_z<LN>), g, dim3(kZBlock), 0, s, spec, tw, out, bt); \
  }
  FDM_LOGN_SWITCH(logn, L_)
#undef L_
  return hipGetLastError();
}

}  // namespace fdm
