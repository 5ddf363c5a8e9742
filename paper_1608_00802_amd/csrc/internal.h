// Internal declarations shared by the HIP translation units of libfdmpm.
// Kernels live next to their launchers; the host API (api.hip) calls the
// launchers only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Dispatch a runtime log2(N) to a template instantiation (N = 16..512).
#define FDM_LOGN_SWITCH(logn, MACRO) \
  switch (logn) {                    \
    case 4: MACRO(4); break;         \
    case 5: MACRO(5); break;         \
    case 6: MACRO(6); break;         \
    case 7: MACRO(7); break;         \
    case 8: MACRO(8); break;         \
    case 9: MACRO(9); break;         \
    default: return hipErrorInvalidValue; \
  }

namespace fdm {

constexpr int kBlock = 256;               // threads per block of the streaming kernels
constexpr int kMassShift = 40;            // one particle = 2^40 integer mass units

// Particle tiles of the sort, the tiled deposit and the tiled gather:
// 2^kTileLX x 2^kTileLY x 2^kTileLZ cells (z clamped to the mesh size).
constexpr int kTileLX = 2, kTileLY = 2, kTileLZ = 5;
__host__ __device__ constexpr int tile_lz(int logn) { return logn < kTileLZ ? logn : kTileLZ; }
__host__ __device__ constexpr int tile_count(int logn) {
  return (1 << (logn - kTileLX)) * (1 << (logn - kTileLY)) * (1 << (logn - tile_lz(logn)));
}

// Sources of the forward z-pass.
enum ZSource : int {
  kSrcMass64 = 0,   // exact integer mass (fixed-point form)
  kSrcAcc32 = 1,    // float CIC accumulator (plain FP32 form)
  kSrcDelta = 2     // caller-provided density contrast
};

struct DeltaConv {
  long long mbar;     // mean integer mass per cell (fixed form)
  double dmbar;       // same, as double
  float acc_norm;     // N^3 / Np (float form)
};

struct QConst {
  float coef;             // -(hbar/m)^2 / 2 in cells^2/time
  float floor_f;          // rho floor (units of the mean)
  float s_floor;          // sqrt(floor) - 1
  double coef_d;          // coef in FP64
  double floor_d;
  double fp64_below;      // FP64 path threshold (fixed form; <= 0 disables)
  long long mbar;         // mean integer mass per cell
  double inv_mbar;        // 1 / mbar
};

struct GatherConst {
  float fg;           // factor on -grad(phi)
  float fq;           // factor on -grad(Q)
  double fd_units;    // drift factor times 2^(32 - log2 N) (fixed) or drift factor (float)
};

// ---- deposit.hip
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_deposit_fixed(const uint32_t* pos, int64_t np, int logn,
                                unsigned long long* mass, hipStream_t s);
hipError_t launch_deposit_f32(const float* pos, int64_t np, int logn, float* acc,
                              hipStream_t s);
// tiled variants: particles sorted by tile, tile ranges start[0..tiles]
hipError_t launch_deposit_fixed_tiled(const uint32_t* pos, int64_t np, int logn,
                                      const unsigned* start, unsigned long long* mass,
                                      hipStream_t s);
hipError_t launch_deposit_f32_tiled(const float* pos, int64_t np, int logn,
                                    const unsigned* start, float* acc, hipStream_t s);

// ---- sort.hip
hipError_t launch_sort_count(bool fixed, const void* pos, int64_t np, int logn,
                             unsigned* counts, unsigned* key, unsigned* rank, hipStream_t s);
hipError_t launch_sort_scan(const unsigned* counts, int n, unsigned* start, hipStream_t s);
hipError_t launch_sort_scatter(const void* pos, const float* vel, const int* ids, int64_t np,
                               const unsigned* key, const unsigned* rank, const unsigned* start,
                               uint32_t* pos_out, float* vel_out, int* ids_out, hipStream_t s);

// ---- fft.hip
// Forward transform of the density contrast and Poisson solve, written as
// five passes over the half-spectrum spec[kz][kx][ky] (kz = 0..N/2).
hipError_t launch_r2c_z(int logn, int src, const void* in, float* delta_out,
                        float2* spec, const float2* tw, DeltaConv conv, hipStream_t s);
hipError_t launch_fft_y(int logn, float2* spec, const float2* tw, bool inverse,
                        hipStream_t s);
hipError_t launch_fft_x_green(int logn, float2* spec, const float2* tw, const float* s2,
                              float green_scale, hipStream_t s);
hipError_t launch_c2r_z(int logn, const float2* spec, const float2* tw, float* out,
                        hipStream_t s);

// ---- stencil.hip
hipError_t launch_qpot(int logn, bool fixed, bool energy, const float* delta,
                       const long long* mass, const float* phi, float* q,
                       const QConst& qc, double* partials, hipStream_t s);
int qpot_blocks(int logn);
hipError_t launch_reduce(const double* partials, int nblocks, int ncomp, double* out,
                         hipStream_t s);

// ---- gather.hip
hipError_t launch_gather(bool fixed, bool has_q, bool drift, int logn, void* pos,
                         float* vel, const float* phi, const float* q, int64_t np,
                         const GatherConst& gc, const unsigned* tile_start, hipStream_t s);
hipError_t launch_force(bool fixed, bool has_q, int logn, const void* pos,
                        const float* phi, const float* q, int64_t np, float fg, float fq,
                        float* acc, hipStream_t s);
hipError_t launch_kinetic(const float* vel, int64_t np, double* partials, int nblocks,
                          hipStream_t s);
int kinetic_blocks(int64_t np);

}  // namespace fdm
