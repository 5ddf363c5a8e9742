// Internal declarations shared by the HIP translation units of libfdmpm.
// Kernels live next to their launchers; the host API (api.hip) calls the
// launchers only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
#ifndef FDM_GATHER_BLOCK
#define FDM_GATHER_BLOCK 512
#endif
constexpr int kGatherBlock = FDM_GATHER_BLOCK;  // threads per block of the tiled gather
#ifndef FDM_GATHER_PREFETCH
#define FDM_GATHER_PREFETCH 1
#endif
// Particles whose loads a tiled-gather thread keeps in flight ahead of the
// one it processes.
constexpr int kGatherPrefetch = FDM_GATHER_PREFETCH;
constexpr int kMassShift = 40;            // one particle = 2^40 integer mass units

// Particle tiles of the sort, the tiled deposit and the tiled gather:
// 2^kTileLX x 2^kTileLY x 2^kTileLZ cells (z clamped to the mesh size).
#ifndef FDM_TILE_LX
#define FDM_TILE_LX 3
#endif
#ifndef FDM_TILE_LY
#define FDM_TILE_LY 3
#endif
#ifndef FDM_TILE_LZ
#define FDM_TILE_LZ 5
#endif
constexpr int kTileLX = FDM_TILE_LX, kTileLY = FDM_TILE_LY, kTileLZ = FDM_TILE_LZ;
// Halo cells around a tile in the LDS windows of the tiled gather (the
// interpolation stencil of particles that drifted up to kGatherHalo cells
// out of their tile is still in LDS) and of the tiled deposit (the same for
// deposits that land up to kDepHalo cells out of the tile).
#ifndef FDM_GATHER_HALO
#define FDM_GATHER_HALO 0
#endif
#ifndef FDM_DEP_HALO
#define FDM_DEP_HALO 1
#endif
constexpr int kGatherHalo = FDM_GATHER_HALO, kDepHalo = FDM_DEP_HALO;
// The fused gather-deposit counts the particles whose deposit fell outside
// their chunk's window ("strays") in kStraySlices counters, one 128-byte line
// apart, stored right after the mass mesh (cleared with it every step).
constexpr int kStraySlices = 16;
constexpr int kStrayStride = 32;   // unsigned counters between slices
constexpr size_t kStrayBytes = 4 * kStraySlices * kStrayStride;
// A tile's particles are processed in chunks of at most kChunk per block, so
// heavily populated tiles spread over many blocks.
#ifndef FDM_CHUNK
#define FDM_CHUNK 8192
#endif
constexpr int kChunk = FDM_CHUNK;
// The sort counts each tile in kSlices sub-counters (chosen by block) to
// spread same-address atomics on densely populated tiles.
constexpr int kSlices = 16;
// Counters of one slice are count_stride(tiles) apart (a multiple of 32
// counters: the slices of a tile sit in different 128-byte lines).
__host__ __device__ constexpr int count_stride(int tiles) { return (tiles + 31) & ~31; }
// Blocks of the two scan kernels (256 tiles each), and their scratch of two
// counters per block.
__host__ __device__ constexpr int scan_blocks(int tiles) { return (tiles + 255) / 256; }
__host__ __device__ constexpr int tile_lx(int logn) { return logn < kTileLX ? logn : kTileLX; }
__host__ __device__ constexpr int tile_ly(int logn) { return logn < kTileLY ? logn : kTileLY; }
__host__ __device__ constexpr int tile_lz(int logn) { return logn < kTileLZ ? logn : kTileLZ; }
__host__ __device__ constexpr int tile_count(int logn) {
  return (1 << (logn - tile_lx(logn))) * (1 << (logn - tile_ly(logn))) *
         (1 << (logn - tile_lz(logn)));
}

// Workgroups of a launch go to the eight XCDs in turn (workgroup b to XCD
// b mod 8), each XCD with its own L2.  xcd_block renumbers them so that each
// XCD takes `group` consecutive logical blocks per round: blocks that share
// halo cells or cache lines then share an L2 and run at about the same time.
// A bijection on [0, used); blocks from the last whole round on keep their
// number (also those >= used).  group 0 leaves the numbering alone.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned used, unsigned group) {
  if (group == 0) return b;
  const unsigned span = kXcds * group;
  if (b >= used / span * span) return b;
  const unsigned r = b % span;
  return b - r + (r % kXcds) * group + r / kXcds;
}
// Tiled launches take eight chunks at a time (a row of tiles along z at
// N = 256: their windows share halo lines): 4-6 us less per gather at 256^3;
// one contiguous run per XCD made the gather of a clustered state 15%
// slower (uneven work per XCD) and the Q stencil 8% slower.  (The x pass of
// the FFT groups its blocks by the 128-byte lines they share.)
#ifndef FDM_XCD_TILES
#define FDM_XCD_TILES 8
#endif
// group size for `used` blocks from one of the settings above
__device__ __forceinline__ unsigned xcd_group(int setting, unsigned used) {
  return setting < 0 ? used / kXcds : (unsigned)setting;
}

// Per-slot constants of a batched launch (runs of one mesh size stepping
// together); indexed by blockIdx.y, the slot's position in the launch.
struct SlotConst {
  float fg;         // kick factor on -grad(phi)
  float fq;         // kick factor on -grad(Q)
  double fd_units;  // drift factor times 2^(32 - log2 N) (fixed) or drift factor (float)
  float qcoef;      // -(hbar/m)^2 / 2 in cells^2/time
  float pad;
  double qcoef_d;
};

// Batched launches: grid.y enumerates slots; every workspace pointer of slot
// s is base + s * ws_stride bytes, every particle array base + s * part_stride.
// The default (slots == nullptr) is a single run in slot 0.
struct Batch {
  const int* slots = nullptr;
  long long ws_stride = 0;
  long long part_stride = 0;
  const SlotConst* consts = nullptr;
  unsigned count = 1;
};
__device__ __forceinline__ int bslot(const Batch& b) { return b.slots ? b.slots[blockIdx.y] : 0; }
template <class T>
__device__ __forceinline__ T* woff(T* p, const Batch& b, int s) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long long)s * b.ws_stride) : p;
}
template <class T>
__device__ __forceinline__ T* poff(T* p, const Batch& b, int s) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (long long)s * b.part_stride) : p;
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
  float psi_g, psi_q;     // kOutPsi: factors on phi and Q (a batch takes them per slot)
};
// What the Q stencil writes: Q; Q and the FP64 energy partials; or the
// combined kick potential psi = psi_g * phi + psi_q * Q that the next gather
// differentiates (one mesh read per cell there instead of two).
enum QOut : int { kOutQ = 0, kOutEnergy = 1, kOutPsi = 2 };

struct GatherConst {
  float fg;           // factor on -grad(phi)
  float fq;           // factor on -grad(Q)
  double fd_units;    // drift factor times 2^(32 - log2 N) (fixed) or drift factor (float)
  int psi = 0;        // phi holds psi with its factors applied: fg = 1, fq unused, and a
                      // batch's per-slot kick factors are not applied again
  // Energy form (kpart set): phi and Q are interpolated separately; (fg, fq)
  // is the closing half-kick of the previous step, which gives the momentum
  // at the synchronised time, and (og, oq) the opening half-kick of this one.
  // Each block stores its FP64 sum of |p|^2 at the synchronised time in
  // kpart[blockIdx.x] (zero for blocks without particles).
  float og = 0.0f, oq = 0.0f;
  double* kpart = nullptr;
};

// Scale factors that turn the per-block partial sums of one synchronised
// state into K, W, U (pm_energies units).
struct EnergyScale {
  double k, w, u;
};

// ---- deposit.hip
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s, const Batch& bt = Batch());
hipError_t launch_deposit_fixed(const uint32_t* pos, int64_t np, int logn,
                                unsigned long long* mass, hipStream_t s,
                                const Batch& bt = Batch());
hipError_t launch_deposit_f32(const float* pos, int64_t np, int logn, float* acc,
                              hipStream_t s, const Batch& bt = Batch());
// Tiled variants.  The particle sort leaves tile ranges and their chunking:
struct TileMap {
  const unsigned* start;        // [tiles + 1] first particle of each tile
  const unsigned* chunk_start;  // [tiles + 1] first chunk of each tile
  int tiles;
};
// upper bound of the number of chunks: every chunk is full except one per tile
inline unsigned tiled_grid(int64_t np, int tiles) {
  return (unsigned)(tiles + (np + kChunk - 1) / kChunk);
}
// Block b of a tiled launch handles chunk b: tile t with chunk_start[t] <= b <
// chunk_start[t + 1] and particles [start[t] + j kChunk, ...) of it,
// j = b - chunk_start[t].  Returns false for blocks beyond the last chunk
// (the same answer for every thread of the block).
__device__ __forceinline__ bool chunk_of(const TileMap& tm, int& tile, unsigned& lo,
                                         unsigned& hi) {
  __shared__ int s_tile;
  __shared__ unsigned s_chunk;
  if (threadIdx.x == 0) {
    const unsigned used = tm.chunk_start[tm.tiles];
    const unsigned b = xcd_block(blockIdx.x, used, xcd_group(FDM_XCD_TILES, used));
    int t = -1;
    if (b < used) {
      int l = 0, r = tm.tiles;  // first index with chunk_start > b lies in (l, r]
      while (r - l > 1) {
        const int m = (l + r) >> 1;
        if (tm.chunk_start[m] <= b) l = m; else r = m;
      }
      t = l;
    }
    s_tile = t;
    s_chunk = b;
  }
  __syncthreads();
  tile = s_tile;
  if (tile < 0) return false;
  const unsigned j = s_chunk - tm.chunk_start[tile];
  lo = tm.start[tile] + j * (unsigned)kChunk;
  const unsigned end = tm.start[tile + 1];
  hi = lo + (unsigned)kChunk < end ? lo + (unsigned)kChunk : end;
  return true;
}

hipError_t launch_deposit_fixed_tiled(const uint32_t* pos, int64_t np, int logn,
                                      const TileMap& tm, unsigned long long* mass,
                                      hipStream_t s, const Batch& bt = Batch());
hipError_t launch_deposit_f32_tiled(const float* pos, int64_t np, int logn, const TileMap& tm,
                                    float* acc, hipStream_t s, const Batch& bt = Batch());

// ---- sort.hip
// counts: [kSlices][count_stride(tiles)]; key[i] = tile * kSlices + slice
hipError_t launch_sort_count(bool fixed, const void* pos, int64_t np, int logn,
                             unsigned* counts, unsigned* key, unsigned* rank, hipStream_t s,
                             const Batch& bt = Batch());
// slice_start: [tiles * kSlices + 1]; tile_start, chunk_start: [tiles + 1];
// sums: scratch of 2 * scan_blocks(tiles) counters
hipError_t launch_sort_scan(const unsigned* counts, int tiles, unsigned* sums,
                            unsigned* slice_start, unsigned* tile_start, unsigned* chunk_start,
                            hipStream_t s, const Batch& bt = Batch());
hipError_t launch_sort_scatter(const void* pos, const float* vel, const int* ids, int64_t np,
                               const unsigned* key, const unsigned* rank,
                               const unsigned* slice_start, uint32_t* pos_out, float* vel_out,
                               int* ids_out, hipStream_t s, const Batch& bt = Batch());
hipError_t launch_sort_copy(uint32_t* pos, float* vel, const uint32_t* pos_tmp,
                            const float* vel_tmp, int64_t np, hipStream_t s, const Batch& bt);

// ---- fft.hip
// Forward transform of the density contrast and Poisson solve, written as
// five passes over the half-spectrum spec[kz][kx][ky] (kz = 0..N/2).
hipError_t launch_r2c_z(int logn, int src, const void* in, float* delta_out,
                        float2* spec, const float2* tw, DeltaConv conv, hipStream_t s,
                        const Batch& bt = Batch());
hipError_t launch_fft_y(int logn, float2* spec, const float2* tw, bool inverse,
                        hipStream_t s, const Batch& bt = Batch());
hipError_t launch_fft_x_green(int logn, float2* spec, const float2* tw, const float* s2,
                              float green_scale, hipStream_t s, const Batch& bt = Batch());
hipError_t launch_c2r_z(int logn, const float2* spec, const float2* tw, float* out,
                        hipStream_t s, const Batch& bt = Batch());

// ---- stencil.hip
hipError_t launch_qpot(int logn, bool fixed, int out, const float* delta,
                       const long long* mass, const float* phi, float* q,
                       const QConst& qc, double* partials, hipStream_t s,
                       const Batch& bt = Batch());
int qpot_blocks(int logn);
hipError_t launch_reduce(const double* partials, int nblocks, int ncomp, double* out,
                         hipStream_t s, const Batch& bt = Batch());
// out[0..3] = K, W, U, K + W + U from the stencil's (delta phi, gradient)
// partials of nq blocks and the gather's |p|^2 partials of nk blocks, each
// summed in a fixed order and scaled by sc.
hipError_t launch_energy_row(const double* qpart, int nq, const double* kpart, int nk,
                             EnergyScale sc, double* out, hipStream_t s);

// ---- gather.hip
// wide (fixed point, fused deposit on a sorted context): the larger windows
// of k_gather_tiled's WIDE form.  pos_out, vel_out (kick without drift on a
// sorted context): write the kicked velocities and a copy of the positions
// there instead of in place.
hipError_t launch_gather(bool fixed, bool has_q, bool drift, int logn, void* pos,
                         float* vel, const float* phi, const float* q, int64_t np,
                         const GatherConst& gc, const TileMap* tm, void* deposit_mass,
                         hipStream_t s, const Batch& bt = Batch(), bool wide = false,
                         void* pos_out = nullptr, float* vel_out = nullptr);
hipError_t preload_wide(int logn);
hipError_t launch_force(bool fixed, bool has_q, int logn, const void* pos,
                        const float* phi, const float* q, int64_t np, float fg, float fq,
                        float* acc, hipStream_t s);
hipError_t launch_kinetic(const float* vel, int64_t np, double* partials, int nblocks,
                          hipStream_t s, const Batch& bt = Batch());
int kinetic_blocks(int64_t np);
// Blocks of a gather launch (the number of |p|^2 partials of its energy form).
unsigned gather_blocks(int64_t np, const TileMap* tm);

// ---- fft.hip, power spectrum: the forward x transform of a spectrum after
// r2c_z and the forward y pass, |X|^2 binned into shells b = 1..nb of integer
// mode number; per-block bins go to partials (power_blocks(logn) x 2 (nb + 1)
// doubles), their sums to out[2 b] (power) and out[2 b + 1] (mode weight).
int power_blocks(int logn);
hipError_t launch_fft_x_power(int logn, const float2* spec, const float2* tw, int nb,
                              double* partials, double* out, hipStream_t s);

// ---- spline.hip: the spline kernel of Eq. (15) with smoothing length h
// (cells); mass (N^3, zeroed by the caller) receives sum_i W(|x_j - q_i|)
// in units of 2^-40 particle masses per cell volume (the units of the CIC
// mass mesh); acc is [3][np].
// With tm (sorted context) the deposit sums each tile chunk in LDS first.
hipError_t launch_spline_deposit(bool fixed, int logn, const void* pos, int64_t np, float h,
                                 const TileMap* tm, unsigned long long* mass, hipStream_t s);
hipError_t launch_spline_qforce(bool fixed, int logn, const void* pos, int64_t np,
                                const float* q, float h, float* acc, hipStream_t s);
// The spline step's half-kick (v += fg g_phi + fq g_q) and drift (x += fd v).
hipError_t launch_spline_kick(float* vel, const float* gphi, const float* gq, int64_t np,
                              float fg, float fq, hipStream_t s);
hipError_t launch_spline_drift(bool fixed, int logn, void* pos, const float* vel, int64_t np,
                               double fd, hipStream_t s);

// ---- diag.hip
// Grid diagnostics: node momenta of one velocity component (FP64 atomics into
// mom, which the caller zeroes), per-block sums of mom^2 / mass over nodes
// with mass, and per-block (sum of squared relative differences, node count).
int diag_blocks(int64_t n, int max_blocks);
// With tm (sorted context) the tiled form sums each chunk in LDS first.
hipError_t launch_deposit_momentum(bool fixed, int logn, const void* pos, int64_t np,
                                   const float* v, double* mom, const TileMap* tm,
                                   hipStream_t s);
hipError_t launch_bulk_nodes(bool fixed, const void* mass, const double* mom, int64_t ncell,
                             double* partials, int nblocks, hipStream_t s);
hipError_t launch_rel_diff_nodes(bool fixed, const void* mass_a, const void* mass_b,
                                 int64_t ncell, double* partials, int nblocks, hipStream_t s);

}  // namespace fdm
