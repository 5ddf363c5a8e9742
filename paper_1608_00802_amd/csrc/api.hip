// Host side of libfdmpm: parameter checks, workspace carving, FP64 time-step
// factors and the launch sequence of one particle-mesh step.  Implements the
// C ABI declared in include/fdmpm.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/fdmpm.h"
#include "internal.h"

using namespace fdm;

namespace {

enum KernelClass : int {
  kcFill, kcDeposit, kcR2C, kcFftY, kcFftX, kcFftYInv, kcC2R, kcQpot, kcGatherKD, kcKick,
  kcForce, kcReduce, kcKinetic, kcSortCount, kcSortScan, kcSortScatter, kcSortCopy,
  kcMomentum, kcDiagNodes, kcPower, kcSpline, kcSplineForce, kcEnergyRow, kcCount
};
const char* const kKernelNames[kcCount] = {
    "fill_zero", "deposit", "r2c_z", "fft_y", "fft_x_green", "fft_y_inv", "c2r_z",
    "qpot", "gather_kick_drift", "kick", "force", "reduce", "kinetic", "sort_count",
    "sort_scan", "sort_scatter", "sort_copy", "momentum_deposit", "diag_nodes", "fft_x_power", "spline_deposit",
    "spline_qforce", "energy_row"};

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Rec {
    int kc;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  double ms[kcCount] = {};
  int64_t launches[kcCount] = {};
};

}  // namespace

struct pm_ctx {
  pm_params p;
  int N, logn, B;
  int64_t np;
  size_t ncell;
  hipStream_t stream;
  bool fixed;
  bool has_q;
  // constants in cell units
  double S;          // static: 4 pi G rho_bar; comoving: 1.5 Om H0^2
  double hm;         // hbar/m in cells^2/time
  DeltaConv conv;
  QConst qc;
  // workspace
  void* mass;        // int64 [N^3] (fixed) or float [N^3] accumulator (fp32)
  float* delta;
  float* phi;
  float* q;
  float2* spec;
  float2* tw;
  float* s2;
  double* partials;  // energy partial sums
  double* kpart;     // |p|^2 partial sums of the energy form of the gather
  double* result;    // reduced energies (device)
  unsigned* tile_counts;  // [kSlices][count_stride(tiles)]
  unsigned* scan_sums;    // [2 * scan_blocks(tiles)]
  unsigned* slice_start;  // [tiles * kSlices + 1]
  unsigned* tile_start;   // [tiles + 1], valid once sorted
  unsigned* chunk_start;  // [tiles + 1]
  TileMap tmap;
  unsigned* sort_key;
  unsigned* sort_rank;
  uint32_t* pos_tmp;
  float* vel_tmp;
  int* ids_tmp;
  int tiles;
  bool sorted;       // tile_start describes a partition of the particles by tile
  int q_blocks;
  int k_blocks;
  bool have_delta;   // delta in the workspace was made by pm_deposit
  bool have_phi;
  bool have_q;
  bool fields_at_pos;  // phi, q correspond to the positions left by pm_step
  Timer timer;
  // adaptive sort interval (PM_SORT_AUTO): a sampled stray count of the
  // fused deposit is copied to pinned memory and read once it has arrived
  unsigned* h_stat = nullptr;   // kStraySlices * kStrayStride counters
  hipEvent_t ev_stat = nullptr;
  bool stat_pending = false;
  int stat_age = 0;             // steps since the sort at the sampled step
  // adaptive sort interval: it starts at the longest and shortens once the
  // strays at the end of an interval call for it
  int sort_interval = 32;
  int sort_base = 32;           // the interval the stray model gives (before the wide windows)
  bool wide_windows = false;    // aged steps take the wide gather windows
  int since_sort = 1 << 30;     // steps since the last sort
};


struct pm_batch {
  pm_ctx base;                 // layout and constants of slot 0
  int slots;
  size_t slot_stride;          // bytes between slot regions
  size_t header;               // bytes before slot 0
  char* ws;                    // workspace start
  int* d_slots;                // device list of active slots
  SlotConst* d_consts;         // device [(max steps + 1) * slots]
  std::vector<double> box, hm;  // per slot, hm in cells^2/time
  std::vector<char> fields_ok, sorted;
  // pinned staging of the per-call slot list and constant table (two
  // buffers, so the host fills one while the other's copy is queued);
  // pageable sources would make every call wait for the stream
  char* h_stage[2] = {nullptr, nullptr};
  hipEvent_t h_done[2] = {nullptr, nullptr};
  int h_next = 0;
  // PM_BATCH_GRAPH: executable graphs of the kernels of captured calls, by
  // shape (listed slots, steps, flags, every listed slot sorted on entry)
  std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

int ilog2_exact(int n) {
  if (n <= 0 || (n & (n - 1)) != 0) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

struct Layout {
  size_t mass, delta, phi, q, spec, tw, s2, partials, kpart, result, tile_counts, scan_sums,
      slice_start, tile_start, chunk_start, sort_key, sort_rank, pos_tmp, vel_tmp, ids_tmp, total;
};

Layout layout_for(const pm_params& p) {
  const size_t n = (size_t)p.n_mesh;
  const size_t nc = n * n * n;
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.mass = take(8 * nc + kStrayBytes);   // mesh, then the stray counters
  L.delta = take(4 * nc);
  L.phi = take(4 * nc);
  L.q = take(4 * nc);
  L.spec = take(8 * (n / 2 + 1) * n * n);
  L.tw = take(8 * n);
  L.s2 = take(4 * n);
  const size_t qb = nc / kBlock;
  L.partials = take(8 * (2 * qb + 1024));
  const int logn = ilog2_exact(p.n_mesh);
  const size_t tiles = logn > 0 ? (size_t)tile_count(logn) : 1;
  const size_t np = (size_t)(p.n_part > 0 ? p.n_part : 1);
  // one |p|^2 partial per gather block: at most 65536 blocks unsorted, one
  // per chunk of a tile sorted
  L.kpart = take(8 * std::max<size_t>(65536, tiles + (np + kChunk - 1) / kChunk));
  L.result = take(8 * 16);
  L.tile_counts = take(4 * (size_t)kSlices * count_stride((int)tiles));
  L.scan_sums = take(8 * (size_t)scan_blocks((int)tiles));
  L.slice_start = take(4 * (tiles * kSlices + 1));
  L.tile_start = take(4 * (tiles + 1));
  L.chunk_start = take(4 * (tiles + 1));
  L.sort_key = take(4 * np);
  L.sort_rank = take(4 * np);
  L.pos_tmp = take(12 * np);
  L.vel_tmp = take(12 * np);
  L.ids_tmp = take(4 * np);
  L.total = off;
  return L;
}

pm_status check_params(const pm_params* p) {
  if (!p) return PM_EINVAL;
  const int logn = ilog2_exact(p->n_mesh);
  if (logn < 4 || logn > 9) return PM_EUNSUPPORTED;
  if (p->precision != PM_FP32 && p->precision != PM_FIXED32) return PM_EINVAL;
  if (p->n_part < 1) return PM_EINVAL;
  if (!(p->box > 0.0) || !isfinite(p->box)) return PM_EINVAL;
  if (p->comoving != 0 && p->comoving != 1) return PM_EINVAL;
  if (p->reserved0 != 0) return PM_EINVAL;
  if (!(p->hbar_over_m >= 0.0) || !isfinite(p->hbar_over_m)) return PM_EINVAL;
  if (!(p->rho_floor > 0.0) || !isfinite(p->rho_floor)) return PM_EINVAL;
  if (!(p->rho_fp64_below >= 0.0) || !isfinite(p->rho_fp64_below)) return PM_EINVAL;
  if (p->comoving) {
    if (!(p->omega_m > 0.0) || !(p->omega_l >= 0.0) || !(p->h0 > 0.0)) return PM_EINVAL;
    if (!isfinite(p->omega_m) || !isfinite(p->omega_l) || !isfinite(p->h0)) return PM_EINVAL;
  } else {
    if (!(p->four_pi_G_rhobar >= 0.0) || !isfinite(p->four_pi_G_rhobar)) return PM_EINVAL;
  }
  // the mean integer mass per cell 2^40 Np / N^3 (deposit units) fits int64
  if ((double)p->n_part * ldexp(1.0, kMassShift - 3 * logn) > 4.0e18) return PM_EINVAL;
  if (p->precision == PM_FIXED32) {
    // mean integer mass per cell must be an integer: 2^40 Np / N^3
    if (3 * logn > kMassShift) return PM_EUNSUPPORTED;
    // a cell can hold at least 2^20 times the mean mass without overflow:
    // mean = 2^40 Np / N^3 <= 2^43
    if ((double)p->n_part > 8.0 * (double)p->n_mesh * p->n_mesh * p->n_mesh) return PM_EINVAL;
  }
  return PM_OK;
}

pm_status dev(hipError_t e) { return e == hipSuccess ? PM_OK : PM_EDEVICE; }

#define PM_TRY(expr)                   \
  do {                                 \
    pm_status st_ = (expr);            \
    if (st_ != PM_OK) return st_;      \
  } while (0)

hipEvent_t take_event(Timer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch through f(); with timing on, bracket it by two events on the stream.
template <class F>
pm_status timed(pm_ctx* c, int kc, F&& f) {
  if (!c->timer.on) return dev(f());
  hipEvent_t a = take_event(c->timer), b = take_event(c->timer);
  if (!a || !b) return PM_EDEVICE;
  if (hipEventRecord(a, c->stream) != hipSuccess) return PM_EDEVICE;
  const hipError_t e = f();
  if (hipEventRecord(b, c->stream) != hipSuccess) return PM_EDEVICE;
  c->timer.pending.push_back({kc, a, b});
  return dev(e);
}

// ------------------------------------------------------------ FP64 quadrature
// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
struct Gauss {
  static constexpr int n = 16;
  double x[n], w[n];
  Gauss() {
    for (int i = 0; i < n; ++i) {
      double z = cos(M_PI * (i + 0.75) / (n + 0.5));
      double pp = 0.0;
      for (int it = 0; it < 100; ++it) {
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0);
        const double dz = p1 / pp;
        z -= dz;
        if (fabs(dz) < 1e-16) break;
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
  }
};

const Gauss& gauss() {
  static const Gauss g;
  return g;
}

double hubble(const pm_params& p, double a) {
  return p.h0 * sqrt(p.omega_m / (a * a * a) + p.omega_l);
}

// int_{a0}^{a1} da / (a^pw H(a)), composite Gauss-Legendre in s = ln a
double a_integral(const pm_params& p, double a0, double a1, int pw) {
  const Gauss& g = gauss();
  const double s0 = log(a0), s1 = log(a1);
  int m = (int)ceil(fabs(s1 - s0) / 0.02);
  if (m < 1) m = 1;
  const double hseg = (s1 - s0) / m;
  double total = 0.0;
  for (int k = 0; k < m; ++k) {
    const double c = s0 + (k + 0.5) * hseg;
    double part = 0.0;
    for (int i = 0; i < Gauss::n; ++i) {
      const double s = c + 0.5 * hseg * g.x[i];
      const double a = exp(s);
      part += g.w[i] * a / (pow(a, pw) * hubble(p, a));  // da = a ds
    }
    total += 0.5 * hseg * part;
  }
  return total;
}

struct Kick {
  double g, q;
};

Kick kick(const pm_params& p, double t0, double t1) {
  if (!p.comoving) return {t1 - t0, t1 - t0};
  return {a_integral(p, t0, t1, 2), a_integral(p, t0, t1, 3)};
}

double drift(const pm_params& p, double t0, double t1) {
  if (!p.comoving) return t1 - t0;
  return a_integral(p, t0, t1, 3);
}

double midpoint(const pm_params& p, double t0, double t1) {
  return p.comoving ? sqrt(t0 * t1) : 0.5 * (t0 + t1);
}

// ------------------------------------------------------------ launch sequences
pm_status run_deposit(pm_ctx* c, const void* pos) {
  PM_TRY(timed(c, kcFill, [&] { return launch_fill_zero(c->mass, 8 * c->ncell + kStrayBytes, c->stream); }));
  return timed(c, kcDeposit, [&] {
    if (c->fixed && c->sorted)
      return launch_deposit_fixed_tiled(static_cast<const uint32_t*>(pos), c->np, c->logn,
                                        c->tmap, static_cast<unsigned long long*>(c->mass),
                                        c->stream);
    if (c->fixed)
      return launch_deposit_fixed(static_cast<const uint32_t*>(pos), c->np, c->logn,
                                  static_cast<unsigned long long*>(c->mass), c->stream);
    if (c->sorted)
      return launch_deposit_f32_tiled(static_cast<const float*>(pos), c->np, c->logn, c->tmap,
                                      static_cast<float*>(c->mass), c->stream);
    return launch_deposit_f32(static_cast<const float*>(pos), c->np, c->logn,
                              static_cast<float*>(c->mass), c->stream);
  });
}

// Forward z-pass from the context's mass mesh (or from a given delta),
// remaining passes, potential into c->phi.
pm_status run_poisson(pm_ctx* c, int src, const void* in) {
  PM_TRY(timed(c, kcR2C, [&] {
    return launch_r2c_z(c->logn, src, in, c->delta, c->spec, c->tw, c->conv, c->stream);
  }));
  PM_TRY(timed(c, kcFftY, [&] { return launch_fft_y(c->logn, c->spec, c->tw, false, c->stream); }));
  const double nn = (double)c->N;
  const float gscale = (float)(-c->S * 2.0 / (nn * nn * nn));
  PM_TRY(timed(c, kcFftX, [&] {
    return launch_fft_x_green(c->logn, c->spec, c->tw, c->s2, gscale, c->stream);
  }));
  PM_TRY(timed(c, kcFftYInv, [&] { return launch_fft_y(c->logn, c->spec, c->tw, true, c->stream); }));
  return timed(c, kcC2R, [&] { return launch_c2r_z(c->logn, c->spec, c->tw, c->phi, c->stream); });
}

pm_status run_qpot(pm_ctx* c, const float* delta, bool use_mass, int out,
                   const Kick* psi = nullptr) {
  QConst qc = c->qc;
  if (!use_mass) qc.fp64_below = -1.0;
  if (psi) {
    qc.psi_g = (float)psi->g;
    qc.psi_q = (float)psi->q;
  }
  return timed(c, kcQpot, [&] {
    return launch_qpot(c->logn, c->fixed, out, delta, static_cast<const long long*>(c->mass),
                       c->phi, c->q, qc, c->partials, c->stream);
  });
}

// deposit + Poisson + Q at the given positions, all into the workspace
// (deposit = false: the mass mesh already holds them, from the fused push).
// With psi (and a quantum potential), q receives the kick potential
// psi->g * phi + psi->q * Q for one gather instead of Q; phi stays phi.
pm_status run_fields(pm_ctx* c, const void* pos, bool energy, bool deposit = true,
                     const Kick* psi = nullptr) {
  if (deposit) PM_TRY(run_deposit(c, pos));
  PM_TRY(run_poisson(c, c->fixed ? kSrcMass64 : kSrcAcc32, c->mass));
  c->have_delta = true;
  c->have_phi = true;
  const bool to_psi = psi && c->has_q && !energy;
  if (c->has_q || energy)
    PM_TRY(run_qpot(c, c->delta, true, energy ? kOutEnergy : to_psi ? kOutPsi : kOutQ, psi));
  c->have_q = c->has_q && !to_psi;
  return PM_OK;
}

pm_status copy_out(pm_ctx* c, float* dst, const float* src) {
  if (!dst || dst == src) return PM_OK;
  return dev(hipMemcpyAsync(dst, src, 4 * c->ncell, hipMemcpyDeviceToDevice, c->stream));
}

size_t batch_header(int slots) {
  return align_up(4 * (size_t)slots) + align_up(sizeof(SlotConst) * (PM_BATCH_MAX_STEPS + 1) *
                                                (size_t)slots);
}

// Release a batch's host resources once its queued uploads are done.
void batch_free(pm_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  for (int i = 0; i < 2; ++i) {
    if (b->h_done[i]) {
      (void)hipEventSynchronize(b->h_done[i]);
      (void)hipEventDestroy(b->h_done[i]);
    }
    if (b->h_stage[i]) (void)hipHostFree(b->h_stage[i]);
  }
  delete b;
}

// Fill a context for the workspace region at base (layout_for(*params)),
// upload its constant tables.  params are already checked.
pm_status ctx_setup(pm_ctx* c, const pm_params* params, char* base, hipStream_t stream) {
  const Layout L = layout_for(*params);
  c->p = *params;
  c->N = params->n_mesh;
  c->logn = ilog2_exact(c->N);
  c->B = 32 - c->logn;
  c->np = params->n_part;
  c->ncell = (size_t)c->N * c->N * c->N;
  c->stream = stream;
  c->fixed = params->precision == PM_FIXED32;
  const double dx = params->box / c->N;
  c->hm = params->hbar_over_m / (dx * dx);
  c->has_q = c->hm > 0.0;
  c->S = params->comoving ? 1.5 * params->omega_m * params->h0 * params->h0
                          : params->four_pi_G_rhobar;
  // mean integer mass per cell, 2^40 Np / N^3 (an integer for N <= 512): the
  // units of the fixed-point CIC deposit and, in both precisions, of the
  // spline deposit
  const int sh = kMassShift - 3 * c->logn;
  const long long mbar = (long long)(params->n_part) << (sh > 0 ? sh : 0);
  c->conv.mbar = mbar;
  c->conv.dmbar = (double)mbar;
  c->conv.acc_norm = (float)((double)c->ncell / (double)c->np);
  QConst& qc = c->qc;
  qc.coef_d = -0.5 * c->hm * c->hm;
  qc.coef = (float)qc.coef_d;
  qc.floor_d = params->rho_floor;
  qc.floor_f = (float)params->rho_floor;
  qc.s_floor = (float)(sqrt(params->rho_floor) - 1.0);
  qc.fp64_below = c->fixed ? params->rho_fp64_below : -1.0;
  qc.mbar = mbar;
  qc.inv_mbar = mbar ? 1.0 / (double)mbar : 0.0;
  c->mass = base + L.mass;
  c->delta = reinterpret_cast<float*>(base + L.delta);
  c->phi = reinterpret_cast<float*>(base + L.phi);
  c->q = reinterpret_cast<float*>(base + L.q);
  c->spec = reinterpret_cast<float2*>(base + L.spec);
  c->tw = reinterpret_cast<float2*>(base + L.tw);
  c->s2 = reinterpret_cast<float*>(base + L.s2);
  c->partials = reinterpret_cast<double*>(base + L.partials);
  c->kpart = reinterpret_cast<double*>(base + L.kpart);
  c->result = reinterpret_cast<double*>(base + L.result);
  c->tile_counts = reinterpret_cast<unsigned*>(base + L.tile_counts);
  c->scan_sums = reinterpret_cast<unsigned*>(base + L.scan_sums);
  c->slice_start = reinterpret_cast<unsigned*>(base + L.slice_start);
  c->tile_start = reinterpret_cast<unsigned*>(base + L.tile_start);
  c->chunk_start = reinterpret_cast<unsigned*>(base + L.chunk_start);
  c->sort_key = reinterpret_cast<unsigned*>(base + L.sort_key);
  c->sort_rank = reinterpret_cast<unsigned*>(base + L.sort_rank);
  c->pos_tmp = reinterpret_cast<uint32_t*>(base + L.pos_tmp);
  c->vel_tmp = reinterpret_cast<float*>(base + L.vel_tmp);
  c->ids_tmp = reinterpret_cast<int*>(base + L.ids_tmp);
  c->tiles = tile_count(c->logn);
  c->tmap.start = c->tile_start;
  c->tmap.chunk_start = c->chunk_start;
  c->tmap.tiles = c->tiles;
  c->sorted = false;
  c->q_blocks = qpot_blocks(c->logn);
  c->k_blocks = kinetic_blocks(c->np);
  // constant tables, built in FP64 and rounded once
  std::vector<float2> tw(c->N);
  std::vector<float> s2(c->N);
  for (int k = 0; k < c->N; ++k) {
    const double ang = -2.0 * M_PI * k / c->N;
    tw[k] = make_float2((float)cos(ang), (float)sin(ang));
    const double sn = sin(M_PI * k / c->N);
    s2[k] = (float)(4.0 * sn * sn);
  }
  hipError_t e = hipMemcpyAsync(c->tw, tw.data(), 8 * c->N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->s2, s2.data(), 4 * c->N, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // host vectors die here
  if (e == hipSuccess && !c->has_q) e = launch_fill_zero(c->q, 4 * c->ncell, c->stream);
  return e == hipSuccess ? PM_OK : PM_EDEVICE;
}

}  // namespace

extern "C" {

pm_status pm_sort(pm_ctx* c, void* d_pos, float* d_vel, int32_t* d_ids);

pm_status pm_workspace_bytes(const pm_params* params, size_t* bytes) {
  if (!bytes) return PM_EINVAL;
  PM_TRY(check_params(params));
  *bytes = layout_for(*params).total;
  return PM_OK;
}

pm_status pm_init(const pm_params* params, void* d_workspace, size_t bytes, void* hip_stream,
                  pm_ctx** out) {
  if (!out || !d_workspace) return PM_EINVAL;
  PM_TRY(check_params(params));
  if (((uintptr_t)d_workspace) % kAlign != 0) return PM_EINVAL;
  if (bytes < layout_for(*params).total) return PM_ENOMEM;
  pm_ctx* c = new (std::nothrow) pm_ctx();
  if (!c) return PM_ENOMEM;
  const pm_status st = ctx_setup(c, params, static_cast<char*>(d_workspace),
                                 static_cast<hipStream_t>(hip_stream));
  if (st != PM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return PM_OK;
}

pm_status pm_deposit(pm_ctx* c, const void* d_pos, float* d_delta) {
  if (!c || !d_pos) return PM_EINVAL;
  PM_TRY(run_deposit(c, d_pos));
  // forward z-pass forms delta (and a spectrum the caller did not ask for);
  // a standalone convert would move the same bytes minus the spectrum write
  PM_TRY(timed(c, kcR2C, [&] {
    return launch_r2c_z(c->logn, c->fixed ? kSrcMass64 : kSrcAcc32, c->mass, c->delta, c->spec,
                        c->tw, c->conv, c->stream);
  }));
  c->have_delta = true;
  c->have_phi = false;
  c->fields_at_pos = false;
  return copy_out(c, d_delta, c->delta);
}

pm_status pm_poisson(pm_ctx* c, const float* d_delta, float* d_phi) {
  if (!c) return PM_EINVAL;
  if (d_delta) {
    PM_TRY(run_poisson(c, kSrcDelta, d_delta));
  } else {
    if (!c->have_delta) return PM_ESTATE;
    PM_TRY(run_poisson(c, kSrcDelta, c->delta));
  }
  c->have_phi = true;
  c->fields_at_pos = false;
  return copy_out(c, d_phi, c->phi);
}

pm_status pm_qpot(pm_ctx* c, const float* d_delta, float* d_q) {
  if (!c) return PM_EINVAL;
  if (d_delta) {
    PM_TRY(run_qpot(c, d_delta, false, kOutQ));
  } else {
    if (!c->have_delta) return PM_ESTATE;
    PM_TRY(run_qpot(c, c->delta, c->fixed, kOutQ));
  }
  c->have_q = true;
  c->fields_at_pos = false;
  return copy_out(c, d_q, c->q);
}

pm_status pm_force(pm_ctx* c, const float* d_phi, const float* d_q, const void* d_pos,
                   float* d_acc, double a) {
  if (!c || !d_pos || !d_acc) return PM_EINVAL;
  if (!(a > 0.0) || !isfinite(a)) return PM_EINVAL;
  if (!c->p.comoving && a != 1.0) return PM_EINVAL;
  const float* phi = d_phi ? d_phi : c->phi;
  const float* q = d_q ? d_q : c->q;
  if (!d_phi && !c->have_phi) return PM_ESTATE;
  const bool use_q = d_q != nullptr || (c->has_q && c->have_q);
  if (!d_q && c->has_q && !c->have_q) return PM_ESTATE;
  return timed(c, kcForce, [&] {
    return launch_force(c->fixed, use_q, c->logn, d_pos, phi, q, c->np, (float)(1.0 / a),
                        (float)(1.0 / (a * a)), d_acc, c->stream);
  });
}

// Adaptive sort interval.  After the last fused gather-deposit of an
// interval the stray counters (particles whose deposit fell outside their
// tile's window) are copied to pinned memory; once the copy has arrived
// (polled, never waited for) the interval is set from the stray fraction
// f_k seen k steps after the sort.  The window's halo absorbs small
// displacements, so strays grow faster than linearly with the age of the
// sort; modelling them as f_k (j/k)^2 at age j, a sort of cost C every L
// steps and strays of cost c each cost C/L + c f_k L^2 / (3 k^2) per step,
// least at L = (kSortBalance k^2 / f_k)^(1/3), with kSortBalance = 3 C / (2 c)
// in units of strays amounting to all particles.  On the 256^3 box at
// a = 0.5 the interval settles at 6-7 steps (plus one step on the wide
// windows): 0.72-0.73 ms per step, against 0.74-0.76 for any fixed interval
// of 4 to 8 steps and 0.96 when the counters were sampled right after each
// sort (where the halo still hides the motion).  From the Zel'dovich state
// at a = 0.01 no strays appear and the interval stays at its maximum.
namespace {

#ifndef FDM_SORT_BALANCE
#define FDM_SORT_BALANCE 0.02
#endif
constexpr double kSortBalance = FDM_SORT_BALANCE;
constexpr int kSortIntervalMax = 32;
#ifndef FDM_WIDE_INTERVAL
#define FDM_WIDE_INTERVAL 8
#endif
constexpr int kWideInterval = FDM_WIDE_INTERVAL;   // 0: never the wide windows
#ifndef FDM_WIDE_EXTRA
#define FDM_WIDE_EXTRA 1
#endif
constexpr int kWideExtra = FDM_WIDE_EXTRA;

pm_status sample_sort_stat(pm_ctx* c) {
  if (!c->sorted) return PM_OK;
  if (!c->h_stat) {
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_stat), kStrayBytes) != hipSuccess) {
      c->h_stat = nullptr;
      return PM_EDEVICE;
    }
    if (hipEventCreateWithFlags(&c->ev_stat, hipEventDisableTiming) != hipSuccess)
      return PM_EDEVICE;
    if (c->fixed) PM_TRY(dev(preload_wide(c->logn)));
  }
  PM_TRY(dev(hipMemcpyAsync(c->h_stat, static_cast<char*>(c->mass) + 8 * c->ncell, kStrayBytes,
                            hipMemcpyDeviceToHost, c->stream)));
  PM_TRY(dev(hipEventRecord(c->ev_stat, c->stream)));
  c->stat_pending = true;
  c->stat_age = c->since_sort;
  return PM_OK;
}

void poll_sort_stat(pm_ctx* c) {
  if (!c->stat_pending || hipEventQuery(c->ev_stat) != hipSuccess) return;
  c->stat_pending = false;
  double strays = 0.0;
  for (int k = 0; k < kStraySlices; ++k) strays += c->h_stat[k * kStrayStride];
  const double f = strays / (double)c->np;
  const double k = c->stat_age > 0 ? c->stat_age : 1;
  // Samples are taken at the end of an interval (strays stay near zero while
  // the halo absorbs the motion and then rise faster than the model, so
  // early samples would overestimate the interval).  A whole interval
  // without strays doubles it.
  int base = c->sort_base;
  if (f > 0.0) {
    const double l = cbrt(kSortBalance * k * k / f);
    base = l < 1.0 ? 1 : (l > kSortIntervalMax ? kSortIntervalMax : (int)l);
  } else if (k >= base) {
    base = std::min(2 * base, kSortIntervalMax);
  }
  c->sort_base = base;
  // Strays are counted against the narrow windows.  Where they set a short
  // interval, the steps after the first since a sort take the wide windows,
  // which absorb about one more step of motion: one step more between sorts.
  c->wide_windows = base <= kWideInterval;
  c->sort_interval = c->wide_windows ? std::min(base + kWideExtra, kSortIntervalMax) : base;
}

}  // namespace

namespace {

// Count, scan and scatter the particles (and ids) into dst by tile; the
// tile map then describes dst.
pm_status sort_into(pm_ctx* c, const void* pos, const float* vel, const int32_t* ids,
                    uint32_t* dst_pos, float* dst_vel, int* dst_ids) {
  const size_t cbytes = 4 * (size_t)kSlices * count_stride(c->tiles);
  PM_TRY(timed(c, kcFill, [&] { return launch_fill_zero(c->tile_counts, cbytes, c->stream); }));
  PM_TRY(timed(c, kcSortCount, [&] {
    return launch_sort_count(c->fixed, pos, c->np, c->logn, c->tile_counts, c->sort_key,
                             c->sort_rank, c->stream);
  }));
  PM_TRY(timed(c, kcSortScan, [&] {
    return launch_sort_scan(c->tile_counts, c->tiles, c->scan_sums, c->slice_start, c->tile_start,
                            c->chunk_start, c->stream);
  }));
  PM_TRY(timed(c, kcSortScatter, [&] {
    return launch_sort_scatter(pos, vel, ids, c->np, c->sort_key, c->sort_rank, c->slice_start,
                               dst_pos, dst_vel, dst_ids, c->stream);
  }));
  c->sorted = true;
  c->since_sort = 0;
  return PM_OK;
}

pm_status copy_particles(pm_ctx* c, void* pos, float* vel, const void* src_pos,
                         const float* src_vel) {
  return timed(c, kcSortCopy, [&] {
    hipError_t e = hipMemcpyAsync(pos, src_pos, 12 * (size_t)c->np, hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(vel, src_vel, 12 * (size_t)c->np, hipMemcpyDeviceToDevice, c->stream);
    return e;
  });
}

}  // namespace

// The step loop of pm_step and pm_step_energies (d_en: device rows of K, W,
// U, E per synchronised time, or null).
static pm_status step_impl(pm_ctx* c, void* d_pos, float* d_vel, const double* times,
                           int32_t nsteps, int32_t flags, double* d_en) {
  if (!c || !d_pos || !d_vel || !times) return PM_EINVAL;
  if (nsteps < 1) return PM_EINVAL;
  if (flags & ~(PM_CONTINUE | PM_SORT_EVERY(0xffff) | PM_SORT_AUTO)) return PM_EINVAL;
  const int sort_every = (flags >> 8) & 0xffff;
  const bool sort_auto = (flags & PM_SORT_AUTO) != 0;
  if (sort_auto && c->p.precision != PM_FIXED32) return PM_EUNSUPPORTED;
  for (int s = 0; s <= nsteps; ++s) {
    if (!isfinite(times[s])) return PM_EINVAL;
    if (c->p.comoving && !(times[s] > 0.0)) return PM_EINVAL;
    if (s > 0 && !(times[s] > times[s - 1])) return PM_EINVAL;
  }
  // A sort scatters the particles into the other of two buffers (the
  // caller's arrays and the workspace copies), which then becomes current;
  // the caller's arrays receive the state once, at the end of the call.
  void* cur_pos = d_pos;
  float* cur_vel = d_vel;
  void* alt_pos = c->pos_tmp;
  float* alt_vel = c->vel_tmp;
  auto sort_step = [&]() -> pm_status {
    PM_TRY(sort_into(c, cur_pos, cur_vel, nullptr, static_cast<uint32_t*>(alt_pos), alt_vel,
                     nullptr));
    std::swap(cur_pos, alt_pos);
    std::swap(cur_vel, alt_vel);
    return PM_OK;
  };
  // the kick before drift s: closing half of step s - 1 plus opening half of step s
  auto merged = [&](int s, const Kick& close) {
    const Kick open = kick(c->p, times[s], midpoint(c->p, times[s], times[s + 1]));
    return Kick{close.g + open.g, close.q + open.q};
  };
  // Energy rows: the stencil at x_s leaves the (delta phi, gradient)
  // partials, the gather of step s (or the closing half-kick) the |p|^2
  // partials of the momentum synchronised at t_s; one small kernel per row
  // reduces them in a fixed order.
  const bool en = d_en != nullptr;
  const double mp = (double)c->ncell / (double)c->np;
  auto energy_row = [&](int s) -> pm_status {
    const double a = c->p.comoving ? times[s] : 1.0;
    const EnergyScale sc = {0.5 * mp / (a * a), 0.5 / a, 0.5 * c->hm * c->hm / (a * a)};
    const int nk = (int)gather_blocks(c->np, c->sorted ? &c->tmap : nullptr);
    return timed(c, kcEnergyRow, [&] {
      return launch_energy_row(c->partials, c->q_blocks, c->kpart, nk, sc, d_en + 4 * (size_t)s,
                               c->stream);
    });
  };
  bool row0 = false;
  // Inside the call the fields for the next gather are written as the one
  // potential psi = F_g phi + F_q Q it needs; the fields left at the end of
  // the call stay phi and Q, for the closing half-kick and a continued call.
  // The energy form keeps phi and Q apart (the gather splits the kick at the
  // synchronised time).
  bool psi = false;
  if (!((flags & PM_CONTINUE) && c->fields_at_pos)) {
    // Sorting before the opening deposit lets it run from tiles: from a
    // clustered state the direct deposit contends on shared cells (6.5 ms
    // against well under 1 ms at 256^3, a = 0.5).  The integer deposit does
    // not depend on the order.
    if (c->fixed && !c->sorted && (sort_auto || sort_every > 0)) PM_TRY(sort_step());
    const Kick k0 = merged(0, Kick{0.0, 0.0});
    PM_TRY(run_fields(c, cur_pos, en, true, en ? nullptr : &k0));
    psi = c->has_q && !en;
    row0 = en;
  }
  c->fields_at_pos = false;
  const double fdu = c->fixed ? ldexp(1.0, c->B) : 1.0;
  Kick close = {0.0, 0.0};
  for (int s = 0; s < nsteps; ++s) {
    const double t0 = times[s], t1 = times[s + 1];
    const double tm = midpoint(c->p, t0, t1);
    const Kick kk = merged(s, close);
    if (sort_auto) {
      poll_sort_stat(c);
      if (!c->sorted || c->since_sort >= c->sort_interval) PM_TRY(sort_step());
    } else if (sort_every > 0 && s % sort_every == 0 && (!c->sorted || c->since_sort > 0)) {
      PM_TRY(sort_step());
    }
    GatherConst gc;
    if (en) {
      const Kick open = kick(c->p, t0, tm);
      gc.fg = (float)close.g;
      gc.fq = (float)close.q;
      gc.og = (float)open.g;
      gc.oq = (float)open.q;
      gc.kpart = c->kpart;
    } else if (psi) {
      gc.fg = 1.0f;
      gc.fq = 0.0f;
      gc.psi = 1;
    } else {
      gc.fg = (float)kk.g;
      gc.fq = (float)kk.q;
    }
    gc.fd_units = drift(c->p, t0, t1) * fdu;
    // gather + kick + drift, fused with the deposit of the drifted particles
    PM_TRY(timed(c, kcFill, [&] { return launch_fill_zero(c->mass, 8 * c->ncell + kStrayBytes, c->stream); }));
    // once the particles have moved since the sort, a state whose adaptive
    // interval is short (strays are frequent) takes the wider windows
    const bool wide = sort_auto && c->sorted && c->wide_windows && c->since_sort > 0;
    PM_TRY(timed(c, kcGatherKD, [&] {
      return launch_gather(c->fixed, c->has_q && !psi, true, c->logn, cur_pos, cur_vel,
                           psi ? c->q : c->phi, c->q, c->np, gc,
                           c->sorted ? &c->tmap : nullptr, c->mass, c->stream, Batch(), wide);
    }));
    ++c->since_sort;
    if (en && (s > 0 || row0)) PM_TRY(energy_row(s));
    // the last step before the next sort samples the strays of the interval
    if (sort_auto && !c->stat_pending && c->since_sort >= c->sort_interval)
      PM_TRY(sample_sort_stat(c));
    close = kick(c->p, tm, t1);
    if (s + 1 < nsteps && !en) {
      const Kick kn = merged(s + 1, close);
      PM_TRY(run_fields(c, cur_pos, false, false, &kn));
      psi = c->has_q;
    } else {
      PM_TRY(run_fields(c, cur_pos, en, false));
      psi = false;
    }
  }
  GatherConst gc;
  gc.fg = (float)close.g;
  gc.fq = (float)close.q;
  gc.fd_units = 0.0;
  if (en) gc.kpart = c->kpart;
  // closing half-kick; if the particles ended in the workspace copies, the
  // same pass writes them back to the caller's arrays
  const bool back = cur_pos != d_pos;
  PM_TRY(timed(c, kcKick, [&] {
    return launch_gather(c->fixed, c->has_q, false, c->logn, cur_pos, cur_vel, c->phi, c->q,
                         c->np, gc, c->sorted ? &c->tmap : nullptr, nullptr, c->stream, Batch(),
                         false, back ? d_pos : nullptr, back ? d_vel : nullptr);
  }));
  if (en) PM_TRY(energy_row(nsteps));
  if (back && !c->sorted) PM_TRY(copy_particles(c, d_pos, d_vel, cur_pos, cur_vel));
  c->fields_at_pos = true;
  return PM_OK;
}

pm_status pm_step(pm_ctx* c, void* d_pos, float* d_vel, const double* times, int32_t nsteps,
                  int32_t flags) {
  return step_impl(c, d_pos, d_vel, times, nsteps, flags, nullptr);
}

pm_status pm_step_energies(pm_ctx* c, void* d_pos, float* d_vel, const double* times,
                           int32_t nsteps, int32_t flags, double* d_energies) {
  if (!d_energies) return PM_EINVAL;
  return step_impl(c, d_pos, d_vel, times, nsteps, flags, d_energies);
}

pm_status pm_sort(pm_ctx* c, void* d_pos, float* d_vel, int32_t* d_ids) {
  if (!c || !d_pos || !d_vel) return PM_EINVAL;
  PM_TRY(sort_into(c, d_pos, d_vel, d_ids, c->pos_tmp, c->vel_tmp, c->ids_tmp));
  PM_TRY(copy_particles(c, d_pos, d_vel, c->pos_tmp, c->vel_tmp));
  if (d_ids)
    PM_TRY(timed(c, kcSortCopy, [&] {
      return hipMemcpyAsync(d_ids, c->ids_tmp, 4 * (size_t)c->np, hipMemcpyDeviceToDevice,
                            c->stream);
    }));
  return PM_OK;
}

pm_status pm_energy(pm_ctx* c, const void* d_pos, const float* d_vel, double a,
                    pm_energies* out) {
  if (!c || !d_pos || !d_vel || !out) return PM_EINVAL;
  if (!(a > 0.0) || !isfinite(a)) return PM_EINVAL;
  if (!c->p.comoving && a != 1.0) return PM_EINVAL;
  PM_TRY(run_fields(c, d_pos, true));
  c->fields_at_pos = false;
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(c->partials, c->q_blocks, 2, c->result, c->stream);
  }));
  double* kp = c->partials + 2 * (size_t)c->q_blocks;
  PM_TRY(timed(c, kcKinetic, [&] {
    return launch_kinetic(d_vel, c->np, kp, c->k_blocks, c->stream);
  }));
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(kp, c->k_blocks, 1, c->result + 2, c->stream);
  }));
  double host[3];
  PM_TRY(dev(hipMemcpyAsync(host, c->result, sizeof(host), hipMemcpyDeviceToHost, c->stream)));
  PM_TRY(dev(hipStreamSynchronize(c->stream)));
  const double mp = (double)c->ncell / (double)c->np;
  out->K = 0.5 * mp * host[2] / (a * a);
  out->W = 0.5 * host[0] / a;
  out->U = 0.5 * c->hm * c->hm * host[1] / (a * a);
  out->E = out->K + out->W + out->U;
  return PM_OK;
}

// After a diagnostic has used delta..spec as FP64 scratch: no field in the
// workspace is valid any more; a context without quantum pressure keeps Q
// at zero.
// Blocks of the node reductions: two partials each fit the workspace's
// 2 N^3 / kBlock + 1024 partial slots.
static int diag_node_blocks(const pm_ctx* c) {
  return diag_blocks((int64_t)c->ncell, 2048);
}

static pm_status diag_done(pm_ctx* c) {
  c->have_delta = false;
  c->have_phi = false;
  c->have_q = false;
  c->fields_at_pos = false;
  if (!c->has_q) PM_TRY(dev(launch_fill_zero(c->q, 4 * c->ncell, c->stream)));
  return PM_OK;
}

pm_status pm_kinetic_split(pm_ctx* c, const void* d_pos, const float* d_vel, double a,
                           pm_kinetic_parts* out) {
  if (!c || !d_pos || !d_vel || !out) return PM_EINVAL;
  if (!(a > 0.0) || !isfinite(a)) return PM_EINVAL;
  if (!c->p.comoving && a != 1.0) return PM_EINVAL;
  PM_TRY(run_deposit(c, d_pos));
  // delta and phi are adjacent 4 N^3-byte blocks: one FP64 mesh
  double* mom = reinterpret_cast<double*>(c->delta);
  const int nb = diag_node_blocks(c);
  for (int d = 0; d < 3; ++d) {
    PM_TRY(timed(c, kcFill, [&] { return launch_fill_zero(mom, 8 * c->ncell, c->stream); }));
    PM_TRY(timed(c, kcMomentum, [&] {
      return launch_deposit_momentum(c->fixed, c->logn, d_pos, c->np, d_vel + d * c->np, mom,
                                     c->sorted ? &c->tmap : nullptr, c->stream);
    }));
    PM_TRY(timed(c, kcDiagNodes, [&] {
      return launch_bulk_nodes(c->fixed, c->mass, mom, (int64_t)c->ncell, c->partials, nb,
                               c->stream);
    }));
    PM_TRY(timed(c, kcReduce, [&] {
      return launch_reduce(c->partials, nb, 1, c->result + 4 + d, c->stream);
    }));
  }
  double* kp = c->partials + 2 * (size_t)c->q_blocks;
  PM_TRY(timed(c, kcKinetic, [&] {
    return launch_kinetic(d_vel, c->np, kp, c->k_blocks, c->stream);
  }));
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(kp, c->k_blocks, 1, c->result + 3, c->stream);
  }));
  double host[4];
  PM_TRY(dev(hipMemcpyAsync(host, c->result + 3, sizeof(host), hipMemcpyDeviceToHost,
                            c->stream)));
  PM_TRY(diag_done(c));
  PM_TRY(dev(hipStreamSynchronize(c->stream)));
  const double mp = (double)c->ncell / (double)c->np;
  out->K = 0.5 * mp * host[0] / (a * a);
  out->K_bulk = 0.5 * mp * (host[1] + host[2] + host[3]) / (a * a);
  out->K_disp = out->K - out->K_bulk;
  return PM_OK;
}

pm_status pm_density_rms_diff(pm_ctx* c, const void* d_pos_a, const void* d_pos_b,
                              double* rms, int64_t* cells) {
  if (!c || !d_pos_a || !d_pos_b || !rms || !cells) return PM_EINVAL;
  // the reference state's mass mesh is kept in delta..phi (8 N^3 bytes)
  void* mass_b = c->delta;
  const size_t mesh_bytes = (c->fixed ? 8 : 4) * c->ncell;
  PM_TRY(run_deposit(c, d_pos_b));
  PM_TRY(dev(hipMemcpyAsync(mass_b, c->mass, mesh_bytes, hipMemcpyDeviceToDevice, c->stream)));
  PM_TRY(run_deposit(c, d_pos_a));
  const int nb = diag_node_blocks(c);
  PM_TRY(timed(c, kcDiagNodes, [&] {
    return launch_rel_diff_nodes(c->fixed, c->mass, mass_b, (int64_t)c->ncell, c->partials, nb,
                                 c->stream);
  }));
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(c->partials, nb, 2, c->result + 8, c->stream);
  }));
  double host[2];
  PM_TRY(dev(hipMemcpyAsync(host, c->result + 8, sizeof(host), hipMemcpyDeviceToHost,
                            c->stream)));
  PM_TRY(diag_done(c));
  PM_TRY(dev(hipStreamSynchronize(c->stream)));
  const int64_t n = (int64_t)host[1];
  *cells = n;
  *rms = n > 0 ? sqrt(host[0] / (double)n) : 0.0;
  return PM_OK;
}

pm_status pm_power_spectrum(pm_ctx* c, const void* d_pos, int32_t nbins, double* k_out,
                            double* p_out, double* counts_out) {
  if (!c || !d_pos || !k_out || !p_out || !counts_out) return PM_EINVAL;
  if (nbins < 1 || nbins > c->N / 2) return PM_EINVAL;
  PM_TRY(run_deposit(c, d_pos));
  PM_TRY(timed(c, kcR2C, [&] {
    return launch_r2c_z(c->logn, c->fixed ? kSrcMass64 : kSrcAcc32, c->mass, c->delta, c->spec,
                        c->tw, c->conv, c->stream);
  }));
  PM_TRY(timed(c, kcFftY, [&] { return launch_fft_y(c->logn, c->spec, c->tw, false, c->stream); }));
  // per-block shell sums in the phi block (4 N^3 bytes hold them for every N)
  double* blk = reinterpret_cast<double*>(c->phi);
  PM_TRY(timed(c, kcPower, [&] {
    return launch_fft_x_power(c->logn, c->spec, c->tw, nbins, blk, c->partials, c->stream);
  }));
  std::vector<double> host(2 * (size_t)(nbins + 1));
  PM_TRY(dev(hipMemcpyAsync(host.data(), c->partials, host.size() * sizeof(double),
                            hipMemcpyDeviceToHost, c->stream)));
  PM_TRY(diag_done(c));
  PM_TRY(dev(hipStreamSynchronize(c->stream)));
  const double nn = (double)c->N;
  const double box = c->p.box;
  const double scale = box * box * box / (nn * nn * nn * nn * nn * nn);
  for (int b = 1; b <= nbins; ++b) {
    const double w = host[2 * b + 1];
    k_out[b - 1] = 2.0 * M_PI * b / box;
    p_out[b - 1] = w > 0.0 ? host[2 * b] / w * scale : 0.0;
    counts_out[b - 1] = w;
  }
  return PM_OK;
}

// Smoothing lengths of at least two cells: below that the lattice sum of the
// kernel of Eq. (15) drifts away from one (a particle's deposited mass varies
// by +-9 % with its position at h = 1.5 and by +-0.2 % at h = 2), and below
// sqrt(3)/2 cells a particle can miss every node.
static bool spline_h_ok(const pm_ctx* c, double h) {
  return isfinite(h) && h >= 2.0 && 2.0 * floor(h) + 2.0 <= (double)c->N && h <= 16.0;
}

// The spline density of the positions into the context's mass mesh, in the
// integer units of the CIC deposit (both precisions).
static pm_status run_spline_density(pm_ctx* c, const void* pos, double h) {
  PM_TRY(timed(c, kcFill, [&] {
    return launch_fill_zero(c->mass, 8 * c->ncell + kStrayBytes, c->stream);
  }));
  return timed(c, kcSpline, [&] {
    return launch_spline_deposit(c->fixed, c->logn, pos, c->np, (float)h,
                                 c->sorted ? &c->tmap : nullptr,
                                 static_cast<unsigned long long*>(c->mass), c->stream);
  });
}

pm_status pm_spline_density(pm_ctx* c, const void* d_pos, double h, float* d_delta) {
  if (!c || !d_pos || !d_delta) return PM_EINVAL;
  if (!spline_h_ok(c, h)) return PM_EINVAL;
  PM_TRY(run_spline_density(c, d_pos, h));
  // delta = mass / mbar - 1 by the exact integer subtraction of the forward
  // z pass (its spectrum is not used)
  PM_TRY(timed(c, kcR2C, [&] {
    return launch_r2c_z(c->logn, kSrcMass64, c->mass, c->delta, c->spec, c->tw, c->conv,
                        c->stream);
  }));
  c->have_delta = true;
  c->have_phi = false;
  c->have_q = false;
  c->fields_at_pos = false;
  if (!c->has_q) PM_TRY(dev(launch_fill_zero(c->q, 4 * c->ncell, c->stream)));
  return copy_out(c, d_delta, c->delta);
}

pm_status pm_spline_qforce(pm_ctx* c, const void* d_pos, const float* d_q, double h,
                           float* d_acc) {
  if (!c || !d_pos || !d_q || !d_acc) return PM_EINVAL;
  if (!spline_h_ok(c, h)) return PM_EINVAL;
  return timed(c, kcSplineForce, [&] {
    return launch_spline_qforce(c->fixed, c->logn, d_pos, c->np, d_q, (float)h, d_acc,
                                c->stream);
  });
}

pm_status pm_spline_step(pm_ctx* c, void* d_pos, float* d_vel, const double* times,
                         int32_t nsteps, double h) {
  if (!c || !d_pos || !d_vel || !times || nsteps < 1) return PM_EINVAL;
  if (!spline_h_ok(c, h)) return PM_EINVAL;
  for (int s = 0; s <= nsteps; ++s) {
    if (!isfinite(times[s]) || (c->p.comoving && !(times[s] > 0.0))) return PM_EINVAL;
    if (s > 0 && !(times[s] > times[s - 1])) return PM_EINVAL;
  }
  // accelerations at the current positions: -grad phi (CIC) and the kernel
  // gradient of Q, [3][Np] floats each in the particle copy buffers
  float* gphi = reinterpret_cast<float*>(c->pos_tmp);
  float* gq = c->vel_tmp;
  auto forces = [&]() -> pm_status {
    PM_TRY(run_spline_density(c, d_pos, h));
    PM_TRY(run_poisson(c, kSrcMass64, c->mass));
    PM_TRY(timed(c, kcForce, [&] {
      return launch_force(c->fixed, false, c->logn, d_pos, c->phi, c->q, c->np, 1.0f, 0.0f,
                          gphi, c->stream);
    }));
    if (!c->has_q)
      // 16-byte multiple: the buffer is a 256-byte aligned region of at least 12 Np bytes
      return timed(c, kcFill, [&] {
        return launch_fill_zero(gq, (12 * (size_t)c->np + 15) & ~(size_t)15, c->stream);
      });
    PM_TRY(run_qpot(c, c->delta, c->fixed, kOutQ));
    return timed(c, kcSplineForce, [&] {
      return launch_spline_qforce(c->fixed, c->logn, d_pos, c->np, c->q, (float)h, gq,
                                  c->stream);
    });
  };
  auto kick_by = [&](const Kick& k) {
    return timed(c, kcKick, [&] {
      return launch_spline_kick(d_vel, gphi, gq, c->np, (float)k.g, (float)k.q, c->stream);
    });
  };
  c->fields_at_pos = false;
  PM_TRY(forces());
  for (int s = 0; s < nsteps; ++s) {
    const double t0 = times[s], t1 = times[s + 1], tm = midpoint(c->p, t0, t1);
    PM_TRY(kick_by(kick(c->p, t0, tm)));
    PM_TRY(timed(c, kcGatherKD, [&] {
      return launch_spline_drift(c->fixed, c->logn, d_pos, d_vel, c->np, drift(c->p, t0, t1),
                                 c->stream);
    }));
    PM_TRY(forces());
    PM_TRY(kick_by(kick(c->p, tm, t1)));
  }
  // delta holds the spline contrast and phi, Q its fields; none of them is
  // what the cloud-in-cell calls expect
  c->have_delta = false;
  c->have_phi = false;
  c->have_q = false;
  if (!c->has_q) PM_TRY(dev(launch_fill_zero(c->q, 4 * c->ncell, c->stream)));
  return PM_OK;
}

pm_status pm_spline_energy(pm_ctx* c, const void* d_pos, const float* d_vel, double h,
                           double a, pm_energies* out) {
  if (!c || !d_pos || !d_vel || !out) return PM_EINVAL;
  if (!spline_h_ok(c, h)) return PM_EINVAL;
  if (!(a > 0.0) || !isfinite(a)) return PM_EINVAL;
  if (!c->p.comoving && a != 1.0) return PM_EINVAL;
  PM_TRY(run_spline_density(c, d_pos, h));
  PM_TRY(run_poisson(c, kSrcMass64, c->mass));
  PM_TRY(run_qpot(c, c->delta, c->fixed, kOutEnergy));
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(c->partials, c->q_blocks, 2, c->result, c->stream);
  }));
  double* kp = c->partials + 2 * (size_t)c->q_blocks;
  PM_TRY(timed(c, kcKinetic, [&] {
    return launch_kinetic(d_vel, c->np, kp, c->k_blocks, c->stream);
  }));
  PM_TRY(timed(c, kcReduce, [&] {
    return launch_reduce(kp, c->k_blocks, 1, c->result + 2, c->stream);
  }));
  double host[3];
  PM_TRY(dev(hipMemcpyAsync(host, c->result, sizeof(host), hipMemcpyDeviceToHost, c->stream)));
  PM_TRY(diag_done(c));
  PM_TRY(dev(hipStreamSynchronize(c->stream)));
  const double mp = (double)c->ncell / (double)c->np;
  out->K = 0.5 * mp * host[2] / (a * a);
  out->W = 0.5 * host[0] / a;
  out->U = 0.5 * c->hm * c->hm * host[1] / (a * a);
  out->E = out->K + out->W + out->U;
  return PM_OK;
}

pm_status pm_timing_enable(pm_ctx* c, int32_t on) {
  if (!c) return PM_EINVAL;
  Timer& t = c->timer;
  if (!t.pending.empty() && hipStreamSynchronize(c->stream) != hipSuccess) return PM_EDEVICE;
  for (auto& r : t.pending) {
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.pending.clear();
  for (int k = 0; k < kcCount; ++k) {
    t.ms[k] = 0.0;
    t.launches[k] = 0;
  }
  t.on = on != 0;
  return PM_OK;
}

pm_status pm_timing_read(pm_ctx* c, pm_kernel_time* out, int32_t max, int32_t* count) {
  if (!c || !count || max < 0 || (max > 0 && !out)) return PM_EINVAL;
  Timer& t = c->timer;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PM_EDEVICE;
  for (auto& r : t.pending) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return PM_EDEVICE;
    t.ms[r.kc] += ms;
    t.launches[r.kc] += 1;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.pending.clear();
  int n = 0;
  for (int k = 0; k < kcCount && n < max; ++k) {
    if (t.launches[k] == 0) continue;
    memset(out[n].name, 0, sizeof(out[n].name));
    strncpy(out[n].name, kKernelNames[k], sizeof(out[n].name) - 1);
    out[n].launches = t.launches[k];
    out[n].total_ms = t.ms[k];
    ++n;
  }
  *count = n;
  return PM_OK;
}

pm_status pm_batch_workspace_bytes(const pm_params* params, int32_t slots, size_t* bytes) {
  if (!bytes || slots < 1) return PM_EINVAL;
  PM_TRY(check_params(params));
  *bytes = batch_header(slots) + (size_t)slots * layout_for(*params).total;
  return PM_OK;
}

pm_status pm_batch_init(const pm_params* params, int32_t slots, void* d_workspace, size_t bytes,
                        void* hip_stream, pm_batch** out) {
  if (!out || !d_workspace || slots < 1) return PM_EINVAL;
  PM_TRY(check_params(params));
  if (((uintptr_t)d_workspace) % kAlign != 0) return PM_EINVAL;
  const size_t stride = layout_for(*params).total;
  const size_t header = batch_header(slots);
  if (bytes < header + (size_t)slots * stride) return PM_ENOMEM;
  pm_batch* b = new (std::nothrow) pm_batch();
  if (!b) return PM_ENOMEM;
  b->slots = slots;
  b->slot_stride = stride;
  b->header = header;
  b->ws = static_cast<char*>(d_workspace);
  b->d_slots = reinterpret_cast<int*>(b->ws);
  b->d_consts = reinterpret_cast<SlotConst*>(b->ws + align_up(4 * (size_t)slots));
  const pm_status st = ctx_setup(&b->base, params, b->ws + header,
                                 static_cast<hipStream_t>(hip_stream));
  if (st != PM_OK) {
    delete b;
    return st;
  }
  for (int i = 0; i < 2; ++i) {
    if (hipHostMalloc(reinterpret_cast<void**>(&b->h_stage[i]), header) != hipSuccess ||
        hipEventCreateWithFlags(&b->h_done[i], hipEventDisableTiming) != hipSuccess) {
      batch_free(b);
      return PM_EDEVICE;
    }
  }
  b->box.assign(slots, params->box);
  b->hm.assign(slots, b->base.hm);
  b->fields_ok.assign(slots, 0);
  b->sorted.assign(slots, 0);
  *out = b;
  return PM_OK;
}

pm_status pm_batch_slot_offset(const pm_batch* b, int32_t slot, size_t* offset) {
  if (!b || !offset || slot < 0 || slot >= b->slots) return PM_EINVAL;
  *offset = b->header + (size_t)slot * b->slot_stride;
  return PM_OK;
}

pm_status pm_batch_set_slot(pm_batch* b, int32_t slot, const pm_slot_params* sp) {
  if (!b || !sp || slot < 0 || slot >= b->slots) return PM_EINVAL;
  if (!(sp->box > 0.0) || !isfinite(sp->box)) return PM_EINVAL;
  if (!(sp->hbar_over_m >= 0.0) || !isfinite(sp->hbar_over_m)) return PM_EINVAL;
  const double dx = sp->box / b->base.N;
  b->box[slot] = sp->box;
  b->hm[slot] = sp->hbar_over_m / (dx * dx);
  b->fields_ok[slot] = 0;
  return PM_OK;
}

pm_status pm_batch_step(pm_batch* b, void* d_pos, float* d_vel, int32_t nactive,
                        const int32_t* slots, const double* times, int32_t nsteps,
                        int32_t flags) {
  if (!b || !d_pos || !d_vel || !slots || !times) return PM_EINVAL;
  if (nactive < 1 || nactive > b->slots) return PM_EINVAL;
  if (nsteps < 1 || nsteps > PM_BATCH_MAX_STEPS) return PM_EINVAL;
  if (flags & ~(PM_CONTINUE | PM_SORT_EVERY(0xffff) | PM_BATCH_GRAPH)) return PM_EINVAL;
  pm_ctx* c = &b->base;
  const bool use_graph = (flags & PM_BATCH_GRAPH) != 0;
  if (use_graph && c->stream == nullptr) return PM_EINVAL;   // no capture on the default stream
  flags &= ~PM_BATCH_GRAPH;
  std::vector<char> seen(b->slots, 0);
  bool all_sorted = true, all_fields = true;
  for (int i = 0; i < nactive; ++i) {
    const int s = slots[i];
    if (s < 0 || s >= b->slots || seen[s]) return PM_EINVAL;
    seen[s] = 1;
    all_sorted = all_sorted && b->sorted[s];
    all_fields = all_fields && b->fields_ok[s];
    const double* t = times + (size_t)i * (nsteps + 1);
    for (int k = 0; k <= nsteps; ++k) {
      if (!isfinite(t[k])) return PM_EINVAL;
      if (c->p.comoving && !(t[k] > 0.0)) return PM_EINVAL;
      if (k > 0 && !(t[k] > t[k - 1])) return PM_EINVAL;
    }
  }
  if ((flags & PM_CONTINUE) && !all_fields) return PM_ESTATE;
  const int sort_every = (flags >> 8) & 0xffff;
  // per-step, per-slot constants: row k < nsteps is the merged kick before
  // drift k, row nsteps the closing half-kick
  const double fdu = c->fixed ? ldexp(1.0, c->B) : 1.0;
  std::vector<SlotConst> tab((size_t)(nsteps + 1) * nactive);
  for (int i = 0; i < nactive; ++i) {
    const int s = slots[i];
    const double* t = times + (size_t)i * (nsteps + 1);
    const double qd = -0.5 * b->hm[s] * b->hm[s];
    Kick close = {0.0, 0.0};
    for (int k = 0; k <= nsteps; ++k) {
      SlotConst& e = tab[(size_t)k * nactive + i];
      e.qcoef = (float)qd;
      e.qcoef_d = qd;
      e.pad = 0.0f;
      if (k < nsteps) {
        const double tm = midpoint(c->p, t[k], t[k + 1]);
        const Kick open = kick(c->p, t[k], tm);
        e.fg = (float)(close.g + open.g);
        e.fq = (float)(close.q + open.q);
        e.fd_units = drift(c->p, t[k], t[k + 1]) * fdu;
        close = kick(c->p, tm, t[k + 1]);
      } else {
        e.fg = (float)close.g;
        e.fq = (float)close.q;
        e.fd_units = 0.0;
      }
    }
  }
  // the buffer's previous copy was queued two calls ago; wait for it
  const int hb = b->h_next;
  b->h_next ^= 1;
  PM_TRY(dev(hipEventSynchronize(b->h_done[hb])));
  char* h = b->h_stage[hb];
  const size_t coff = (size_t)(reinterpret_cast<char*>(b->d_consts) - b->ws);
  memcpy(h, slots, 4 * (size_t)nactive);
  memcpy(h + coff, tab.data(), sizeof(SlotConst) * tab.size());
  auto upload = [&]() -> pm_status {
    PM_TRY(dev(hipMemcpyAsync(b->ws, h, coff + sizeof(SlotConst) * tab.size(),
                              hipMemcpyHostToDevice, c->stream)));
    return dev(hipEventRecord(b->h_done[hb], c->stream));
  };
  Batch bt;
  bt.slots = b->d_slots;
  bt.ws_stride = (long long)b->slot_stride;
  bt.part_stride = 12ll * c->np;
  bt.count = (unsigned)nactive;
  auto row = [&](int k) {
    Batch r = bt;
    r.consts = b->d_consts + (size_t)k * nactive;
    return r;
  };
  bool sorted = all_sorted;
  const float gscale = (float)(-c->S * 2.0 / ((double)c->N * c->N * c->N));
  // to_psi: q receives psi = F_g phi + F_q Q with the factors of bq's row
  auto fields = [&](const Batch& bq, bool to_psi) -> pm_status {
    PM_TRY(dev(launch_r2c_z(c->logn, c->fixed ? kSrcMass64 : kSrcAcc32, c->mass, c->delta,
                            c->spec, c->tw, c->conv, c->stream, bt)));
    PM_TRY(dev(launch_fft_y(c->logn, c->spec, c->tw, false, c->stream, bt)));
    PM_TRY(dev(launch_fft_x_green(c->logn, c->spec, c->tw, c->s2, gscale, c->stream, bt)));
    PM_TRY(dev(launch_fft_y(c->logn, c->spec, c->tw, true, c->stream, bt)));
    PM_TRY(dev(launch_c2r_z(c->logn, c->spec, c->tw, c->phi, c->stream, bt)));
    return dev(launch_qpot(c->logn, c->fixed, to_psi ? kOutPsi : kOutQ, c->delta,
                           static_cast<const long long*>(c->mass), c->phi, c->q, c->qc,
                           c->partials, c->stream, bq));
  };
  auto sort_all = [&]() -> pm_status {
    const size_t cbytes = 4 * (size_t)kSlices * count_stride(c->tiles);
    PM_TRY(dev(launch_fill_zero(c->tile_counts, cbytes, c->stream, bt)));
    PM_TRY(dev(launch_sort_count(c->fixed, d_pos, c->np, c->logn, c->tile_counts, c->sort_key,
                                 c->sort_rank, c->stream, bt)));
    PM_TRY(dev(launch_sort_scan(c->tile_counts, c->tiles, c->scan_sums, c->slice_start, c->tile_start,
                                c->chunk_start, c->stream, bt)));
    PM_TRY(dev(launch_sort_scatter(d_pos, d_vel, nullptr, c->np, c->sort_key, c->sort_rank,
                                   c->slice_start, c->pos_tmp, c->vel_tmp, nullptr, c->stream,
                                   bt)));
    PM_TRY(dev(launch_sort_copy(static_cast<uint32_t*>(d_pos), d_vel, c->pos_tmp, c->vel_tmp,
                                c->np, c->stream, bt)));
    sorted = true;
    return PM_OK;
  };
  // Every kernel of the call, in stream order after the upload of its slot
  // list and constant table.  Every launch argument depends only on the
  // call's shape (the slot identities and the factors are read from the
  // uploaded table), so a captured graph of one call's kernels serves every
  // later call of the same shape.  The upload itself stays outside the graph:
  // an event recorded in a capturing stream is not replayed, and the host
  // must know when each staging buffer's copy is done.
  auto enqueue = [&]() -> pm_status {
  if (!(flags & PM_CONTINUE)) {
    PM_TRY(dev(launch_fill_zero(c->mass, 8 * c->ncell + kStrayBytes, c->stream, bt)));
    if (c->fixed)
      PM_TRY(dev(sorted ? launch_deposit_fixed_tiled(static_cast<const uint32_t*>(d_pos), c->np,
                                                     c->logn, c->tmap,
                                                     static_cast<unsigned long long*>(c->mass),
                                                     c->stream, bt)
                        : launch_deposit_fixed(static_cast<const uint32_t*>(d_pos), c->np,
                                               c->logn,
                                               static_cast<unsigned long long*>(c->mass),
                                               c->stream, bt)));
    else
      PM_TRY(dev(sorted ? launch_deposit_f32_tiled(static_cast<const float*>(d_pos), c->np,
                                                   c->logn, c->tmap,
                                                   static_cast<float*>(c->mass), c->stream, bt)
                        : launch_deposit_f32(static_cast<const float*>(d_pos), c->np, c->logn,
                                             static_cast<float*>(c->mass), c->stream, bt)));
    PM_TRY(fields(row(0), true));
  }
  // inside the call the fields hold psi for the next row's factors; the last
  // fields stay phi and Q (closing half-kick, continued calls)
  bool psi = !(flags & PM_CONTINUE);
  for (int i = 0; i < nactive; ++i) b->fields_ok[slots[i]] = 0;
  GatherConst unused;
  unused.fg = unused.fq = 0.0f;
  unused.fd_units = 0.0;
  GatherConst gpsi;
  gpsi.fg = 1.0f;
  gpsi.fq = 0.0f;
  gpsi.fd_units = 0.0;
  gpsi.psi = 1;
  for (int k = 0; k < nsteps; ++k) {
    if (sort_every > 0 && k % sort_every == 0) PM_TRY(sort_all());
    PM_TRY(dev(launch_fill_zero(c->mass, 8 * c->ncell + kStrayBytes, c->stream, bt)));
    PM_TRY(dev(launch_gather(c->fixed, !psi, true, c->logn, d_pos, d_vel, psi ? c->q : c->phi,
                             c->q, c->np, psi ? gpsi : unused, sorted ? &c->tmap : nullptr,
                             c->mass, c->stream, row(k))));
    psi = k + 1 < nsteps;
    PM_TRY(fields(row(psi ? k + 1 : k), psi));
  }
  return dev(launch_gather(c->fixed, true, false, c->logn, d_pos, d_vel, c->phi, c->q, c->np,
                           unused, sorted ? &c->tmap : nullptr, nullptr, c->stream, row(nsteps)));
  };
  PM_TRY(upload());
  if (!use_graph) {
    PM_TRY(enqueue());
  } else {
    const auto key = std::make_tuple((int)nactive, (int)nsteps, (int)flags, (int)all_sorted);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
      if (b->graphs.size() >= 64) {
        for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
        b->graphs.clear();
      }
      PM_TRY(dev(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)));
      const pm_status st = enqueue();
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(c->stream, &graph);
      if (st != PM_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return st != PM_OK ? st : PM_EDEVICE;
      }
      hipGraphExec_t exec = nullptr;
      const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return PM_EDEVICE;
      it = b->graphs.emplace(key, exec).first;
    }
    PM_TRY(dev(hipGraphLaunch(it->second, c->stream)));
  }
  sorted = all_sorted || (sort_every > 0) || sorted;
  for (int i = 0; i < nactive; ++i) {
    b->fields_ok[slots[i]] = 1;
    if (sorted) b->sorted[slots[i]] = 1;
  }
  return PM_OK;
}

pm_status pm_batch_destroy(pm_batch* b) {
  if (!b) return PM_EINVAL;
  batch_free(b);
  return PM_OK;
}

pm_status pm_destroy(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  if (!c->timer.pending.empty() || c->stat_pending) (void)hipStreamSynchronize(c->stream);
  if (c->ev_stat) (void)hipEventDestroy(c->ev_stat);
  if (c->h_stat) (void)hipHostFree(c->h_stat);
  for (auto& r : c->timer.pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->timer.pool) (void)hipEventDestroy(e);
  delete c;
  return PM_OK;
}

const char* pm_strerror(pm_status s) {
  switch (s) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_ENOMEM: return "workspace too small";
    case PM_EDEVICE: return "HIP runtime or kernel launch error";
    case PM_EUNSUPPORTED: return "unsupported mesh size (power of two in [16, 512])";
    case PM_ESTATE: return "required fields not computed yet";
  }
  return "unknown status";
}

}  // extern "C"
