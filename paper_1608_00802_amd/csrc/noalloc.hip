// The Poisson solve of pm_poisson for callers that cannot allocate device
// memory: its spectrum and constant tables live in a file-scope device
// array of the library (one copy per GPU, alive until the process ends),
// so the call needs neither a context nor a workspace.
#include <math.h>

#include <mutex>

#include "../../include/fdmpm.h"
#include "internal.h"

using namespace fdm;

namespace {

constexpr int kStaticMaxN = 128;
constexpr size_t kSpecBytes = 8ull * (kStaticMaxN / 2 + 1) * kStaticMaxN * kStaticMaxN;
constexpr size_t kStaticScratchBytes =
    (kSpecBytes + 8 * kStaticMaxN + 4 * kStaticMaxN + 255) / 256 * 256;

// The scratch: spectrum [8 (N/2 + 1) N^2 bytes], then the twiddles
// exp(-2 pi i k / N) (float2 [N]) and 4 sin^2(pi k / N) (float [N]).  In
// host code its name is a host-side stand-in: kernels get the per-device
// address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Address of this device's scratch, looked up once per device with that
// device current.
pm_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PM_EDEVICE;
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PM_EDEVICE;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return PM_OK;
}

// The FFT's constant tables, computed in FP64 on the device and rounded once.
__global__ void k_static_tables(float2* __restrict__ tw, float* __restrict__ s2, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double sn, cs;
  sincospi(-2.0 * k / n, &sn, &cs);
  tw[k] = make_float2((float)cs, (float)sn);
  const double h = sinpi((double)k / n);
  s2[k] = (float)(4.0 * h * h);
}

}  // namespace

extern "C" pm_status pm_poisson_static(int32_t n_mesh, double S, const float* d_delta,
                                       float* d_phi, void* hip_stream) {
  if (!d_delta || !d_phi || !isfinite(S)) return PM_EINVAL;
  if (n_mesh < 16 || (n_mesh & (n_mesh - 1)) != 0) return PM_EUNSUPPORTED;
  if (n_mesh > kStaticMaxN) return PM_ENOMEM;
  int logn = 0;
  while ((1 << logn) < n_mesh) ++logn;
  void* base = nullptr;
  const pm_status st = scratch_ptr(&base);
  if (st != PM_OK) return st;
  const size_t n = (size_t)n_mesh;
  float2* spec = static_cast<float2*>(base);
  float2* tw = reinterpret_cast<float2*>(static_cast<char*>(base) + 8 * (n / 2 + 1) * n * n);
  float* s2 = reinterpret_cast<float*>(tw + n);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipLaunchKernelGGL(k_static_tables, dim3((n_mesh + 127) / 128), dim3(128), 0, s, tw, s2,
                     n_mesh);
  DeltaConv conv = {};
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_r2c_z(logn, kSrcDelta, d_delta, nullptr, spec, tw, conv, s);
  if (e == hipSuccess) e = launch_fft_y(logn, spec, tw, false, s);
  const double nn = (double)n_mesh;
  if (e == hipSuccess)
    e = launch_fft_x_green(logn, spec, tw, s2, (float)(-S * 2.0 / (nn * nn * nn)), s);
  if (e == hipSuccess) e = launch_fft_y(logn, spec, tw, true, s);
  if (e == hipSuccess) e = launch_c2r_z(logn, spec, tw, d_phi, s);
  return e == hipSuccess ? PM_OK : PM_EDEVICE;
}
