// Kinetic-energy spectrum: E(k) = sum over the wavevectors with round(|k|) = k of
// |u_hat|^2 / 2, u_hat = FFT(u / u0) / n^3 (Section 3.5, spectra at peak activity).
// The transforms are rocFFT's; the binning is a grid-stride pass over the
// half-spectrum of each component into per-block LDS histograms, reduced over
// the blocks in a fixed order.
#include "postproc.hpp"

#include <rocfft/rocfft.h>

#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>

namespace stgv {
namespace {

constexpr int kShellBlocks = 1024;
constexpr int kShellThreads = 256;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// One component's half spectrum c[(n/2 + 1) n n] (kx fastest): the Hermitian twins of
// 0 < kx < n/2 are counted twice.  scale = 1 / (2 n^6 u0^2).
__global__ __launch_bounds__(kShellThreads) void shell_kernel(const float2* __restrict__ c, int n,
                                                              int nshell, double scale,
                                                              double* __restrict__ partial) {
  extern __shared__ double hist[];
  for (int s = threadIdx.x; s < nshell; s += blockDim.x) hist[s] = 0.0;
  __syncthreads();
  const int nh = n / 2 + 1;
  const int64_t total = (int64_t)nh * n * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int kx = (int)(i % nh);
    const int64_t r = i / nh;
    const int ky0 = (int)(r % n), kz0 = (int)(r / n);
    const int ky = ky0 <= n / 2 ? ky0 : ky0 - n;
    const int kz = kz0 <= n / 2 ? kz0 : kz0 - n;
    const double k = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
    const int s = (int)floor(k + 0.5);
    const float2 v = c[i];
    const double w = (kx == 0 || 2 * kx == n) ? 1.0 : 2.0;
    atomicAdd(&hist[s], w * ((double)v.x * v.x + (double)v.y * v.y) * scale);
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nshell; s += blockDim.x) partial[(int64_t)blockIdx.x * nshell + s] = hist[s];
}

__global__ __launch_bounds__(256) void shell_reduce_kernel(const double* __restrict__ partial, int nparts,
                                                           int nshell, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshell) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += partial[(int64_t)b * nshell + s];
  out[s] = acc;
}

struct Plan {
  rocfft_plan plan = nullptr;
  size_t work = 0;
};
std::mutex g_mutex;
std::map<int, Plan> g_plans;
bool g_setup = false;

const Plan* get_plan(int n, char* err) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_setup) {
    if (rocfft_setup() != rocfft_status_success) {
      snprintf(err, 512, "rocfft_setup failed");
      return nullptr;
    }
    g_setup = true;
  }
  auto it = g_plans.find(n);
  if (it != g_plans.end()) return &it->second;
  Plan p;
  const size_t lengths[3] = {(size_t)n, (size_t)n, (size_t)n};
  if (rocfft_plan_create(&p.plan, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                         rocfft_precision_single, 3, lengths, 1, nullptr) != rocfft_status_success) {
    snprintf(err, 512, "rocfft_plan_create failed for %d^3", n);
    return nullptr;
  }
  if (rocfft_plan_get_work_buffer_size(p.plan, &p.work) != rocfft_status_success) {
    snprintf(err, 512, "rocfft_plan_get_work_buffer_size failed");
    rocfft_plan_destroy(p.plan);
    return nullptr;
  }
  return &(g_plans[n] = p);
}

struct Layout {
  size_t complex_off, partial_off, fft_off, total;
};

Layout layout(int n, size_t fft_work) {
  Layout l;
  const size_t cbytes = (size_t)(n / 2 + 1) * n * n * sizeof(float2);
  l.complex_off = 0;
  l.partial_off = align256(cbytes);
  l.fft_off = l.partial_off + align256((size_t)3 * kShellBlocks * spectrum_shells(n) * sizeof(double));
  l.total = l.fft_off + align256(fft_work);
  return l;
}

}  // namespace

int spectrum_shells(int n) { return (int)std::floor(std::sqrt(3.0) * n / 2.0 + 0.5) + 1; }

size_t spectrum_extra_bytes(int n, char* err) {
  const Plan* p = get_plan(n, err);
  return p ? layout(n, p->work).total : 0;
}

hipError_t spectrum_launch(const float* ux, const float* uy, const float* uz, int n, double u0, void* work,
                           size_t work_bytes, double* out, hipStream_t st, char* err) {
  const Plan* p = get_plan(n, err);
  if (!p) return hipErrorUnknown;
  const Layout l = layout(n, p->work);
  if (work_bytes < l.total) {
    snprintf(err, 512, "spectrum work buffer has %zu bytes, needs %zu", work_bytes, l.total);
    return hipErrorInvalidValue;
  }
  char* base = static_cast<char*>(work);
  float2* cbuf = reinterpret_cast<float2*>(base + l.complex_off);
  double* partial = reinterpret_cast<double*>(base + l.partial_off);
  rocfft_execution_info info = nullptr;
  if (rocfft_execution_info_create(&info) != rocfft_status_success) {
    snprintf(err, 512, "rocfft_execution_info_create failed");
    return hipErrorUnknown;
  }
  hipError_t e = hipSuccess;
  bool ok = rocfft_execution_info_set_stream(info, st) == rocfft_status_success;
  if (ok && p->work > 0)
    ok = rocfft_execution_info_set_work_buffer(info, base + l.fft_off, p->work) == rocfft_status_success;
  const int nshell = spectrum_shells(n);
  const double scale = 1.0 / (2.0 * std::pow((double)n, 6.0) * u0 * u0);
  const float* comps[3] = {ux, uy, uz};
  for (int c = 0; ok && c < 3; ++c) {
    void* in[1] = {const_cast<float*>(comps[c])};
    void* outp[1] = {cbuf};
    ok = rocfft_execute(p->plan, in, outp, info) == rocfft_status_success;
    if (!ok) break;
    hipLaunchKernelGGL(shell_kernel, dim3(kShellBlocks), dim3(kShellThreads), nshell * sizeof(double), st, cbuf, n,
                       nshell, scale, partial + (size_t)c * kShellBlocks * nshell);
    e = hipGetLastError();
    if (e != hipSuccess) break;
  }
  rocfft_execution_info_destroy(info);
  if (!ok) {
    snprintf(err, 512, "rocFFT execution failed for %d^3", n);
    return hipErrorUnknown;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(shell_reduce_kernel, dim3((nshell + 255) / 256), dim3(256), 0, st, partial, 3 * kShellBlocks,
                     nshell, out);
  return hipGetLastError();
}

}  // namespace stgv
