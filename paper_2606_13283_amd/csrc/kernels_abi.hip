// Kernel-level entry points (include/arche_kernels.h): FFT and Fermi-Dirac
// evaluation on caller-owned device buffers.
#include <map>
#include <mutex>
#include <tuple>

#include "../../include/arche_kernels.h"
#include "arche_internal.h"

namespace {

__global__ void __launch_bounds__(ARCHE_BLOCK)
k_fd_eval(const FdTables* fdt, int64_t n, const double* x, double* im12, double* ip12, double* ip32) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    double a, b;
    fd_m12_p12(fdt, v, a, b);
    if (im12) im12[i] = a;
    if (ip12) ip12[i] = b;
    if (ip32) ip32[i] = fd_eval_order(fdt, 2, v);
  }
}

// d^m I_{1/2}/dx^m, m = 0..3, as the SCF kernel evaluates them (LDS table)
__global__ void __launch_bounds__(ARCHE_BLOCK)
k_fd_derivs(const FdTables* fdt, int64_t n, const double* x, double* d0, double* d1, double* d2, double* d3) {
  __shared__ FdLds fdl;
  fd_lds_load(&fdl, fdt);
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double d[4];
    fd_p12_derivs<3>(fdl, x[i], d);
    if (d0) d0[i] = d[0];
    if (d1) d1[i] = d[1];
    if (d2) d2[i] = d[2];
    if (d3) d3[i] = d[3];
  }
}

std::mutex g_plan_mtx;
std::map<std::tuple<int, int, int, int>, FftPlan*> g_plans;  // (device, Nx, Ny, Nz), kept for the process

FftPlan* plan_for(const int32_t grid[3]) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(g_plan_mtx);
  auto key = std::make_tuple(dev, (int)grid[0], (int)grid[1], (int)grid[2]);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) return it->second;
  FftPlan* p = new FftPlan();
  int N[3] = {grid[0], grid[1], grid[2]};
  if (!fft_plan_create(p, N)) {
    delete p;
    return nullptr;
  }
  g_plans[key] = p;
  return p;
}

// ---------------------------------------------------------------------------
// Scratch of arche_k_fft_c2r_noalloc, one copy per device for the life of the
// process: first the twiddle tables exp(-2 pi i m / L) of every supported line
// length (each table starting on a 16-entry boundary, written once per device
// at set-up), then the work copy of the half spectrum that the C2R passes
// transform in place.
constexpr int64_t tw_table_slots() {
  int64_t n = 0;
  for (int L = 2; L <= 1024; L += 2) {
    int r = L;
    while (r % 2 == 0) r /= 2;
    while (r % 3 == 0) r /= 3;
    while (r % 5 == 0) r /= 5;
    if (r == 1) n += (L + 15) / 16 * 16;
  }
  return n;
}
constexpr int64_t kTwSlots = tw_table_slots();
constexpr int64_t kScratchSlots = kTwSlots + ARCHE_NOALLOC_MAX_NH;  // complex values

}  // namespace

static __device__ __align__(256) double scratch[2 * kScratchSlots];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mtx;
cplx* g_scratch_ptr[kMaxDevices] = {};  // device address of scratch, per device
int32_t g_tw_off[1025];                 // first slot of the table of length L
cplx g_tw_host[kTwSlots];               // host copy of the tables, built once

// Set-up on the current device (first call there): resolve the array's device
// address and upload the twiddle tables.  Returns the address or null.
cplx* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mtx);
  if (g_scratch_ptr[dev]) return g_scratch_ptr[dev];
  static bool host_built = false;
  if (!host_built) {
    int64_t off = 0;
    for (int L = 2; L <= 1024; L += 2) {
      if (!fft_size_supported(L)) continue;
      g_tw_off[L] = (int32_t)off;
      fft_twiddles_host(L, g_tw_host + off);
      off += (L + 15) / 16 * 16;
    }
    host_built = true;
  }
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
  if (hipMemcpy(p, g_tw_host, kTwSlots * sizeof(cplx), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  g_scratch_ptr[dev] = (cplx*)p;
  return g_scratch_ptr[dev];
}

bool grid_ok(const int32_t* grid) {
  if (!grid) return false;
  for (int a = 0; a < 3; ++a)
    if (!fft_size_supported(grid[a])) return false;
  return true;
}

}  // namespace

extern "C" {

arche_status arche_k_fft_r2c(const int32_t grid[3], const double* d_in, double* d_out, void* stream) {
  if (!grid_ok(grid) || !d_in || !d_out) return ARCHE_EINVAL;
  FftPlan* p = plan_for(grid);
  if (!p) return ARCHE_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  if (fft_r2c(p, d_in, (cplx*)d_out, 1.0, 1.0, s) != hipSuccess) return ARCHE_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? ARCHE_OK : ARCHE_EHIP;
}

arche_status arche_k_fft_c2r(const int32_t grid[3], const double* d_in, double* d_out, void* stream) {
  if (!grid_ok(grid) || !d_in || !d_out) return ARCHE_EINVAL;
  FftPlan* p = plan_for(grid);
  if (!p) return ARCHE_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  cplx* work = nullptr;
  if (hipMalloc(&work, p->nh * sizeof(cplx)) != hipSuccess) return ARCHE_ENOMEM;
  hipError_t e = hipMemcpyAsync(work, d_in, p->nh * sizeof(cplx), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = fft_c2r(p, work, d_out, 1.0, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(work);
  return e == hipSuccess ? ARCHE_OK : ARCHE_EHIP;
}

arche_status arche_k_fft_c2r_noalloc(const int32_t grid[3], const double* d_in, double* d_out, void* stream) {
  if (!grid_ok(grid) || !d_in || !d_out) return ARCHE_EINVAL;
  FftPlan p;
  const int N[3] = {grid[0], grid[1], grid[2]};
  if (!fft_plan_describe(&p, N)) return ARCHE_EINVAL;
  if (p.nh > ARCHE_NOALLOC_MAX_NH) return ARCHE_EINVAL;
  cplx* base = noalloc_scratch();
  if (!base) return ARCHE_EHIP;
  for (int a = 0; a < 3; ++a) p.ax[a].tw = base + g_tw_off[p.ax[a].L];
  p.ok = true;
  cplx* work = base + kTwSlots;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(work, d_in, p.nh * sizeof(cplx), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = fft_c2r(&p, work, d_out, 1.0, s);
  return e == hipSuccess ? ARCHE_OK : ARCHE_EHIP;
}

arche_status arche_k_fermi_dirac(int64_t n, const double* d_x, double* d_im12, double* d_ip12, double* d_ip32,
                                 void* stream) {
  if (n < 0 || (n > 0 && !d_x)) return ARCHE_EINVAL;
  if (n == 0) return ARCHE_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ARCHE_EHIP;
  const FdTables* t = fd_tables_device(dev);
  if (!t) return ARCHE_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  int64_t b = (n + ARCHE_BLOCK - 1) / ARCHE_BLOCK;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fd_eval, dim3((unsigned)b), dim3(ARCHE_BLOCK), 0, s, t, n, d_x, d_im12, d_ip12, d_ip32);
  if (hipGetLastError() != hipSuccess) return ARCHE_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? ARCHE_OK : ARCHE_EHIP;
}

arche_status arche_k_fermi_dirac_derivs(int64_t n, const double* d_x, double* d_d0, double* d_d1, double* d_d2,
                                        double* d_d3, void* stream) {
  if (n < 0 || (n > 0 && !d_x)) return ARCHE_EINVAL;
  if (n == 0) return ARCHE_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ARCHE_EHIP;
  const FdTables* t = fd_tables_device(dev);
  if (!t) return ARCHE_ENOMEM;
  hipStream_t s = (hipStream_t)stream;
  int64_t b = (n + ARCHE_BLOCK - 1) / ARCHE_BLOCK;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(k_fd_derivs, dim3((unsigned)b), dim3(ARCHE_BLOCK), 0, s, t, n, d_x, d_d0, d_d1, d_d2, d_d3);
  if (hipGetLastError() != hipSuccess) return ARCHE_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? ARCHE_OK : ARCHE_EHIP;
}

}  // extern "C"

extern "C" int32_t arche_fft_tile(int32_t pass, int32_t L, int32_t force) { return fft_tile_variant(pass, L, force); }
