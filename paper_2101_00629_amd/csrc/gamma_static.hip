// ka_gamma_apply_static: the raw fused kernel product with its scratch (split-K
// partial sums, BF16 hi/lo parts of Y) in a file-scope device array instead of
// a caller-provided or library-allocated workspace, for callers that cannot
// allocate device memory (code under stream capture, serving loops that forbid
// allocation).  The kernels are those of ka_gamma_apply.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ka_internal.hpp"

namespace {

// One copy per GPU, held until the process ends.  In host code `scratch` names
// a host-side stand-in; its device address comes from hipGetSymbolAddress.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current); nullptr and an error message on failure.
void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ka::set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t ka_gamma_static_capacity(void) { return kStaticScratchBytes; }

int ka_gamma_apply_static(int kernel, double sigma, double ell, const float* xr_dev, int64_t nr, const float* xc_dev,
                          int64_t nc, const float* Y_dev, int b, float* Z_dev, int precision, void* stream) {
  using namespace ka;
  if (kernel != KA_GAUSSIAN && kernel != KA_EXP_L1) return fail(KA_ERR_ARG, "bad kernel");
  if (precision != KA_FP32 && precision != KA_BF16X3) return fail(KA_ERR_ARG, "bad precision");
  if (b != 16 && b != 32 && b != 64) return fail(KA_ERR_ARG, "b must be 16, 32 or 64");
  if (nr < 0 || nc < 0) return fail(KA_ERR_ARG, "negative size");
  if (!(ell > 0) || !(sigma > 0)) return fail(KA_ERR_ARG, "ell and sigma must be > 0");
  if (nr == 0) return KA_OK;
  if (!xr_dev || !Z_dev || (nc > 0 && (!xc_dev || !Y_dev))) return fail(KA_ERR_ARG, "NULL pointer");
  if (((uintptr_t)Y_dev & 15) != 0) return fail(KA_ERR_ARG, "Y must be 16-byte aligned");
  const GammaPlan gp = gamma_plan(nr, nc, b, precision);
  if (gp.work_bytes > kStaticScratchBytes)
    return fail(KA_ERR_ARG, "product needs " + std::to_string(gp.work_bytes) + " scratch bytes, more than the " +
                                std::to_string(kStaticScratchBytes) + " of the static scratch (use ka_gamma_apply)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return fail(KA_ERR_HIP, "no current device");
  void* work = scratch_ptr(dev);
  if (!work) return KA_ERR_HIP;
  GammaLaunch g;
  g.xr = xr_dev;
  g.xr_stride = 3;
  g.rs = nullptr;
  g.nr = nr;
  g.xc = xc_dev;
  g.xc_stride = 3;
  g.nc = nc;
  g.Y = Y_dev;
  g.Z = Z_dev;
  g.partial = (float*)work;   // every entry a launch reads is written by the same launch first
  g.ys = nullptr;             // launch_gamma places it in the scratch
  g.coord_scale = kernel_coord_scale(kernel, ell);
  g.out_scale = (float)(sigma * sigma);
  g.nsplit = 1;
  g.cols_per_split = 0;
  g.row_blocks = 0;
  g.xcd_splits = 0;
  const hipError_t e = launch_gamma(g, kernel, b, precision, (hipStream_t)stream);
  if (e != hipSuccess) return fail(KA_ERR_HIP, std::string("kernel product launch: ") + hipGetErrorString(e));
  return KA_OK;
}

}  // extern "C"
