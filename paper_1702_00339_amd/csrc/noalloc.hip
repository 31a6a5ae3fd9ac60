// lhf_fourier_blocks_noalloc: the separable Fourier-block formation without a
// caller workspace, for callers that cannot allocate device memory.
//
// The only scratch of the separable formation is the 1D-transformed Grams of
// dimensions 2 and 3 (complex128, T L m0^2 per lattice and dimension), which
// gram_dft_kernel writes in full before sep_fused_kernel reads them, so
// nothing in it has to start at zero.  Here it lives in a file-scope device
// array of fixed size.  Every GPU the library runs on holds its own copy of
// the array at its own address until the process ends; that address is
// looked up once per device with hipGetSymbolAddress (in host code the
// array's name is not a device address) and passed to the kernels like the
// workspace pointer of lhf_fourier_blocks.  Calls that overlap on one device
// share the array and race on it.
#include <mutex>
#include <string>

#include "plan.h"

static constexpr size_t kScratchBytes = LHF_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % sizeof(double2) == 0, "whole complex128 elements");

static __device__ __align__(256) double2 scratch[kScratchBytes / sizeof(double2)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double2* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev` (looked up on
// the first call there).
int32_t scratch_address(int dev, double2** out) {
  if (dev < 0 || dev >= kMaxDevices) {
    lhf::set_error("device index " + std::to_string(dev) + " beyond the static scratch table");
    return LHF_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      lhf::set_error(std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
      return LHF_ERR_HIP;
    }
    g_scratch[dev] = static_cast<double2*>(ptr);
  }
  *out = g_scratch[dev];
  return LHF_OK;
}

}  // namespace

extern "C" int32_t lhf_fourier_blocks_noalloc(lhf_plan_t p, const double* grams64, void* H_bar64, void* S_bar64,
                                              lhf_stream_t stream) {
  if (!p) { lhf::set_error("NULL plan"); return LHF_ERR_INVALID; }
  if (!grams64 || !H_bar64 || !S_bar64) {
    lhf::set_error("grams64, H_bar64 and S_bar64 are required");
    return LHF_ERR_INVALID;
  }
  if (!p->sep_ok) {
    lhf::set_error("separable formation needs every lattice's first-dimension band within 32 slots and 64 KiB of LDS");
    return LHF_ERR_UNSUPPORTED;
  }
  const size_t need = (size_t)p->gh_elems * sizeof(double2);
  if (need > kScratchBytes) {
    lhf::set_error("the plan's transformed Grams need " + std::to_string(need) + " bytes, the static scratch holds " +
                   std::to_string(kScratchBytes) + ": use lhf_fourier_blocks with a workspace");
    return LHF_ERR_UNSUPPORTED;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    lhf::set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return LHF_ERR_HIP;
  }
  if (dev != p->device) {
    lhf::set_error("the plan lives on device " + std::to_string(p->device) + ", the current device is " +
                   std::to_string(dev));
    return LHF_ERR_INVALID;
  }
  double2* gh = nullptr;
  int32_t st = scratch_address(dev, &gh);
  if (st != LHF_OK) return st;
  e = lhf::launch_fourier_sep(p, grams64, gh, static_cast<double2*>(H_bar64), static_cast<double2*>(S_bar64),
                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    lhf::set_error(std::string("separable fourier blocks: ") + hipGetErrorString(e));
    return LHF_ERR_HIP;
  }
  return LHF_OK;
}
