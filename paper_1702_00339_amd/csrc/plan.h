// Host-side plan of the lattice core-Hamiltonian library and the launch
// functions each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lhf_internal.h"
#include "../../include/lhf.h"

struct lhf_plan_s {
  int32_t prec = 0;
  int32_t gram = 0;
  int32_t nlat = 0;
  int device = 0;
  std::vector<lhf::LatDev> lat;         // host copy of the device table
  lhf::LatDev* d_lat = nullptr;         // device table [nlat]
  double2* d_tw64 = nullptr;            // twiddles, complex128
  float2* d_tw32 = nullptr;             // twiddles, complex64
  int32_t* d_canon = nullptr;           // canonical block of each conjugate pair, per lattice
  lhf::GramItem* d_gram_items = nullptr;  // grouped Gram work list
  int32_t n_gram_items = 0;
  std::vector<int64_t> canon_off;       // offset of each lattice's list in d_canon
  std::vector<int32_t> ncanon;          // list length per lattice
  lhf_sizes sizes{};
  // element counts of the workspace sections
  int64_t fac_doubles = 0;
  int64_t part_elems = 0;
  int64_t dft_tmp_elems = 0;            // complex elements of one DFT ping-pong buffer
  // byte offsets of the workspace sections
  size_t ws_fac = 0, ws_grams64 = 0, ws_grams32 = 0, ws_part64 = 0, ws_part32 = 0;
  size_t ws_dft_a = 0, ws_dft_b = 0, ws_U = 0, ws_info = 0;
};

namespace lhf {

void set_error(const std::string& msg);

// Workspace view of one call.
struct Ws {
  double* fac;
  double* grams64;
  float* grams32;
  double* part64;
  float* part32;
  void* dft_a;
  void* dft_b;
  float2* U;
  int32_t* info32;
};
Ws ws_view(const lhf_plan_s* p, void* base);

// factors.hip
hipError_t launch_factors(const lhf_plan_s* p, int li, double* fac, hipStream_t s);
// gram.hip: every lattice and dimension of the plan in one grouped launch
// (mode LHF_GRAM_*), then one grouped split-K reduction into the Gram layout
hipError_t launch_grams(const lhf_plan_s* p, int mode, const double* fac, void* part, void* grams,
                        hipStream_t s);
// combine.hip
hipError_t launch_combine(const lhf_plan_s* p, int li, const double* g64, const float* g32,
                          double* H64, double* S64, float* H32, float* S32, hipStream_t s);
// blockdft.hip
hipError_t launch_block_dft(const lhf_plan_s* p, int li, int prec, const void* gen_h, const void* gen_s,
                            void* bar_h, void* bar_s, void* tmp_a, void* tmp_b, hipStream_t s);
int64_t block_dft_tmp_elems(const LatDev& L);
// heev.hip
hipError_t launch_heev(const lhf_plan_s* p, int li, uint32_t flags, const void* Hbar,
                       const void* Sbar, const void* Hbar64, const void* Sbar64,
                       const double* Hgen64, const double* Sgen64, double* w, void* V,
                       int32_t* info, float2* U, int32_t* info32, hipStream_t s);

}  // namespace lhf
