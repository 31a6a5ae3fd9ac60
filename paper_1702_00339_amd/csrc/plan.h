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
  // grouped work tables (device), built once by lhf_plan_create
  lhf::GramItem* d_gram_items = nullptr;
  int32_t n_gram_items = 0;
  lhf::FacItem* d_fac_items = nullptr;
  int32_t n_fac_items = 0;
  int64_t* d_elem_start = nullptr;      // [nlat] first combine thread of each lattice (multiple of 256)
  int64_t combine_threads = 0;          // padded total
  lhf::DftTask* d_dft_tasks = nullptr;  // every task of every pass
  std::vector<lhf::DftLaunch> dft_launches;
  lhf::FusedTask* d_fused = nullptr;    // lattices transformed by the fused kernel
  int32_t n_fused = 0;
  int64_t fused_wgs = 0;
  int32_t fused_bmax = 0;               // largest band over the fused lattices' dimensions
  int32_t fused_lds = 0;                // bytes of LDS per workgroup for complex128
  // separable Fourier-block formation (every lattice, when each qualifies)
  bool sep_ok = false;
  lhf::FusedTask* d_sep = nullptr;      // one task per lattice that is not a chain
  int32_t n_sep = 0;
  lhf::FusedTask* d_sep_chain = nullptr;  // one task per chain (L2 = L3 = 1)
  int32_t n_sep_chain = 0;
  int64_t sep_chain_wgs = 0;
  int64_t sep_wgs = 0;
  int32_t sep_bmax = 0;                 // largest first-dimension band
  int32_t sep_lds = 0;                  // bytes of LDS per workgroup
  bool sep_async = false;               // the separable kernel stages by asynchronous copies (every lattice allows it)
  lhf::GhItem* d_gh_items = nullptr;    // 1D transforms of the Grams along dimensions 2, 3
  int32_t n_gh_items = 0;
  int64_t gh_threads = 0;
  int64_t gh_elems = 0;                 // complex elements of the transformed Grams
  int2* d_canon[4] = {nullptr, nullptr, nullptr, nullptr};  // (lattice, block) per size class M = 4, 8, 16, 32
  int32_t ncanon[4] = {0, 0, 0, 0};
  // eigensolver layout per class: one matrix entry per thread (wide) when the
  // four-entries-per-thread launch would leave SIMDs without a wavefront
  bool heev_wide[4] = {false, false, false, false};
  bool heev_fp64[4] = {false, false, false, false};   // mixed plans: class takes the FP64 solve alone
  int32_t gram_tile = 64;               // Gram work-item output tile: 64 or 32
  uint64_t tuning_gen = 0;              // bumped by every change of tuning; graphs record it
  static constexpr int64_t kWideWaves = 1024;   // one wavefront per SIMD of the device
  // tunables (planner defaults, refined by lhf_plan_autotune)
  int32_t dft_target_threads = 131072;  // threads one DFT pass aims to run
  int32_t gram_grid = 4096;             // workgroups of the grouped Gram launch
  int32_t gram_split = 256;             // split-K target: workgroups per (lattice, dimension)
  int32_t tol32_scale = 1;              // mixed plans: FP32 Jacobi tolerance multiplier
  int32_t fourier_sep = 1;              // whole steps form the Fourier blocks separably (when sep_ok)
  uint64_t signature = 0;               // plan_signature() at creation
  lhf_sizes sizes{};
  // element counts of the workspace sections
  int64_t fac_doubles = 0;
  int64_t part_elems = 0;
  int64_t dft_tmp_elems = 0;            // complex elements of the DFT intermediates
  // byte offsets of the workspace sections
  size_t ws_fac = 0, ws_grams64 = 0, ws_grams32 = 0, ws_part64 = 0, ws_part32 = 0;
  size_t ws_dft = 0, ws_U = 0, ws_info = 0, ws_gh = 0;
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
  void* dft;
  float2* U;
  int32_t* info32;
  double2* gh;
};
Ws ws_view(const lhf_plan_s* p, void* base);

constexpr int kGramSplitMax = 256;   // split-K target the workspace is sized for
void set_gram_split(LatDev& L, int d, int target);
void plan_grams(const std::vector<LatDev>& lats, std::vector<GramItem>& items, int tile);
uint64_t plan_signature(const lhf_plan_s* p);

// factors.hip: nodal factors and lattice-window potential factors of every lattice
void plan_factors(const std::vector<LatDev>& lats, std::vector<FacItem>& items);
hipError_t launch_factors(const lhf_plan_s* p, double* fac, hipStream_t s);
// gram.hip: every lattice and dimension of the plan in one grouped launch
// (mode LHF_GRAM_*), then one grouped split-K reduction into the Gram layout
hipError_t launch_grams(const lhf_plan_s* p, int mode, const double* fac, void* part, void* grams,
                        hipStream_t s);
// combine.hip: generator stacks of every lattice
hipError_t launch_combine(const lhf_plan_s* p, const double* g64, const float* g32, double* H64,
                          double* S64, float* H32, float* S32, hipStream_t s);
// blockdft.hip: planner of the grouped passes (task table, launch list and
// intermediate size in complex elements), and their launch
void plan_block_dft(const std::vector<LatDev>& lats, int64_t target_threads, std::vector<DftTask>& tasks,
                    std::vector<DftLaunch>& launches, int64_t& tmp_elems, std::vector<FusedTask>& fused,
                    int64_t& fused_wgs, int32_t& fused_bmax, int32_t& fused_lds);
// b32_h, b32_s (FP64 transforms only, may be NULL): complex64 copies of the blocks;
// half: write only the Hermitian half-space along k3, layout [L1][L2][L3/2+1][m0][m0]
// at LatDev::half_off (no complex64 copies then)
hipError_t launch_block_dft(const lhf_plan_s* p, int prec, const void* gen_h, const void* gen_s,
                            void* bar_h, void* bar_s, void* tmp, float2* b32_h, float2* b32_s, hipStream_t s,
                            bool half = false);
// blockdft.hip: separable Fourier blocks from the FP64 Grams (complex128 out)
void plan_separable(const std::vector<LatDev>& lats, std::vector<FusedTask>& tasks, std::vector<GhItem>& items,
                    int64_t& wgs, int32_t& bmax, int32_t& lds, int64_t& gh_threads, std::vector<FusedTask>& chain,
                    int64_t& chain_wgs, bool& ok, bool& async);
hipError_t launch_fourier_sep(const lhf_plan_s* p, const double* g64, double2* gh, double2* bar_h, double2* bar_s,
                              hipStream_t s, bool half = false);
// eigvec.hip: full-lattice eigenvectors of selected (block, column) pairs of one lattice
hipError_t launch_eigvecs(const lhf_plan_s* p, int li, const double2* V, int nsel, const int32_t* sel, double2* U,
                          hipStream_t s);
// heev.hip: every canonical block of every lattice, one launch per size class
int heev_class(int m0);
hipError_t launch_heev(const lhf_plan_s* p, uint32_t flags, const void* Hbar, const void* Sbar,
                       const void* Hbar64, const void* Sbar64, const double* Hgen64, const double* Sgen64,
                       double* w, void* V, int32_t* info, float2* U, int32_t* info32, hipStream_t s);

}  // namespace lhf
