// extern "C" hot-path entry points: argument checks, workspace carving and
// the launch sequence of each stage.  Nothing here allocates.
#include <string>

#include "plan.h"

using namespace lhf;

namespace {

int32_t check_ws(const lhf_plan_s* p, const void* ws, size_t bytes) {
  if (p->sizes.ws_bytes > 0 && (!ws || bytes < p->sizes.ws_bytes)) {
    set_error("workspace of " + std::to_string(bytes) + " bytes given, " +
              std::to_string(p->sizes.ws_bytes) + " needed");
    return LHF_ERR_WORKSPACE;
  }
  return LHF_OK;
}

int32_t hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LHF_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return LHF_ERR_HIP;
}

}  // namespace

extern "C" {

int32_t lhf_assemble_blocks(lhf_plan_t p, void* H_gen, void* S_gen, double* grams64, double* H_gen64,
                            double* S_gen64, void* ws, size_t ws_bytes, lhf_stream_t stream) {
  if (!p) { set_error("NULL plan"); return LHF_ERR_INVALID; }
  if ((H_gen == nullptr) != (S_gen == nullptr)) { set_error("give both stacks H_gen and S_gen or neither"); return LHF_ERR_INVALID; }
  if ((H_gen64 == nullptr) != (S_gen64 == nullptr)) { set_error("give both FP64 stacks or neither"); return LHF_ERR_INVALID; }
  const bool grams_only = !H_gen && !H_gen64;   // factors and FP64 Grams only (for lhf_fourier_blocks)
  if (!H_gen && H_gen64 && p->prec != LHF_PREC_MIXED) {
    set_error("H_gen and S_gen are required (a mixed plan may omit them when it writes the FP64 stacks)");
    return LHF_ERR_INVALID;
  }
  if (p->prec == LHF_PREC_FP64 && H_gen64) { set_error("FP64 plans write their FP64 stacks to H_gen/S_gen"); return LHF_ERR_INVALID; }
  int32_t st = check_ws(p, ws, ws_bytes);
  if (st != LHF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = ws_view(p, ws);
  double* g64 = grams64 ? grams64 : w.grams64;
  hipError_t e;
  const bool mixed = p->prec == LHF_PREC_MIXED;
  if (grams_only) {
    e = launch_factors(p, w.fac, s);
    if ((st = hip_status(e, "factors")) != LHF_OK) return st;
    return hip_status(launch_grams(p, LHF_GRAM_FP64, w.fac, w.part64, g64, s), "gram fp64");
  }
  const bool want32 = !mixed || H_gen != nullptr;   // mixed plans: FP32 stacks only when asked for
  const bool split = mixed && p->gram != LHF_GRAM_FP64 && want32;
  const bool need64 = !mixed || !split || grams64 || H_gen64;
  e = launch_factors(p, w.fac, s);
  if ((st = hip_status(e, "factors")) != LHF_OK) return st;
  if (need64) {
    e = launch_grams(p, LHF_GRAM_FP64, w.fac, w.part64, g64, s);
    if ((st = hip_status(e, "gram fp64")) != LHF_OK) return st;
  }
  if (split) {
    e = launch_grams(p, p->gram, w.fac, w.part32, w.grams32, s);
    if ((st = hip_status(e, "gram split")) != LHF_OK) return st;
  }
  if (!mixed)
    e = launch_combine(p, g64, nullptr, (double*)H_gen, (double*)S_gen, nullptr, nullptr, s);
  else
    e = launch_combine(p, g64, split ? w.grams32 : nullptr, H_gen64, S_gen64, want32 ? (float*)H_gen : nullptr,
                       want32 ? (float*)S_gen : nullptr, s);
  return hip_status(e, "combine");
}

static int32_t block_fft(lhf_plan_t p, int32_t prec, const void* H_gen, const void* S_gen, void* H_bar,
                         void* S_bar, void* ws, size_t ws_bytes, lhf_stream_t stream, bool half) {
  if (!p) { set_error("NULL plan"); return LHF_ERR_INVALID; }
  if (prec != LHF_PREC_FP64 && prec != LHF_PREC_MIXED) { set_error("bad precision"); return LHF_ERR_INVALID; }
  if (!H_gen || !S_gen || !H_bar || !S_bar) { set_error("all four stacks are required"); return LHF_ERR_INVALID; }
  int32_t st = check_ws(p, ws, ws_bytes);
  if (st != LHF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = ws_view(p, ws);
  return hip_status(launch_block_dft(p, prec, H_gen, S_gen, H_bar, S_bar, w.dft, nullptr, nullptr, s, half),
                    "block dft");
}

int32_t lhf_block_fft(lhf_plan_t p, int32_t prec, const void* H_gen, const void* S_gen, void* H_bar,
                      void* S_bar, void* ws, size_t ws_bytes, lhf_stream_t stream) {
  return block_fft(p, prec, H_gen, S_gen, H_bar, S_bar, ws, ws_bytes, stream, false);
}

int32_t lhf_block_fft_half(lhf_plan_t p, int32_t prec, const void* H_gen, const void* S_gen, void* H_half,
                           void* S_half, void* ws, size_t ws_bytes, lhf_stream_t stream) {
  return block_fft(p, prec, H_gen, S_gen, H_half, S_half, ws, ws_bytes, stream, true);
}

int32_t lhf_block_fft_dual(lhf_plan_t p, const double* H_gen64, const double* S_gen64, void* H_bar64,
                           void* S_bar64, void* H_bar32, void* S_bar32, void* ws, size_t ws_bytes,
                           lhf_stream_t stream) {
  if (!p) { set_error("NULL plan"); return LHF_ERR_INVALID; }
  if (!H_gen64 || !S_gen64 || !H_bar64 || !S_bar64 || !H_bar32 || !S_bar32) {
    set_error("all six stacks are required");
    return LHF_ERR_INVALID;
  }
  int32_t st = check_ws(p, ws, ws_bytes);
  if (st != LHF_OK) return st;
  Ws w = ws_view(p, ws);
  return hip_status(launch_block_dft(p, LHF_PREC_FP64, H_gen64, S_gen64, H_bar64, S_bar64, w.dft, (float2*)H_bar32,
                                     (float2*)S_bar32, static_cast<hipStream_t>(stream)),
                    "block dft");
}

static int32_t fourier_blocks(lhf_plan_t p, const double* grams64, void* H_bar64, void* S_bar64, void* ws,
                              size_t ws_bytes, lhf_stream_t stream, bool half) {
  if (!p) { set_error("NULL plan"); return LHF_ERR_INVALID; }
  if (!H_bar64 || !S_bar64) { set_error("H_bar64 and S_bar64 are required"); return LHF_ERR_INVALID; }
  if (!p->sep_ok) {
    set_error("separable formation needs every lattice's first-dimension band within 32 slots and 64 KiB of LDS");
    return LHF_ERR_UNSUPPORTED;
  }
  int32_t st = check_ws(p, ws, ws_bytes);
  if (st != LHF_OK) return st;
  Ws w = ws_view(p, ws);
  return hip_status(launch_fourier_sep(p, grams64 ? grams64 : w.grams64, w.gh, static_cast<double2*>(H_bar64),
                                       static_cast<double2*>(S_bar64), static_cast<hipStream_t>(stream), half),
                    "separable fourier blocks");
}

int32_t lhf_fourier_blocks(lhf_plan_t p, const double* grams64, void* H_bar64, void* S_bar64, void* ws,
                           size_t ws_bytes, lhf_stream_t stream) {
  return fourier_blocks(p, grams64, H_bar64, S_bar64, ws, ws_bytes, stream, false);
}

int32_t lhf_fourier_blocks_half(lhf_plan_t p, const double* grams64, void* H_half64, void* S_half64, void* ws,
                                size_t ws_bytes, lhf_stream_t stream) {
  return fourier_blocks(p, grams64, H_half64, S_half64, ws, ws_bytes, stream, true);
}

int32_t lhf_heev_batched(lhf_plan_t p, uint32_t flags, const void* H_bar, const void* S_bar,
                         const void* H_bar64, const void* S_bar64, const double* H_gen64,
                         const double* S_gen64, double* w_out, void* V, int32_t* info, void* ws,
                         size_t ws_bytes, lhf_stream_t stream) {
  if (!p) { set_error("NULL plan"); return LHF_ERR_INVALID; }
  const bool direct = p->prec == LHF_PREC_MIXED && (flags & LHF_HEEV_REFINE_FP64) && !H_bar && !S_bar &&
                      H_bar64 && S_bar64;   // the FP32 solve reads the complex128 blocks
  if ((!direct && (!H_bar || !S_bar)) || !w_out || !info) {
    set_error("H_bar, S_bar (or, refining a mixed plan, H_bar64 and S_bar64 alone), w and info are required");
    return LHF_ERR_INVALID;
  }
  if (flags & ~(uint32_t)(LHF_HEEV_VECTORS | LHF_HEEV_REFINE_FP64 | LHF_HEEV_FP32_SOLVE)) {
    set_error("unknown flags");
    return LHF_ERR_INVALID;
  }
  if ((flags & LHF_HEEV_VECTORS) && !V) { set_error("LHF_HEEV_VECTORS needs V"); return LHF_ERR_INVALID; }
  const bool refine = p->prec == LHF_PREC_MIXED && (flags & LHF_HEEV_REFINE_FP64);
  if (p->prec == LHF_PREC_FP64 && (flags & LHF_HEEV_REFINE_FP64)) {
    set_error("refinement applies to mixed-precision plans");
    return LHF_ERR_INVALID;
  }
  if (refine && !((H_bar64 && S_bar64) || (H_gen64 && S_gen64))) {
    set_error("refinement needs complex128 blocks or the FP64 generator stacks");
    return LHF_ERR_INVALID;
  }
  int32_t st = check_ws(p, ws, ws_bytes);
  if (st != LHF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ws w = ws_view(p, ws);
  return hip_status(launch_heev(p, flags, H_bar, S_bar, H_bar64, S_bar64, H_gen64, S_gen64, w_out, V, info,
                                w.U, w.info32, s),
                    "heev");
}

}  // extern "C"
