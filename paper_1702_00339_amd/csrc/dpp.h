// Cross-lane moves and all-reduces of FP64 values inside a wavefront, by DPP
// (data-parallel primitives) within 16-lane rows and lane shuffles across
// rows.  Shared by the batched eigensolver and the dense Rayleigh-Ritz
// eigensolver.
#pragma once

#include <hip/hip_runtime.h>

namespace lhf {

// FP64 lane moves within a 16-lane row (DPP control CTRL) and an all-reduce
// over aligned groups of P lanes (P a power of two <= 64): quad permutes pair
// i with i^1 and i^2, then the mirrors i <-> 7-i and i <-> 15-i join two
// halves that are already reduced; across rows the gfx950 lane swaps
// (v_permlane16_swap: odd rows of one operand with even rows of the other;
// v_permlane32_swap: upper half with lower half) applied to two copies of a
// value leave {x_i, x_(i^16)} or {x_i, x_(i^32)} in the two results, with no
// LDS round trip.
// Every source lane of these patterns lies in the destination's own group
// and is active whenever the group is, so the moves keep no old value.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
// op(x_i, x_(i^16)) and op(x_i, x_(i^32)) for every lane of a full wavefront.
template <typename F>
__device__ __forceinline__ double swap16_op(double v, F op) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return op(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
}
template <typename F>
__device__ __forceinline__ double swap32_op(double v, F op) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return op(__hiloint2double((int)h[0], (int)l[0]), __hiloint2double((int)h[1], (int)l[1]));
}

template <int P, typename F>
__device__ __forceinline__ double lane_reduce(double v, F op) {
  if constexpr (P >= 2) v = op(v, dpp_move<0xB1>(v));    // quad_perm [1, 0, 3, 2]
  if constexpr (P >= 4) v = op(v, dpp_move<0x4E>(v));    // quad_perm [2, 3, 0, 1]
  if constexpr (P >= 8) v = op(v, dpp_move<0x141>(v));   // row_half_mirror
  if constexpr (P >= 16) v = op(v, dpp_move<0x140>(v));  // row_mirror
  if constexpr (P >= 32) v = swap16_op(v, op);
  if constexpr (P >= 64) v = swap32_op(v, op);
  return v;
}
// Two independent all-reduces, level by level, so their latencies overlap.
template <int P, typename F>
__device__ __forceinline__ void lane_reduce2(double& a, double& b, F op) {
  if constexpr (P >= 2) { const double x = dpp_move<0xB1>(a), y = dpp_move<0xB1>(b); a = op(a, x); b = op(b, y); }
  if constexpr (P >= 4) { const double x = dpp_move<0x4E>(a), y = dpp_move<0x4E>(b); a = op(a, x); b = op(b, y); }
  if constexpr (P >= 8) { const double x = dpp_move<0x141>(a), y = dpp_move<0x141>(b); a = op(a, x); b = op(b, y); }
  if constexpr (P >= 16) { const double x = dpp_move<0x140>(a), y = dpp_move<0x140>(b); a = op(a, x); b = op(b, y); }
  if constexpr (P >= 32) {
    a = swap16_op(a, op);
    b = swap16_op(b, op);
  }
  if constexpr (P >= 64) {
    a = swap32_op(a, op);
    b = swap32_op(b, op);
  }
}

}  // namespace lhf
