// Internal descriptors and launch functions of the three-level
// block-Toeplitz operator of a lattice in a box (toeplitz3.hip).
// Plain-old-data only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lhf_internal.h"

namespace lhf {

// The box lattice, its cell template and its grids, per dimension l:
// multi-cell dimensions (L >= 2) have cell-aligned nodes x0 + i h and their
// Grams are taken on the node set extended without walls; one-cell
// dimensions are box dimensions with nodes x0 + i h, i = 1..n, and walls.
struct Toep3Dev {
  int32_t L[3], n[3], L0[3], P[3];
  int32_t m0, M0, R, pad0;
  double a;
  double h[3], x0[3];
  int32_t lpow[kMaxM0][3];
  double alpha[kMaxM0];
  double cen[kMaxM0][3];
  double Z[kMaxNuc];
  double nuc[kMaxNuc][3];
  double tq[kMaxR];
  double wq[kMaxR];
  int64_t vpot_off[3];   // potential factors of dimension l: [M0 R][vpot_len]
  int32_t vpot_len[3];   // nc (multi-cell) or n (one-cell)
  int32_t pad1;
  int64_t gram_off[3];   // 1D Grams of dimension l: [L0 + 1][T][m0][m0], T = 2 + M0 R
  int64_t gh_off[3];     // their transforms: [T][P][m0][m0] complex
};

// One (dimension, shift) of the 1D Grams; nodes [ilo, ihi] hold every
// non-negligible factor value.
struct Gram3Job {
  int32_t dim, shift, ilo, ihi;
};

// Potential factors, 1D Grams, their transforms and the embedding's
// per-frequency blocks cH, cS ([P1 P2 P3][m0][m0], complex128).
hipError_t toep3_launch_assembly(const Toep3Dev* d, const Toep3Dev& host, const Gram3Job* jobs, int njobs, int wmax,
                                 double* vpot, double* grams, double2* gh, double2* cH, double2* cS, hipStream_t s);
// Generators A_s, [2 L0_1 + 1][2 L0_2 + 1][2 L0_3 + 1][m0][m0] FP64.
hipError_t toep3_launch_generators(const Toep3Dev* d, const Toep3Dev& host, const double* grams, double* gH,
                                   double* gS, hipStream_t s);
// Workspace bytes of one embedding product of ncols columns.
size_t toep3_apply_ws_bytes(const Toep3Dev& host, int ncols, bool fp64);
// y_H = op_H x, y_S = op_S x (op_S may be NULL: one operator) through the
// embedding, in complex128 (LHF_PREC_FP64) or complex64; tw[l]: twiddles
// exp(-2 pi i k / P_l), k < P_l / 2, of the arithmetic's complex type.
hipError_t toep3_launch_apply(const Toep3Dev& host, int prec, const void* const* tw, int ncols, const double* x,
                              int ld, const void* opH, const void* opS, double* yH, double* yS, void* ws,
                              hipStream_t s);

}  // namespace lhf
