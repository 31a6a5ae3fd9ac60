// Internal descriptors and launch functions of the Dirichlet-chain operator
// (perturbed block-Toeplitz model) and of the dense FP64 kernels its block
// LOBPCG driver uses.  Plain-old-data only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "lhf_internal.h"

namespace lhf {

constexpr int kMaxSmall = 112;   // largest dense eigenproblem of the LOBPCG driver (LDS bound)
constexpr int kMaxCols = 128;    // vectors per matvec call

// The chain, its cell template and its grids.
struct ToepDev {
  int32_t L, nc, n, m0, M0, R, L0, P, ndef, margin;
  double a, h, x0;                   // chain node i (any integer) at x0 + i h; box nodes i = 1..n
  int32_t nt[2];                     // transverse nodes (dimensions 2, 3), i = 1..nt
  double ht[2], t0[2];               // transverse spacing and origin
  int32_t lpow[kMaxM0][3];
  double alpha[kMaxM0];
  double cen[kMaxM0][3];
  double Z[kMaxNuc];
  double nuc[kMaxNuc][3];
  double tq[kMaxR];
  double wq[kMaxR];
};

// One block of the model: rows = functions of cell k, columns = functions of
// cell m.  mode 0: pristine generator on the wall-free grid; 1: cross block of
// the actual basis on the box grid; 2: block of the exact box operator (the
// actual basis on the box grid, the finite lattice's own potential).  dk, dm: defect index of the cells or -1;
// pair: index of the transverse Grams for the pair of exponent scales;
// chain nodes [ilo, ihi] (inclusive) carry every non-negligible factor value.
struct ToepJob {
  int32_t k, m, mode, pair, ilo, ihi, dk, dm;
};

// A pair of exponent scales (defect index or -1 for the pristine cell).
struct ScalePair {
  int32_t dk, dm;
};

// One term of a cross correction of block row k: y_k += D x_m with
// D = H_model(k, m) - T(k, m), built from cross block `blk` (transposed when
// the block is stored as (m, k)).
struct CrossEntry {
  int32_t m, blk, trans, pad;
};

struct Defect {
  int32_t cell, pad;
  double Z, scale;
};

// assembly (toeplitz.hip)
hipError_t toep_launch_vrep(const ToepDev* d, double* vrep, int M0R, int nc, hipStream_t s);
// the finite lattice's potential along the chain on every box node [M0 R][n]
// (Z w_q folded in; cell_def[c]: defect index of cell c or -1)
hipError_t toep_launch_vbox(const ToepDev* d, const Defect* defs, const int32_t* cell_def, double* vbox, int M0R,
                            int n, hipStream_t s);
hipError_t toep_launch_transverse(const ToepDev* d, const Defect* defs, const ScalePair* pairs, int npairs,
                                  int m0, int M0R, double* trans, hipStream_t s);
// wmax: largest chain window (ihi - ilo + 1) over the jobs
// vbox: the finite-lattice potential for mode-2 jobs (may be NULL without them)
hipError_t toep_launch_blocks(const ToepDev* d, const Defect* defs, const ToepJob* jobs, int njobs, int m0, int wmax,
                              const double* vrep, const double* vbox, const double* trans, double* outH,
                              double* outS, hipStream_t s);
// genH, genS NULL: the entries are the model blocks themselves (no T to subtract)
hipError_t toep_launch_delta(const ToepDev* d, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                             const CrossEntry* ent, const double* genH, const double* genS, const double* crossH,
                             const double* crossS, double* dH, double* dS, int m0, hipStream_t s);
hipError_t toep_launch_chat(const ToepDev* d, const double* genH, const double* genS, double2* cH, double2* cS,
                            int m0, int P, int L0, hipStream_t s);
hipError_t toep_launch_minv(const double2* V, const double* w, double sigma, double2* minv64, float2* minv32,
                            int P, int m0, hipStream_t s);
hipError_t toep_launch_to32(const double2* src, float2* dst, int64_t n, hipStream_t s);
// y = T x (+ crosses); prec: LHF_PREC_FP64 or LHF_PREC_MIXED.  op2 may be NULL
// (one operator: yS unused).  cross lists may be empty (nrows = 0).  exact:
// no Toeplitz part; y = the block rows' entries applied to x (every block row
// must have entries).
hipError_t toep_launch_apply(int prec, int L, int m0, int P, int ncols, const double* x, int ld,
                             const void* opH, const void* opS, const void* tw, void* xhat, void* yhatH,
                             void* yhatS, double* yH, double* yS, const int32_t* row_ptr, const int32_t* row_cell,
                             int nrows, const CrossEntry* ent, const double* dH, const double* dS, hipStream_t s,
                             bool exact = false);
// the same with FP32 x and y: complex64 transform, crosses accumulated in FP64
hipError_t toep_launch_apply32(int L, int m0, int P, int ncols, const float* x, int ld, const void* opH,
                               const void* opS, const void* tw, void* xhat, void* yhatH, void* yhatS, float* yH,
                               float* yS, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                               const CrossEntry* ent, const double* dH, const double* dS, hipStream_t s,
                               bool exact = false);

// dense FP64 kernels (lobpcg.hip); row-major [N][ld] blocks of vectors
hipError_t dense_gram(int N, int k1, int k2, const double* A, int lda, const double* B, int ldb, double* part,
                      int nchunk, double* G, int ldg, hipStream_t s);
// Y = beta Z + A T   (Z may alias nothing; beta = 0 ignores Z)
hipError_t dense_combine(int N, int k1, int k2, const double* A, int lda, const double* T, int ldt, double beta,
                         const double* Z, int ldz, double* Y, int ldy, hipStream_t s);
// Y_a = A_a T for three blocks sharing T (one launch); k2 <= kMaxSmall
hipError_t dense_combine3(int N, int k1, int k2, const double* A0, const double* A1, const double* A2, int lda,
                          const double* T, int ldt, double* Y0, double* Y1, double* Y2, int ldy, hipStream_t s);
// the k lowest eigenpairs (ascending in w, eigenvector i in column i of V,
// row-major, ldv >= k; 1 <= k <= m <= kMaxSmall): tridiagonalisation,
// bisection, inverse iteration, back-transform (rrsyev.hip), in LDS
hipError_t dense_syev_low(int m, int k, const double* A, int lda, double* w, double* V, int ldv, hipStream_t s);
hipError_t dense_residual(int N, int k, const double* HX, const double* SX, int ld, const double* theta, double* R,
                          int ldr, double* part, int nchunk, double* norms, hipStream_t s);
hipError_t dense_random(int N, int k, uint64_t seed, double* X, int ld, hipStream_t s);
hipError_t dense_copy_cols(int N, int k, const double* A, int lda, double* B, int ldb, hipStream_t s);
// Cholesky-QR with deflation of the Gram matrix G (read as (G + G^T) / 2 and
// scaled on load to Gs = D G D, D = diag(G)^-1/2): columns whose pivot (the
// squared distance of scaled column j from the span of the kept columns
// before it) is <= drop are dropped; T (m x kk) = D L^-T diag(p)^-1/2 on the
// kept columns, so T^T G T = I; kk written to *kk_out as a double
hipError_t dense_cholqr(int m, const double* G, int ldg, double drop, double* T, int ldt, double* kk_out,
                        hipStream_t s);

}  // namespace lhf
