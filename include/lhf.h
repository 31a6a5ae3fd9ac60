/*
 * lhf.h -- C ABI of the MI355X (gfx950) lattice core-Hamiltonian library.
 *
 * The library implements the periodic-lattice hot path of Khoromskaia and
 * Khoromskij, "Block circulant and Toeplitz structures in the linearized
 * Hartree-Fock equation on finite lattices: tensor approach"
 * (arXiv:1702.00339):
 *   1. assemble the m0 x m0 generator blocks of the three-level
 *      block-circulant Galerkin matrices H (core Hamiltonian) and S (overlap)
 *      from 1D Gram contractions on the grid                  (lhf_assemble_blocks)
 *   2. block-diagonalise them by a Fourier transform over the lattice
 *      index                                                  (lhf_block_fft)
 *   3. solve the L1 L2 L3 small generalized Hermitian eigenproblems
 *                                                             (lhf_heev_batched)
 * plus the Dirichlet-box block-Toeplitz matvec by circulant embedding
 * (lhf_toeplitz_*).
 *
 * Conventions
 *   * Units: bohr and hartree.
 *   * Every pointer named d_* or documented "device" is HIP device memory the
 *     caller owns; every other pointer is host memory read before the call
 *     returns.  The library never keeps a caller pointer.
 *   * Hot calls (assemble, fft, heev, toeplitz_matvec) enqueue work on the
 *     given stream (a hipStream_t; NULL is the null stream), return at once,
 *     allocate nothing and use only the caller's workspace.  Buffers must stay
 *     alive until the stream has completed the work.
 *   * Argument errors are reported synchronously by the return code before
 *     anything is launched; numerical failures are reported per block in the
 *     device array `info` (LAPACK style).  lhf_last_error() gives a message
 *     for the last failing call of the calling thread.
 *   * Plans are immutable after creation apart from their tuning
 *     (lhf_plan_set_tuning, lhf_plan_autotune, which need the plan idle) and
 *     may be used from several streams at once, each with its own workspace.
 */
#ifndef LHF_H
#define LHF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* lhf_stream_t;          /* a hipStream_t */
typedef struct lhf_plan_s* lhf_plan_t;
typedef struct lhf_toeplitz_s* lhf_toeplitz_t;

/* Status codes returned by every call. */
enum {
  LHF_OK = 0,
  LHF_ERR_INVALID = -1,      /* an argument or descriptor is invalid          */
  LHF_ERR_UNSUPPORTED = -2,  /* valid input outside what the library supports */
  LHF_ERR_WORKSPACE = -3,    /* workspace missing or smaller than required    */
  LHF_ERR_HIP = -4,          /* a HIP runtime call failed                     */
  LHF_ERR_ALLOC = -5         /* plan creation could not allocate              */
};

/* Pipeline precision. */
enum {
  LHF_PREC_FP64 = 0,   /* FP64 Grams, FP64 stacks, complex128 blocks, FP64 solve */
  LHF_PREC_MIXED = 1   /* split-precision MFMA Grams, FP32 stacks, complex64 blocks,
                          FP32 Jacobi, FP64 eigenpair refinement                 */
};

/* Arithmetic of the Gram contractions that feed the mixed-precision stack. */
enum {
  LHF_GRAM_FP64 = 0,   /* FP64 MFMA (also what the FP64 pipeline always uses)  */
  LHF_GRAM_FP32 = 1,   /* FP32 MFMA on FP32-rounded operands                   */
  LHF_GRAM_BF16X3 = 2, /* bf16 hi+lo split, hi*hi + hi*lo + lo*hi, FP32 accum.  */
  LHF_GRAM_FP16X3 = 3  /* FP16 hi+lo split as above, operand rows and columns
                          scaled by powers of two per work item (22 bits)     */
};

/* Boundary conditions. */
enum { LHF_BC_PERIODIC = 0, LHF_BC_DIRICHLET = 1 };

/* Angular type of a basis function: power 1 of one coordinate. */
enum { LHF_ANG_S = 0, LHF_ANG_PX = 1, LHF_ANG_PY = 2, LHF_ANG_PZ = 3 };

/* heev flags. */
enum {
  LHF_HEEV_VECTORS = 1u,      /* write eigenvectors to V                          */
  LHF_HEEV_REFINE_FP64 = 2u,  /* mixed precision: refine every eigenpair in FP64 */
  LHF_HEEV_FP32_SOLVE = 4u    /* mixed precision: every size class takes the FP32
                                 solve + FP64 refinement, whatever the tuning's
                                 heev_fp64 mask; the autotuner then keeps it 0 */
};

/*
 * Unit cell (paper Sec. 2.1, eqs. ElectrostPot and expand; Sec. 2.3):
 * m0 Gaussian basis functions g(x) = prod_l N (x_l - c_l)^{p_l}
 * exp(-alpha |x - c|^2) with p = 0 except p_l = 1 for a p function along l,
 * each 1D factor normalised to one; M0 nuclei of charge Z.  Positions are
 * relative to the cell centre.
 */
typedef struct {
  int32_t m0;            /* 1..32                                    */
  const double* alpha;   /* [m0] exponents, > 0                      */
  const double* centre;  /* [m0][3]                                  */
  const int32_t* ang;    /* [m0] LHF_ANG_*, NULL = all s             */
  int32_t M0;            /* 1..4                                     */
  const double* Z;       /* [M0] charges, > 0                        */
  const double* nuc;     /* [M0][3]                                  */
} lhf_cell;

/*
 * Lattice system (paper Sec. 2.3 and 3.3): L1 x L2 x L3 cells of step a,
 * n nodes per dimension, periodic or Dirichlet.  A dimension is periodic when
 * bc is periodic and L >= 2: nodes x_i = i h, h = L a / n (n a multiple of L),
 * cell k centred at (k + 1/2) a.  Otherwise it is a box dimension of width
 * L a + 2 pad with nodes -W/2 + i h, i = 1..n, h = W / (n + 1) and zero
 * Dirichlet values outside.  1/r is the R-term Gaussian sum with nodes
 * t_q = exp(sinc_u0 + q sinc_step) and weights 2/sqrt(pi) sinc_step t_q
 * (eq. sinc_general).  L0[l] is the generator band half-width: blocks with a
 * lattice offset beyond L0 in dimension l are taken as zero; a negative value
 * lets the library choose it from the smallest exponent (Gaussian overlap
 * decay below 1e-22), a value >= (L-1)/2 keeps every offset.
 */
typedef struct {
  int32_t L[3];
  int32_t n[3];
  double a;
  double pad[3];
  int32_t bc;            /* LHF_BC_*                                  */
  int32_t R;             /* 1..64, M0 R <= 96                         */
  double sinc_u0;
  double sinc_step;
  int32_t L0[3];
  lhf_cell cell;
} lhf_lattice;

/* Element counts of the caller's buffers for a plan (all lattices concatenated). */
typedef struct {
  int64_t nlat;
  int64_t nblocks;       /* sum L1 L2 L3: Fourier blocks (k points)               */
  int64_t gen_elems;     /* sum L1 L2 L3 m0^2: one generator / Fourier-block stack */
  int64_t w_elems;       /* sum L1 L2 L3 m0: eigenvalues                           */
  int64_t grams_elems;   /* FP64 elements of the 1D Gram buffer                    */
  size_t ws_bytes;       /* workspace bytes every hot call of this plan needs      */
  int64_t half_elems;    /* sum L1 L2 (L3/2 + 1) m0^2: a Fourier-block stack in the
                            Hermitian half-space along k3 (lhf_block_fft_half)     */
} lhf_sizes;

/* ---------------------------------------------------------------- plans
 * Validate nlat lattice descriptors, derive grids, bands, split factors and
 * buffer offsets, and upload the per-lattice tables to device memory of the
 * current HIP device (synchronously; this is the only call that allocates).
 * prec: LHF_PREC_*; gram: LHF_GRAM_* (the stack Gram of the mixed pipeline;
 * ignored for FP64).  Periodic and one-cell dimensions only; a Dirichlet
 * dimension with L >= 2 is accepted only by lhf_toeplitz_create.
 * Errors: LHF_ERR_INVALID (bad descriptor), LHF_ERR_UNSUPPORTED (m0 > 32,
 * M0 R > 96, ...), LHF_ERR_ALLOC, LHF_ERR_HIP.  *out is NULL on error. */
int32_t lhf_plan_create(const lhf_lattice* lats, int32_t nlat, int32_t prec, int32_t gram,
                        lhf_plan_t* out);
int32_t lhf_plan_sizes(lhf_plan_t plan, lhf_sizes* out);
/* Workspace bytes for every hot call of the plan (same as lhf_sizes.ws_bytes). */
size_t lhf_workspace_size(lhf_plan_t plan);
/* Generator slots per dimension of lattice `index` (nshift[l]: offsets
 * 0..L-1 when full[l] = 1, else -L0..L0 with L0[l] given) -- the band the
 * plan uses for the Grams, the generator stacks and the block DFT.
 * Errors: LHF_ERR_INVALID (NULL pointer, index out of range). */
int32_t lhf_plan_band(lhf_plan_t plan, int32_t index, int32_t* nshift, int32_t* L0, int32_t* full);
/* Free the plan's device tables.  No work using it may be pending. */
int32_t lhf_plan_destroy(lhf_plan_t plan);

/* ---------------------------------------------------------------- assembly
 * Generator blocks A_k = block(k, 0) of the block-circulant matrices, i.e.
 * A_k(mu, nu) = <g_(k,mu), Op g_(0,nu)> for Op = H and S (Lemma 3.4, eqs.
 * BC-Core, BC-mass, BC-Laplace), from 1D Gram matrices of nodal factors
 * (Prop. 2.2, eqs. Mass_Gal_fact, Lapl_Gal_fact; eq. nuc_pot with the
 * lattice-summed rank-R potential of eqs. EwaldTensorGl / EwaldSumP):
 *   S_k = S1[k1] o S2[k2] o S3[k3]
 *   H_k = 1/2 (K1 o S2 o S3 + S1 o K2 o S3 + S1 o S2 o K3) - sum_r M1_r o M2_r o M3_r
 * d_H_gen, d_S_gen: device, gen_elems elements each, layout per lattice
 *   [k1][k2][k3][mu][nu]; FP64 for LHF_PREC_FP64, FP32 for LHF_PREC_MIXED.
 * d_grams64: device, optional (NULL skips it), grams_elems FP64: the FP64 1D
 *   Grams per lattice and dimension, [term][slot][mu][nu] with term 0 = S
 *   (mass), 1 = K (stiffness, int g' g'), 2 + nu R + q = potential term with
 *   Z_nu w_q folded into dimension 1.  Needed by FP64 refinement and by the
 *   FP64 generator stack of a mixed pipeline (see d_H_gen64).
 * d_H_gen64, d_S_gen64: device, optional FP64 stacks written in mixed mode
 *   (the FP64 generator band used by refinement); must be NULL in FP64 mode.
 *   A mixed plan given the FP64 stacks may pass d_H_gen = d_S_gen = NULL:
 *   then only the FP64 stacks are written (lhf_block_fft_dual makes the
 *   complex64 blocks from them).
 * With all four stacks NULL only the factors and the FP64 Grams are computed
 * (into d_grams64, or the workspace when it is NULL), for
 * lhf_fourier_blocks.
 * Errors: LHF_ERR_INVALID (bad plan, one of a pair NULL), LHF_ERR_WORKSPACE. */
int32_t lhf_assemble_blocks(lhf_plan_t plan, void* d_H_gen, void* d_S_gen, double* d_grams64,
                            double* d_H_gen64, double* d_S_gen64,
                            void* d_ws, size_t ws_bytes, lhf_stream_t stream);

/* ---------------------------------------------------------------- block DFT
 * Fourier blocks Hbar_j = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) A_k,
 * w_l = exp(-2 pi i / L_l) (Lemma 3.1, Prop. 5.1), for every lattice of the
 * plan; only generator offsets inside the band are read (the others are
 * zero by construction).  prec selects the arithmetic: LHF_PREC_FP64 reads
 * FP64 stacks and writes complex128, LHF_PREC_MIXED reads FP32 stacks and
 * writes complex64 (interleaved re, im), layout per lattice
 * [j1][j2][j3][mu][nu].  All four buffers are required.
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE. */
int32_t lhf_block_fft(lhf_plan_t plan, int32_t prec, const void* d_H_gen, const void* d_S_gen,
                      void* d_H_bar, void* d_S_bar, void* d_ws, size_t ws_bytes,
                      lhf_stream_t stream);

/* lhf_block_fft restricted to the Hermitian half-space along k3: the
 * generators are real symmetric, so Hbar_(-j) = conj(Hbar_j) (Prop. 5.1) and
 * the blocks j3 > L3/2 carry no information beyond the kept ones (their
 * conjugates at (-j1, -j2, L3 - j3) mod L).  Same transform and arithmetic as
 * lhf_block_fft; only the blocks 0 <= j3 <= L3/2 are formed and written, in
 * the layout per lattice [j1][j2][j3 <= L3/2][mu][nu] at the lattice's
 * offset in a stack of half_elems elements (lhf_plan_sizes; a one-cell third
 * dimension keeps every block).  The fused and separable kernels run no
 * workgroup for j3 > L3/2.  d_H_half, d_S_half: device, half_elems complex
 * elements each (complex128 for LHF_PREC_FP64, complex64 for LHF_PREC_MIXED).
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE. */
int32_t lhf_block_fft_half(lhf_plan_t plan, int32_t prec, const void* d_H_gen, const void* d_S_gen,
                           void* d_H_half, void* d_S_half, void* d_ws, size_t ws_bytes, lhf_stream_t stream);

/* The FP64 block DFT of the mixed pipeline: reads the FP64 stacks, writes the
 * complex128 blocks (d_H_bar64, d_S_bar64, for refinement) and their
 * complex64 roundings (d_H_bar32, d_S_bar32, for the FP32 solve) in one pass.
 * Same transform and layouts as lhf_block_fft; all six buffers required.
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE. */
int32_t lhf_block_fft_dual(lhf_plan_t plan, const double* d_H_gen64, const double* d_S_gen64,
                           void* d_H_bar64, void* d_S_bar64, void* d_H_bar32, void* d_S_bar32,
                           void* d_ws, size_t ws_bytes, lhf_stream_t stream);

/* Separable formation of the Fourier blocks (Theorem 3.3, Remark 3.5): the
 * same Hbar_j, Sbar_j as lhf_block_fft of the FP64 stacks, without generator
 * stacks.  The generator is a sum of Hadamard products of 1D Grams, so its
 * transform over dimensions 2 and 3 is the same sum of products of the
 * 1D-transformed Grams G^_l[j_l] = sum_s w_l^(j_l k_s) G_l[s]:
 *   Sbar_j = S^1[j1] o S^2[j2] o S^3[j3],
 *   Hbar_j = 1/2 (K^1 o S^2 o S^3 + S^1 o K^2 o S^3 + S^1 o S^2 o K^3)
 *            - sum_r M^1_r o M^2_r o M^3_r,
 * with the band-pruned transform over dimension 1 done last; every block is
 * written once.  FP64 arithmetic on either plan precision.
 * d_grams64: the FP64 Grams written by lhf_assemble_blocks (any mode), or
 *   NULL for the copy in the workspace from the last assembly on it.
 * d_H_bar64, d_S_bar64: device complex128 [gen_elems], layout as
 *   lhf_block_fft.
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE, LHF_ERR_UNSUPPORTED (a lattice
 * whose first-dimension band is wider than 32 slots, or whose first axis
 * and band need more than 64 KiB of LDS per workgroup). */
int32_t lhf_fourier_blocks(lhf_plan_t plan, const double* d_grams64, void* d_H_bar64, void* d_S_bar64,
                           void* d_ws, size_t ws_bytes, lhf_stream_t stream);
/* lhf_fourier_blocks restricted to the Hermitian half-space along k3, in the
 * half layout of lhf_block_fft_half (d_H_half64, d_S_half64: device
 * complex128 [half_elems]); workgroups of the blocks j3 > L3/2 are not run.
 * Errors: as lhf_fourier_blocks. */
int32_t lhf_fourier_blocks_half(lhf_plan_t plan, const double* d_grams64, void* d_H_half64, void* d_S_half64,
                                void* d_ws, size_t ws_bytes, lhf_stream_t stream);

/* lhf_fourier_blocks for callers that cannot allocate device memory or pass
 * a workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same transform, kernels, layouts and results as
 * lhf_fourier_blocks; its one scratch buffer, the 1D-transformed Grams of
 * dimensions 2 and 3 (complex128, sum over lattices and those dimensions of
 * (2 + M0 R) L m0^2 elements), is a static device array of
 * LHF_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends.  The call allocates nothing, launches only
 * kernels (no memsets or copies), and uses the plan's device, which must be
 * current.  Every call on one device shares that device's array and leaves
 * its contents behind: calls that overlap on one device (several streams or
 * threads) race and must be serialised by the caller.
 * d_grams64: the FP64 Grams written by lhf_assemble_blocks (required here).
 * d_H_bar64, d_S_bar64: device complex128 [gen_elems], as lhf_fourier_blocks.
 * Errors: LHF_ERR_INVALID (NULL argument, another device current),
 * LHF_ERR_UNSUPPORTED (plan not separable, as lhf_fourier_blocks, or its
 * transformed Grams larger than the static array), LHF_ERR_HIP. */
#define LHF_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
int32_t lhf_fourier_blocks_noalloc(lhf_plan_t plan, const double* d_grams64, void* d_H_bar64, void* d_S_bar64,
                                   lhf_stream_t stream);

/* ---------------------------------------------------------------- eigensolve
 * For every block j: Hbar_j u = lambda Sbar_j u (eq. HF-FSpace-Block), by
 * Cholesky reduction to a standard Hermitian problem, then, for FP64
 * eigenvalues without vectors, Householder reduction to tridiagonal form and
 * bisection on Sturm counts (eigenvalues to a few ulps of the block's norm),
 * otherwise cyclic parallel-order complex Jacobi sweeps; the union over j is
 * the spectrum of the full matrix pair (eq. lambdAbc).
 * Conjugate blocks j and -j share their spectrum; each pair is solved once.
 * d_H_bar, d_S_bar: device, complex128 (FP64 plan) or complex64 (mixed plan);
 *   mixed plans with LHF_HEEV_REFINE_FP64 may pass both NULL together with
 *   d_H_bar64 and d_S_bar64: the FP32 solve then reads the complex128 blocks
 *   and rounds them itself (no complex64 copy is needed).
 * flags: LHF_HEEV_VECTORS, LHF_HEEV_REFINE_FP64 (mixed plans: after the FP32
 *   solve, form U^H Hbar U and U^H Sbar U in FP64 with FP64-accurate blocks
 *   and re-solve them in FP64), LHF_HEEV_FP32_SOLVE (mixed plans: no class
 *   takes the FP64 solve alone).
 * d_H_bar64, d_S_bar64: device complex128 Fourier blocks used by refinement;
 *   may be NULL, then refinement regenerates each block from the FP64
 *   generator stacks d_H_gen64 / d_S_gen64 (band offsets only), which then
 *   must be given.  All four are ignored without LHF_HEEV_REFINE_FP64.
 * d_w: device FP64 [w_elems], ascending per block.
 * d_V: device, optional, complex (plan precision; complex128 after
 *   refinement) [nblocks][m0][m0], column c = eigenvector c, S-orthonormal.
 * d_info: device int32 [nblocks]: 0 ok; k > 0 Sbar not positive definite at
 *   column k; -1 Jacobi did not converge; -2 non-finite input (the
 *   bisection always ends within its bound and reports 0).
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE. */
int32_t lhf_heev_batched(lhf_plan_t plan, uint32_t flags, const void* d_H_bar, const void* d_S_bar,
                         const void* d_H_bar64, const void* d_S_bar64,
                         const double* d_H_gen64, const double* d_S_gen64,
                         double* d_w, void* d_V, int32_t* d_info,
                         void* d_ws, size_t ws_bytes, lhf_stream_t stream);

/* ---------------------------------------------------------------- eigenvectors
 * Eigenvectors of the full lattice problem H u = lambda S u from the
 * Fourier-block eigenvectors (Prop. 5.1, eq. eigvecA): U = (F^* x I_m0)
 * bdiag(Ubar_j), F = F_L1 x F_L2 x F_L3 unitary, (F_L)_(j,k) = w^(j k) /
 * sqrt(L), w = exp(-2 pi i / L).  Selection s = (j, c) -- Fourier block j =
 * (j1 L2 + j2) L3 + j3 of lattice `lattice`, eigenvector column c -- gives the
 * vector whose block on cell k = (k1 L2 + k2) L3 + k3 is
 *   U[s][k][mu] = L^(-1/2) exp(+2 pi i (j1 k1/L1 + j2 k2/L2 + j3 k3/L3)) Ubar_j(mu, c),
 * with eigenvalue lambda_(j, c); Sbar_j-orthonormal columns of Ubar_j give
 * S-orthonormal vectors.  The conjugate block -j gives the complex conjugate
 * vector (the same eigenvalue); Re and Im of the pair span the real
 * eigenvectors of the real symmetric H.
 * d_V: device complex128 [gen_elems], the eigenvectors lhf_heev_batched wrote
 *   with LHF_HEEV_VECTORS (FP64 plans, or mixed plans with
 *   LHF_HEEV_REFINE_FP64), column c of block j = eigenvector c (ascending).
 * d_sel: device int32 [nsel][2] (j, c); a selection out of range gives a
 *   vector of NaN (checked in the kernel, no out-of-range access).
 * d_U: device complex128 [nsel][L1 L2 L3][m0], cell-major.
 * nsel = 0 launches nothing.
 * Errors: LHF_ERR_INVALID (NULL plan or pointer, lattice out of range,
 * nsel < 0), LHF_ERR_UNSUPPORTED (more than 2^31 - 1 workgroups of 256
 * outputs), LHF_ERR_HIP. */
int32_t lhf_eigvecs_lattice(lhf_plan_t plan, int32_t lattice, const void* d_V, int32_t nsel, const int32_t* d_sel,
                            void* d_U, lhf_stream_t stream);

/* ---------------------------------------------------------------- Dirichlet chain
 * A box chain of L cells along dimension 1 (all dimensions Dirichlet, L2 = L3
 * = 1) with defect cells, as a perturbed block-Toeplitz pair (Sec. 3, the
 * box-case discussion of defects; Remark 3.2 for the circulant embedding):
 *   * T: block-Toeplitz from the pristine cell, A_s = <g_(0,mu), H_rep g_(s,nu)>,
 *     s = 0..L0, on the chain grid without walls; H_rep carries the central
 *     cell's lattice-window potential (window of L cells) replicated to every
 *     cell; T(k, m) = A_(m-k), A_(-s) = A_s^T, zero beyond the band L0;
 *   * crosses: every block (k, m), |k - m| <= L0, with k or m in X = defect
 *     cells and cells within L0 of a wall, is the block of the actual basis
 *     (defect exponents scaled) on the box grid with its walls and potential
 *     H_rep's plus, for each defect cell c in {k, m}, (Z_def - Z_nu) times the
 *     rank-R potential of nucleus nu of cell c;
 *   * L0 from the smallest exponent over pristine and defect cells (overlap
 *     decay below 1e-22), capped at L - 1.
 * The chain's nodes must be cell aligned: n1 = nc L and pad1 = a / (2 nc).
 * The same model is built by the CPU oracle. */
typedef struct {
  lhf_lattice lat;          /* bc = LHF_BC_DIRICHLET, L = {L, 1, 1}; lat.L0 ignored   */
  int32_t ndef;             /* defect cells, >= 0                                       */
  const int32_t* def_cells; /* [ndef] distinct cell indices in [0, L)                   */
  const double* def_Z;      /* [ndef] charge of every nucleus of the defect cell, > 0   */
  const double* def_scale;  /* [ndef] factor on every exponent of the defect cell, > 0  */
} lhf_box;

typedef struct {
  int32_t L, m0, L0;        /* cells, functions per cell, band half-width             */
  int32_t N;                /* m0 L                                                   */
  int32_t P;                /* circulant embedding length (power of two >= L + L0)    */
  int32_t ncross;           /* cells in X                                             */
  int32_t ncross_blocks;    /* cross blocks (k, m) with k <= m                         */
  double sigma;             /* shift of the circulant preconditioner                  */
} lhf_toeplitz_info;

/* Validate, derive the model and assemble it on the current device
 * (synchronous; allocates the operator's device tables: generators, cross
 * blocks, the embedding's per-frequency blocks and the preconditioner).
 * Errors: LHF_ERR_INVALID (descriptor), LHF_ERR_UNSUPPORTED (not a cell-aligned
 * Dirichlet chain, m0 > 32, ...), LHF_ERR_ALLOC, LHF_ERR_HIP. */
int32_t lhf_toeplitz_create(const lhf_box* box, lhf_toeplitz_t* out);
/* The exact box operator of the same chain (Sec. 2.3, case (B)): the
 * potential is the finite lattice's own, eq. EwaldSumE in the factor form of
 * eq. EwaldTensorGl -- along the chain, sum over every cell c = 0..L-1 of
 * Z_(nu, c) times the rank-R potential of nucleus nu of cell c, Z_(nu, c) =
 * def_Z on defect cells, Z_nu elsewhere; no window, no replication -- and
 * every block (k, m), |k - m| <= L0, is the block of the actual basis
 * (defect exponents scaled) on the box grid with its walls.  It keeps the
 * asymmetry of the finite lattice sum and the wall layer that the
 * block-Toeplitz model of lhf_toeplitz_create replaces by the central cell.
 * Returns a handle of the same kind: lhf_toeplitz_matvec applies the
 * block-sparse operator (every block row in FP64, either precision),
 * lhf_toeplitz_eigs runs block LOBPCG on it with the same circulant
 * preconditioner (the embedding of the pristine generators),
 * lhf_toeplitz_get_info reports ncross = L and ncross_blocks = every band
 * block (k <= m), and lhf_toeplitz_blocks returns those blocks as the cross
 * blocks.  Errors: as lhf_toeplitz_create. */
int32_t lhf_box_exact_create(const lhf_box* box, lhf_toeplitz_t* out);
/* The three-level block-Toeplitz operator of an L1 x L2 x L3 lattice in a box
 * (Sec. 2.3, item (A): the central cell's potential replicated to every cell
 * makes the box matrix shift invariant; Def. 5.4: a symmetric three-level
 * block-Toeplitz matrix), applied through its three-level block-circulant
 * embedding (Remark 3.2: about double size at each level):
 *   T(k, m) = A_(m-k),  A_s(mu, nu) = <g_(0,mu), H_rep g_(s,nu)>,
 * s signed in every dimension with |s_l| <= L0_l, zero beyond.  Readings:
 *   * every dimension is a box dimension; a dimension with L >= 2 needs
 *     cell-aligned nodes (n = nc L, pad = a / (2 nc)) and its generators are
 *     taken on its node set extended without walls; a one-cell dimension is
 *     an ordinary box dimension with its walls;
 *   * H_rep carries, per multi-cell dimension, the lattice-window factors of
 *     the central cell (window of L cells: odd L symmetric, even L with half
 *     weights on the two end cells) repeated with period a; per one-cell
 *     dimension the nucleus's own factor;
 *   * L0_l from the smallest exponent (overlap decay below 1e-22), capped at
 *     L_l - 1; embedding lengths P_l: smallest powers of two >= L_l + L0_l.
 * The walls of multi-cell dimensions and defects are not modelled (the wall
 * layer, item (B), is what the exact chain operator keeps).  The embedding's
 * per-frequency blocks are Hadamard combinations of 1D-transformed Grams
 * (Theorem 3.3 applied to the embedding), built without a 3D generator
 * array.  Returns a handle of the same kind: lhf_toeplitz_matvec (x and y
 * cell-major, cell (k1 L2 + k2) L3 + k3, complex128 or complex64 transform),
 * lhf_toeplitz_eigs (preconditioner (C_H - sigma C_S)^-1 per frequency of the
 * embedding), lhf_toeplitz_get_info (L = L1 L2 L3 cells, L0 = the largest
 * L0_l, P = P1 P2 P3, ncross = ncross_blocks = 0); lhf_toeplitz_blocks is
 * refused (LHF_ERR_UNSUPPORTED): use lhf_toeplitz3_generators.
 * Synchronous; allocates the operator's device tables.
 * Errors: LHF_ERR_INVALID (descriptor), LHF_ERR_UNSUPPORTED (not Dirichlet,
 * nodes not cell aligned, m0 > 32, an embedding level longer than 4096 or
 * more than 2^22 frequencies, ...), LHF_ERR_ALLOC, LHF_ERR_HIP. */
int32_t lhf_toeplitz3_create(const lhf_lattice* lat, lhf_toeplitz_t* out);
/* The generators A_s of a three-level operator: d_gen_H, d_gen_S device FP64
 * [2 L0_1 + 1][2 L0_2 + 1][2 L0_3 + 1][m0][m0], index s_l + L0_l, row mu,
 * column nu.  Synchronous.  Errors: LHF_ERR_INVALID (NULL pointer, not a
 * three-level operator), LHF_ERR_HIP. */
int32_t lhf_toeplitz3_generators(lhf_toeplitz_t tp, double* d_gen_H, double* d_gen_S);
int32_t lhf_toeplitz_get_info(lhf_toeplitz_t tp, lhf_toeplitz_info* out);
/* Copy the model's blocks to device buffers (each may be NULL):
 * d_gen_H, d_gen_S: FP64 [L0 + 1][m0][m0], A_s row mu, column nu;
 * d_cross_km: int32 [ncross_blocks][2] (k, m), k <= m, ascending;
 * d_cross_H, d_cross_S: FP64 [ncross_blocks][m0][m0], the model's block (k, m).
 * Synchronous.  Errors: LHF_ERR_INVALID. */
int32_t lhf_toeplitz_blocks(lhf_toeplitz_t tp, double* d_gen_H, double* d_gen_S, int32_t* d_cross_km,
                            double* d_cross_H, double* d_cross_S);
/* Workspace bytes of lhf_toeplitz_matvec for up to ncols vectors. */
size_t lhf_toeplitz_matvec_workspace(lhf_toeplitz_t tp, int32_t ncols);
/* y_H = H_model x, y_S = S_model x for ncols vectors: T x through the block
 * circulant embedding (forward FFT over the cell index, one m0 x m0 product
 * per frequency, inverse FFT, first L blocks) plus the cross corrections.
 * x, y_H, y_S: device FP64, row-major [N][ld] (ld >= ncols; column j is
 * vector j; row k m0 + mu is function mu of cell k).  prec: LHF_PREC_FP64
 * (complex128 transform) or LHF_PREC_MIXED (the Toeplitz part with FP32
 * inputs and complex64 transform; the crosses in FP64).  y_S may be NULL.
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE. */
int32_t lhf_toeplitz_matvec(lhf_toeplitz_t tp, int32_t prec, int32_t ncols, const double* x, double* y_H,
                            double* y_S, int32_t ld, void* d_ws, size_t ws_bytes, lhf_stream_t stream);
/* lhf_toeplitz_matvec of the FP32 route with FP32 input and output: the
 * Toeplitz part through the complex64 circulant embedding (Remark 3.2) and the
 * cross corrections accumulated in FP64 registers, x, y_H, y_S device FP32
 * [N][ld] (half the vector bytes of the FP64-interface call); the same
 * workspace as lhf_toeplitz_matvec.  y_S may be NULL.
 * Errors: LHF_ERR_INVALID, LHF_ERR_WORKSPACE, LHF_ERR_UNSUPPORTED (a
 * three-level operator: FP64 input only). */
int32_t lhf_toeplitz_matvec_f32(lhf_toeplitz_t tp, int32_t ncols, const float* x, float* y_H, float* y_S,
                                int32_t ld, void* d_ws, size_t ws_bytes, lhf_stream_t stream);
/* Workspace bytes of lhf_toeplitz_eigs for nev wanted eigenpairs. */
size_t lhf_toeplitz_eigs_workspace(lhf_toeplitz_t tp, int32_t nev);
/* The nev lowest eigenpairs of (H_model, S_model) by block LOBPCG (Knyazev)
 * with nev + 4 vectors: basis [X, W, P], W the residuals through the circulant
 * preconditioner (H_c - sigma S_c)^-1 per frequency (H_c, S_c the embedding's
 * blocks; sigma below their spectrum), images recomputed by matvecs every
 * iteration, S-orthonormalised in FP64 (Cholesky-QR in the column order
 * [X, W, P], dropping columns whose squared distance from the span of the
 * ones before them is below 1e-10), FP64 Rayleigh-Ritz; matvecs in
 * FP32 until the largest residual of the wanted pairs is below 1e-4 or stops
 * falling (no 30% drop over five iterations), then in FP64 until it is below
 * tol.  The start block is drawn from a counter-based
 * generator (SplitMix64) with `seed`.  Runs on `stream` and synchronises it
 * once per iteration (convergence test on the host).
 * d_w: device FP64 [nev] ascending; d_V: device FP64 [N][nev] or NULL
 * (S-orthonormal eigenvectors); *iters (host, may be NULL): iterations used.
 * Returns LHF_OK also when maxit is reached (then *iters == maxit and the
 * residual test failed; *resid (host, may be NULL) gets the largest residual).
 * Errors: LHF_ERR_INVALID (nev < 1, nev + 4 > N, 3 (nev + 4) > 112),
 * LHF_ERR_WORKSPACE, LHF_ERR_HIP. */
int32_t lhf_toeplitz_eigs(lhf_toeplitz_t tp, int32_t nev, int32_t maxit, double tol, uint64_t seed,
                          double* d_w, double* d_V, int32_t* iters, double* resid, void* d_ws,
                          size_t ws_bytes, lhf_stream_t stream);
int32_t lhf_toeplitz_destroy(lhf_toeplitz_t tp);
/* The k lowest eigenpairs of a dense real symmetric m x m matrix, the
 * Rayleigh-Ritz problem of the block LOBPCG of lhf_toeplitz_eigs: Householder
 * tridiagonalisation, bisection on Sturm counts for the k lowest eigenvalues,
 * inverse iteration on the tridiagonal matrix (vectors of eigenvalues closer
 * than 1e-8 of the matrix norm orthogonalised against each other; others
 * orthogonal to about 1e-16 norm / gap), and the back-transform, in one
 * workgroup.  d_A: device FP64 row-major, lda >= m, read as (A + A^T) / 2;
 * d_w: device FP64 [k] ascending; d_V: device FP64 row-major m x k with
 * ldv >= k (column i the unit eigenvector of w[i]); d_A may not overlap d_w
 * or d_V.  Every intermediate (the reflectors included) stays in the
 * workgroup's LDS: no workspace.  Asynchronous on `stream`; allocates nothing.
 * Errors: LHF_ERR_INVALID (1 <= k <= m <= 112, lda, ldv, NULL pointers),
 * LHF_ERR_HIP. */
int32_t lhf_dense_syev(int32_t m, int32_t k, const double* d_A, int32_t lda, double* d_w, double* d_V, int32_t ldv,
                       lhf_stream_t stream);

/* ---------------------------------------------------------------- whole step
 * The buffers of one step of the plan: assembly, block DFT and eigensolve.
 * Same meaning, layout and precision as in the calls above.  Required:
 * H_gen, S_gen, H_bar, S_bar, w, info, ws.  Mixed plans with
 * LHF_HEEV_REFINE_FP64 also need H_gen64 and S_gen64 (written by the
 * assembly); when H_bar64 and S_bar64 are given as well, the step fills them
 * with a complex128 block DFT and refinement reads them, otherwise
 * refinement regenerates each block from the FP64 band.  With H_bar64 given,
 * H_gen and S_gen may be NULL: the step then skips the FP32 stacks and makes
 * H_bar and S_bar with lhf_block_fft_dual; if H_bar and S_bar are NULL too,
 * the step runs the FP64 block DFT only and the FP32 solve reads H_bar64 and
 * S_bar64.  grams64 may be
 * NULL (the workspace holds the Grams), V is needed with LHF_HEEV_VECTORS. */
typedef struct {
  void* H_gen;
  void* S_gen;
  double* grams64;
  double* H_gen64;
  double* S_gen64;
  void* H_bar;
  void* S_bar;
  void* H_bar64;
  void* S_bar64;
  double* w;
  void* V;
  int32_t* info;
  void* ws;
  size_t ws_bytes;
  uint32_t heev_flags;   /* LHF_HEEV_* */
} lhf_step_args;

/* Enqueue one whole step (the calls above in order) on `stream`.
 * Errors: those of the calls above; nothing is enqueued after the first. */
int32_t lhf_step(lhf_plan_t plan, const lhf_step_args* args, lhf_stream_t stream);

/* A step captured once into a HIP graph (every launch of the plan, grouped
 * over its lattices; no memset nodes) and replayed with one call.  The
 * buffers named in `args` are baked into the graph: they must stay allocated
 * while it exists, and a replay overwrites them as lhf_step would.
 * lhf_graph_create allocates (graph and executable graph; capture runs on a
 * private stream of default priority) and launches nothing; replays of one
 * graph on several streams at once race on its buffers.  The plan's launch
 * shapes and work tables are baked in too: the plan must outlive its graphs,
 * and a change of its tuning (lhf_plan_set_tuning, lhf_plan_autotune) makes
 * every graph captured before it stale: lhf_graph_launch then returns
 * LHF_ERR_INVALID without launching, and the step must be captured again.
 * Errors: those of lhf_step, LHF_ERR_HIP (capture or instantiation failed). */
typedef struct lhf_graph_s* lhf_graph_t;
int32_t lhf_graph_create(lhf_plan_t plan, const lhf_step_args* args, lhf_graph_t* out);
int32_t lhf_graph_launch(lhf_graph_t graph, lhf_stream_t stream);
int32_t lhf_graph_destroy(lhf_graph_t graph);

/* ---------------------------------------------------------------- autotuner
 * Launch shapes and sweep schedule of a plan:
 *   dft_threads  threads one grouped block-DFT pass aims to run (sets the
 *                outputs per thread along the transformed axis);
 *   gram_split   split-K target of the Gram contraction, workgroups per
 *                (lattice, dimension), <= 256;
 *   gram_grid    workgroups of the persistent grouped Gram launch;
 *   tol32_scale  mixed plans: multiplier of the FP32 Jacobi stopping
 *                tolerance (the FP64 refinement converges to the same
 *                tolerance whatever the FP32 schedule);
 *   heev_wide    bit c (size class M = 4 << c): the eigensolver runs one
 *                matrix entry per thread instead of four (for batches too
 *                small to fill the device); 0..15, the planner sets the
 *                classes whose four-entry launch has fewer wavefronts than
 *                the device has SIMDs;
 *   fourier_sep  1: whole steps (lhf_step, graphs) form the complex128
 *                Fourier blocks separably from the FP64 Grams
 *                (lhf_fourier_blocks) instead of generator stacks and a block
 *                DFT, on FP64 plans and on mixed plans whose FP32 solve reads
 *                the complex128 blocks; the generator stacks are then not
 *                written.  Reads 0 when the plan does not qualify;
 *   heev_fp64    mixed plans, bit c (size class M = 4 << c): a refined solve
 *                that is given the complex128 blocks solves that class by the
 *                FP64 solver of FP64 plans alone, with no FP32 solve and no
 *                refinement (tridiagonal reduction and bisection without
 *                vectors, Jacobi with them: where rotation latency, not
 *                arithmetic, sets the FP32 solve's time, or where bisection
 *                beats Jacobi); 0..15, default 0, reads 0 on FP64 plans.
 *                The eigenvalues of such a class meet the FP64 tolerance,
 *                which is tighter than the refined one;
 *   gram_tile    output tile of one Gram work item, 64 (default) or 32 (for
 *                launches with fewer items than the device has CUs: four
 *                times the items).
 * Apart from heev_fp64, none of them changes what is computed; the Gram split
 * changes the order of the FP64 partial sums and the eigensolver layout the
 * order of its sums. */
typedef struct {
  int32_t dft_threads;
  int32_t gram_split;
  int32_t gram_grid;
  int32_t tol32_scale;
  int32_t heev_wide;
  int32_t fourier_sep;
  int32_t heev_fp64;
  int32_t gram_tile;
  double step_ms;        /* autotune: mean time of one step with these settings */
  int32_t from_cache;    /* autotune: 1 when read from the cache file         */
} lhf_tuning;

int32_t lhf_plan_get_tuning(lhf_plan_t plan, lhf_tuning* out);
/* Apply settings (fields outside their range -> LHF_ERR_INVALID).  Rebuilds
 * and uploads the plan's work tables synchronously: no work of the plan may
 * be pending. */
int32_t lhf_plan_set_tuning(lhf_plan_t plan, const lhf_tuning* in);
/* Time candidate settings stage by stage on `stream` with HIP events (runs
 * steps with `args`, overwriting its buffers), keep the fastest, and report
 * them in *out (may be NULL).  cache_path (may be NULL): a JSON file keyed by
 * the plan's work signature and the device (architecture, compute units);
 * a hit applies the stored settings without timing, a miss appends the
 * result.  Synchronous; no other work of the plan may be pending.
 * Errors: those of lhf_step, LHF_ERR_HIP. */
int32_t lhf_plan_autotune(lhf_plan_t plan, const lhf_step_args* args, lhf_stream_t stream,
                          const char* cache_path, lhf_tuning* out);

/* ---------------------------------------------------------------- status */
const char* lhf_status_string(int32_t status);
const char* lhf_last_error(void);
int32_t lhf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LHF_H */
