// Batched generalized Hermitian eigensolver for the Fourier blocks
// (eq. HF-FSpace-Block; union of block spectra, Prop. 5.1 eq. lambdAbc).
//
// Per block j (one matrix = (M/2)^2 threads, matrices in LDS):
//   1. Gaussian elimination on Sbar (no pivoting; it is Hermitian positive
//      definite) carrying W = L^-1 along, Sbar = L D L^H, one barrier per
//      column; the Cholesky factor is C = L D^1/2, so C^-1 = D^-1/2 W;
//   2. reduction A = C^-1 Hbar C^-H by two register-tiled products;
//   3. cyclic Jacobi sweeps in the parallel round-robin ordering: in each of
//      the M-1 rounds of a sweep the M/2 index pairs (p, q) are disjoint and a
//      thread owns the 2 x 2 block {p_i, q_i} x {p_j, q_j} of pairs (i, j):
//      it rotates that block in registers, A <- J_i^H A J_j with
//      J = [[c, s b/|b|], [-s conj(b)/|b|, c]] (b = A_pq; c, s from the stable
//      tangent formula), and the columns {p_j, q_j} of rows {p_i, q_i} of V;
//      sweeps stop when the off-diagonal Frobenius norm is below 4 M eps of
//      the norm of A (eigenvalues only: or earlier, when a second-order
//      closure is within that bound);
//   4. eigenvalues sorted ascending, eigenvectors C^-H V = W^H D^-1/2 V.
// Blocks j and -j are complex conjugates (real symmetric generators): only
// the canonical block of each pair is solved and its results are written for
// both.  The plan lists the canonical (lattice, block) pairs of every lattice
// per size class, so one launch per class serves the whole plan.
//
// Refinement (mixed precision): the FP32 solve leaves eigenvectors U; in FP64
// the block pair is rebuilt accurately (from complex128 Fourier blocks, or
// regenerated from the FP64 generator band) and the Rayleigh-Ritz pair
// (U^H Hbar U, U^H Sbar U) -- nearly diagonal -- is reduced with the series
// (I + E)^-1/2 of the overlap and goes through the FP64 sweeps, which stop
// after one sweep or none.  If the FP32 solve failed for a
// block, U = I and the FP64 solve does the whole work.
//
// Sizes: M in {4, 8, 16, 32} >= m0; padded rows/columns are decoupled (unit
// overlap, zero Hamiltonian) and never written out.  Workgroups hold 64/(M/2)^2
// matrices for M <= 16 (one wavefront) and one matrix for M = 32.
#include <algorithm>
#include <type_traits>

#include "plan.h"
#include "sturm.h"
#include "dpp.h"

namespace lhf {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { typedef double2 T; };
template <> struct Cx<float> { typedef float2 T; };

template <typename C> __device__ __forceinline__ C cmk(decltype(C{}.x) a, decltype(C{}.x) b) { C r; r.x = a; r.y = b; return r; }
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) { return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) { return cmk<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C, typename R> __device__ __forceinline__ C cscale(C a, R s) { return cmk<C>(a.x * s, a.y * s); }

// Reciprocal and reciprocal square root: FP32 through the hardware
// approximations (v_rcp_f32, v_rsq_f32, within about one ulp), FP64 correctly
// rounded.
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsq_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_(double x) { return 1.0 / sqrt(x); }
// 1 / x for a normal x to within a few ulps: the hardware estimate, refined
// by two Newton steps in FP64.
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_fast(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// Round-robin schedule: pair i of round s (0 <= s < M-1).
template <int M>
__device__ __forceinline__ void pair_of(int i, int s, int& p, int& q) {
  constexpr int m = M - 1;
  if (i == 0) { p = 0; q = 1 + s; }
  else { p = 1 + (s + i) % m; q = 1 + (s - i + m) % m; }
}

__device__ __forceinline__ int conj_block(const LatDev& L, int b) {
  const int k3 = b % L.L[2];
  const int k2 = (b / L.L[2]) % L.L[1];
  const int k1 = b / (L.L[2] * L.L[1]);
  const int c1 = k1 ? L.L[0] - k1 : 0, c2 = k2 ? L.L[1] - k2 : 0, c3 = k3 ? L.L[2] - k3 : 0;
  return (c1 * L.L[1] + c2) * L.L[2] + c3;
}

template <typename R, int M, int G, bool HASU, bool HASV, bool NOF = false>
struct Smem {
  typedef typename Cx<R>::T C;
  // F (the reduction's W, the refinement's series) is absent in the
  // refinement without vectors for M >= 16, which keeps those in the dead U
  // instead (more resident matrices; at M <= 8 the fourth matrix costs less
  // than the extra passes), and in the FP64 eigenvalue solve at M = 8, 32
  // (NOF), which keeps W in the upper triangle of B
  static constexpr bool HASF = !NOF && (HASV || !HASU || M <= 8);
  C A[G][M][M + 1];
  C B[G][M][M + 1];
  C F[HASF ? G : 1][HASF ? M : 1][M + 1];
  C V[HASV ? G : 1][HASV ? M : 1][M + 1];
  C U[HASU ? G : 1][HASU ? M : 1][M + 1];
  R red[G][16];                  // cross-wave partial sums
  R lam[G][M];
  R jc[G][M / 2];                // rotation cosine per pair
  C js[G][M / 2];                // s b / |b| per pair
  R dn[G][M];                    // rotated diagonal
  R dsc[G][M];                   // D^-1/2 of the overlap's L D L^H
  int rank[G][M];
  int flag[G][4];                // 0: Cholesky failure column, 1: non-finite, 2: converged
};

// Sum over the TPM = M^2 / W threads of one matrix (W entries per thread);
// all threads of the workgroup call it.
template <int W, typename R, int M, int G, bool HASU, bool HASV>
__device__ __forceinline__ R group_sum(Smem<R, M, G, HASU, HASV>& sh, int g, int t, R v) {
  constexpr int TPM = M * M / W;
  if constexpr (TPM <= 64) {
#pragma unroll
    for (int o = TPM / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
  } else {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((t & 63) == 0) sh.red[g][t >> 6] = v;
    __syncthreads();
    R s = R(0);
#pragma unroll
    for (int w = 0; w < TPM / 64; ++w) s += sh.red[g][w];
    __syncthreads();
    return s;
  }
}

// Entries owned by thread t of a matrix in the elementwise phases:
// t + k TPM, k < W (W = 4 entries per thread, or 1 in the wide layout).
#define LHF_FOR_ENTRIES                                   \
  _Pragma("unroll") for (int k = 0; k < W; ++k)           \
    if (const int e = t + k * TPM, r = e / M, c = e % M; true)

// Register-tiled products: thread t of a matrix owns the NT x NT tile of
// rows {ti + a S} and columns {tj + b S}, S = M / NT, ti = t / S, tj = t % S
// (NT = 2 with four entries per thread, where every operand entry loaded
// from LDS feeds two products, four when two products share an operand;
// NT = 1 in the wide layout).
template <int M> struct Tile {
  static constexpr int UR = M <= 8 ? M : 4;   // q-loop unroll
};
template <int W> struct TileOf {
  static constexpr int NT = W == 4 ? 2 : 1;
};
template <int M, int NT>
__device__ __forceinline__ void tile_coords(int t, int& ti, int& tj) {
  ti = t / (M / NT);
  tj = t % (M / NT);
}

// P1 = X1 Y, P2 = X2 Y
template <int M, int NT, typename C>
__device__ __forceinline__ void mm_shared_right(const C (&X1)[M][M + 1], const C (&X2)[M][M + 1],
                                                const C (&Y)[M][M + 1], int ti, int tj, C (&p1)[NT][NT],
                                                C (&p2)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) { p1[a][b] = cmk<C>(0, 0); p2[a][b] = cmk<C>(0, 0); }
#pragma unroll Tile<M>::UR
  for (int q = 0; q < M; ++q) {
    C y[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) y[b] = Y[q][tj + b * S];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const C x1 = X1[ti + a * S][q], x2 = X2[ti + a * S][q];
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        p1[a][b] = cadd(p1[a][b], cmul(x1, y[b]));
        p2[a][b] = cadd(p2[a][b], cmul(x2, y[b]));
      }
    }
  }
}

// P1 = X^H Y1, P2 = X^H Y2
template <int M, int NT, typename C>
__device__ __forceinline__ void mm_shared_left_h(const C (&X)[M][M + 1], const C (&Y1)[M][M + 1],
                                                 const C (&Y2)[M][M + 1], int ti, int tj, C (&p1)[NT][NT],
                                                 C (&p2)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) { p1[a][b] = cmk<C>(0, 0); p2[a][b] = cmk<C>(0, 0); }
#pragma unroll Tile<M>::UR
  for (int q = 0; q < M; ++q) {
    C x[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) x[a] = X[q][ti + a * S];
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const C y1 = Y1[q][tj + b * S], y2 = Y2[q][tj + b * S];
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        p1[a][b] = cadd(p1[a][b], cmulc(x[a], y1));
        p2[a][b] = cadd(p2[a][b], cmulc(x[a], y2));
      }
    }
  }
}

// P = X Y (+ d I when ADDI)
template <int M, int NT, bool ADDI, typename C, typename R>
__device__ __forceinline__ void mm_tile(const C (&X)[M][M + 1], const C (&Y)[M][M + 1], int ti, int tj, R d,
                                        C (&p)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) p[a][b] = cmk<C>(0, 0);
#pragma unroll Tile<M>::UR
  for (int q = 0; q < M; ++q) {
    C y[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) y[b] = Y[q][tj + b * S];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const C x = X[ti + a * S][q];
#pragma unroll
      for (int b = 0; b < NT; ++b) p[a][b] = cadd(p[a][b], cmul(x, y[b]));
    }
  }
  if constexpr (ADDI) {
    if (ti == tj) {
#pragma unroll
      for (int a = 0; a < NT; ++a) p[a][a].x += d;
    }
  }
}

template <int M, int NT, typename C>
__device__ __forceinline__ void store_tile(C (&Z)[M][M + 1], int ti, int tj, const C (&p)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) Z[ti + a * S][tj + b * S] = p[a][b];
}

// P = X Y^H
template <int M, int NT, typename C>
__device__ __forceinline__ void mm_tile_rh(const C (&X)[M][M + 1], const C (&Y)[M][M + 1], int ti, int tj,
                                           C (&p)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) p[a][b] = cmk<C>(0, 0);
#pragma unroll Tile<M>::UR
  for (int q = 0; q < M; ++q) {
    C y[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) y[b] = Y[tj + b * S][q];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const C x = X[ti + a * S][q];
#pragma unroll
      for (int b = 0; b < NT; ++b)
        p[a][b] = cadd(p[a][b], cmk<C>(x.x * y[b].x + x.y * y[b].y, x.y * y[b].x - x.x * y[b].y));
    }
  }
}

// P = X^H diag(d) Y
template <int M, int NT, typename C, typename R>
__device__ __forceinline__ void mm_tile_lh_diag(const C (&X)[M][M + 1], const R (&d)[M], const C (&Y)[M][M + 1],
                                                int ti, int tj, C (&p)[NT][NT]) {
  constexpr int S = M / NT;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) p[a][b] = cmk<C>(0, 0);
#pragma unroll Tile<M>::UR
  for (int q = 0; q < M; ++q) {
    const R dq = d[q];
    C y[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) y[b] = cscale(Y[q][tj + b * S], dq);
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const C x = X[q][ti + a * S];
#pragma unroll
      for (int b = 0; b < NT; ++b) p[a][b] = cadd(p[a][b], cmulc(x, y[b]));
    }
  }
}

// Complex M x M products on the FP64 matrix cores (v_mfma_f64_16x16x4f64)
// for one matrix per workgroup (M >= 16): wavefront w < (M/16)^2 owns the
// 16 x 16 output tile (w / (M/16), w % (M/16)), the others idle.  In each
// 4-wide k step lane (lr, lk) = (lane % 16, lane / 16) supplies A[row lr][k lk]
// and B[k lk][col lr]; it holds output rows lk + 4 v of column lr.  The real
// and imaginary parts take four real products per step.
typedef double mf4 __attribute__((ext_vector_type(4)));

template <int M>
struct MfTile {
  static constexpr int NTL = M / 16;
  int r0 = 0, c0 = 0, lr = 0, lk = 0;
  bool on = false;
  __device__ __forceinline__ MfTile() {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    on = wave < NTL * NTL;
    r0 = on ? 16 * (wave / NTL) : 0;
    c0 = on ? 16 * (wave % NTL) : 0;
    lr = lane & 15;
    lk = lane >> 4;
  }
};

// (re, im) = op(X) Y with op(X) = X, or X^H when XH
template <int M, bool XH>
__device__ __forceinline__ void mf_product(const MfTile<M>& f, const double2 (&X)[M][M + 1],
                                           const double2 (&Y)[M][M + 1], mf4& re, mf4& im) {
  re = mf4{0.0, 0.0, 0.0, 0.0};
  im = mf4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < M; k0 += 4) {
    const double2 x = XH ? X[k0 + f.lk][f.r0 + f.lr] : X[f.r0 + f.lr][k0 + f.lk];
    const double xi = XH ? -x.y : x.y;
    const double2 y = Y[k0 + f.lk][f.c0 + f.lr];
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-xi, y.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(xi, y.x, im, 0, 0, 0);
  }
}

// the tile into Z, plus d on the diagonal
template <int M>
__device__ __forceinline__ void mf_store(const MfTile<M>& f, double2 (&Z)[M][M + 1], const mf4& re, const mf4& im,
                                         double d) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = f.r0 + f.lk + 4 * v, c = f.c0 + f.lr;
    Z[r][c] = make_double2(re[v] + (r == c ? d : 0.0), im[v]);
  }
}

// 1-2. Reduction to standard form.  Gaussian elimination without pivoting on
// the overlap B (Hermitian positive definite: the pivots are those of its
// L D L^H factorisation), applying the same row operations to W = I, leaves
// W = L^-1 (unit lower triangular, in F) and D on the diagonal of B; with the
// Cholesky factor C = L D^1/2, C^-1 = D^-1/2 W (D^-1/2 in dsc), and
// A <- C^-1 A C^-H = D^-1/2 (W A W^H) D^-1/2 by two tiled products, made
// Hermitian.  One barrier per column; V <- I when HASV.  A non-positive
// pivot j is reported as j + 1 in flag 0.
// W goes to F, or to U where F is absent (WINU).
template <int W, bool WINU, typename R, int M, int G, bool HASU, bool HASV>
__device__ void chol_reduce(Smem<R, M, G, HASU, HASV>& sh, int g, int t) {
  typedef typename Cx<R>::T C;
  auto& Wm = [&]() -> auto& {
    if constexpr (WINU) return sh.U[g]; else return sh.F[g];
  }();
  constexpr int TPM = M * M / W, NT = TileOf<W>::NT, S = M / NT;
  LHF_FOR_ENTRIES { Wm[r][c] = cmk<C>(r == c ? R(1) : R(0), R(0)); }
  __syncthreads();
#pragma unroll 1
  for (int j = 0; j < M - 1; ++j) {
    const R d = sh.B[g][j][j].x;
    const bool ok = d > R(0);
    const R dinv = ok ? rcp_(d) : R(1);
    if (t == 0 && !ok && sh.flag[g][0] == 0) sh.flag[g][0] = j + 1;
    // entries right of column j update B, the others W; the W entries of a
    // thread share column t % M (TPM is a multiple of M), so row j's entry of
    // that column is read once
    const int c = t % M;
    const C pj = c > j ? sh.B[g][j][c] : Wm[j][c];
    C xv[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      xv[k] = cmk<C>(R(0), R(0));
      if (r > j) {
        const C f = cscale(sh.B[g][r][j], dinv);
        xv[k] = csub(c > j ? sh.B[g][r][c] : Wm[r][c], cmul(f, pj));
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      if (r > j) {
        if (c > j) sh.B[g][r][c] = xv[k];
        else Wm[r][c] = xv[k];
      }
    }
    __syncthreads();
  }
  if (t < M) {
    const R d = sh.B[g][t][t].x;
    sh.dsc[g][t] = d > R(0) ? rsq_(d) : R(1);
    if (t == M - 1 && !(d > R(0)) && sh.flag[g][0] == 0) sh.flag[g][0] = M;
  }
  if constexpr (sizeof(R) == 8 && M >= 16 && G == 1) {
    // FP64 matrix cores, one 16 x 16 tile per wavefront: W A, stored as its
    // conjugate transpose A W^H (A Hermitian), then W (A W^H) scaled by
    // D^-1/2 on both sides
    const MfTile<M> mft;
    mf4 re, im;
    if (mft.on) mf_product<M, false>(mft, Wm, sh.A[g], re, im);
    __syncthreads();
    if (mft.on) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mft.r0 + mft.lk + 4 * v, c = mft.c0 + mft.lr;
        sh.A[g][c][r] = cmk<C>(re[v], -im[v]);
      }
    }
    __syncthreads();
    if (mft.on) {
      mf_product<M, false>(mft, Wm, sh.A[g], re, im);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mft.r0 + mft.lk + 4 * v, c = mft.c0 + mft.lr;
        const R sc = sh.dsc[g][r] * sh.dsc[g][c];
        sh.B[g][r][c] = cmk<C>(re[v] * sc, im[v] * sc);
      }
    }
    __syncthreads();
  } else {
    int ti, tj;
    tile_coords<M, NT>(t, ti, tj);
    C p[NT][NT];
    mm_tile_rh<M, NT>(sh.A[g], Wm, ti, tj, p);   // T = A W^H
    __syncthreads();
    store_tile<M, NT>(sh.A[g], ti, tj, p);
    __syncthreads();
    mm_tile<M, NT, false>(Wm, sh.A[g], ti, tj, R(0), p);   // W T, scaled by D^-1/2 on both sides
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) p[a][b] = cscale(p[a][b], sh.dsc[g][ti + a * S] * sh.dsc[g][tj + b * S]);
    store_tile<M, NT>(sh.B[g], ti, tj, p);
    __syncthreads();
  }
  LHF_FOR_ENTRIES {
    const C x = sh.B[g][r][c], y = sh.B[g][c][r];
    C s = cmk<C>(R(0.5) * (x.x + y.x), R(0.5) * (x.y - y.y));
    if (r == c) s.y = R(0);
    sh.A[g][r][c] = s;
    if constexpr (HASV) sh.V[g][r][c] = cmk<C>(r == c ? R(1) : R(0), R(0));
  }
  __syncthreads();
}

// Jacobi rotation of the Hermitian 2 x 2 block [[app, b], [conj b, aqq]]:
// cosine c, s = sin * b / |b| and the rotated diagonal (dp, dq), from the
// stable tangent t = sign(tau) / (|tau| + sqrt(1 + tau^2)), tau = (aqq - app) / (2 |b|).
// FP64 small angles (|b| < 1e-4 |d|, d = aqq - app: nearly diagonal matrices,
// late sweeps and refinement) use the expansions in x = |b|^2 / d^2,
//   t = (|b| / d)(1 - x + 2 x^2),  c = 1 - t^2 / 2 + 3 t^4 / 8,
// exact to below 1e-23 relative, with one division and no square root.
template <typename R, typename C>
__device__ __forceinline__ void rotation(R app, R aqq, C b, R& c, C& s, R& dp, R& dq) {
  const R ab2 = b.x * b.x + b.y * b.y;
  const R d = aqq - app;
  if constexpr (sizeof(R) == 8) {
    if (ab2 < R(1e-8) * d * d) {
      const R id = R(1) / d;
      const R x = ab2 * id * id;
      const R f = R(1) - x + R(2) * x * x;
      const R t2 = x * f * f;
      c = R(1) - R(0.5) * t2 + R(0.375) * t2 * t2;
      s = cscale(b, id * f * c);
      const R tb = ab2 * id * f;   // t |b|
      dp = app - tb;
      dq = aqq + tb;
      return;
    }
  }
  if (ab2 > R(0) && (sizeof(R) == 8 || ab2 > R(1e-30))) {
    const R ri = rsq_(ab2);        // 1 / |b|
    const R ab = ab2 * ri;
    const R tau = d * R(0.5) * ri;
    const R at = fabs(tau);
    R t;
    if (at > R(1e15)) {
      t = R(0.5) * rcp_(tau);
    } else {
      const R q = R(1) + tau * tau;
      t = (tau >= R(0) ? R(1) : R(-1)) * rcp_(at + q * rsq_(q));
    }
    c = rsq_(R(1) + t * t);
    s = cscale(b, t * c * ri);
    dp = app - t * ab;
    dq = aqq + t * ab;
  } else {
    c = R(1);
    s = cmk<C>(R(0), R(0));
    dp = app;
    dq = aqq;
  }
}

// 3. Jacobi sweeps on A (and V <- V J when WANTV).  In each round the thread
// owning a diagonal pair block computes that pair's rotation and publishes it
// in LDS; after a barrier every thread rotates its own 2 x 2 block in
// registers and writes it back in place (each entry belongs to exactly one
// block per round).  Wide layout (W = 1): lane 4 blk + 2 a + b owns entry
// (a ? q_i : p_i, b ? q_j : p_j) of pair block blk = (i, j); every lane of
// the block reads the block's four entries before the round's first barrier
// and writes its own after it.  Returns the buffer holding the result
// (always A here).
template <int W, typename R, int M, int G, bool HASU, bool HASV, bool WANTV>
__device__ int jacobi(Smem<R, M, G, HASU, HASV>& sh, int g, int t, int maxsw, R tol) {
  typedef typename Cx<R>::T C;
  constexpr int H = M / 2, TPM = M * M / W;
  R nloc = R(0);
  LHF_FOR_ENTRIES {
    const C a = sh.A[g][r][c];
    nloc += a.x * a.x + a.y * a.y;
  }
  const R nrm2 = group_sum<W>(sh, g, t, nloc);
  const int blk = W == 4 ? t : t >> 2;
  const int bi = blk / H, bj = blk % H;
  const int ea = W == 4 ? 0 : (t >> 1) & 1, eb = W == 4 ? 0 : t & 1;   // wide: entry within the block
#pragma unroll 1
  for (int sw = 0;; ++sw) {
    R oloc = R(0);
    LHF_FOR_ENTRIES {
      const C a = sh.A[g][r][c];
      if (r != c) oloc += a.x * a.x + a.y * a.y;
    }
    const R off = group_sum<W>(sh, g, t, oloc);
    int st = off <= tol * tol * nrm2 ? 1 : 0;
    R corr[W];
    if constexpr (!WANTV) {
      // Second-order closure for eigenvalues only.  With D = diag(A), E the
      // off-diagonal part and rho_pq = |e_pq| / |d_p - d_q|, the eigenvalue
      // of D + E next to d_p is d_p + sum_q |e_pq|^2 / (d_p - d_q) + r_p with
      // the third-order term bounded by max|e| (sum_q rho_pq)^2 (higher orders
      // by a geometric factor when sum_q rho_pq <= 1/8).  When that bound is
      // below the stopping bound tol ||A||_F for every row, the corrected
      // diagonal is the result and the remaining sweep is skipped.
      // Tried only once (off / ||A||^2)^3 <= M^4 tol^2, which every accepted
      // case satisfies (rho of the largest entry >= sqrt(off) / (2 M ||A||_F)).
      const R x = off / nrm2;
      bool rowok = false;
#pragma unroll
      for (int k = 0; k < W; ++k) corr[k] = R(0);
      if (x * x * x <= R(M * M) * R(M * M) * tol * tol) {
        const R dc = sh.A[g][t % M][t % M].x;
        const R emax = sqrt(off);
        rowok = true;
        LHF_FOR_ENTRIES {
          const C a = sh.A[g][r][c];
          const R d = sh.A[g][r][r].x - dc;
          const R ab2 = a.x * a.x + a.y * a.y;
          R term = R(0), rho = R(0);
          if (r != c) {
            const R ad = fabs(d);
            rho = ad > R(0) ? sqrt(ab2) / ad : R(1e30);
            term = ad > R(0) ? ab2 / d : R(0);
          }
#pragma unroll
          for (int o = M / 2; o > 0; o >>= 1) {
            term += __shfl_xor(term, o, 64);
            rho += __shfl_xor(rho, o, 64);
          }
          corr[k] = term;
          rowok = rowok && rho <= R(0.125) && emax * rho * rho <= R(0.25) * tol * sqrt(nrm2);
        }
      }
      const R nbad = group_sum<W>(sh, g, t, rowok ? R(0) : R(1));
      if (st == 0 && nbad == R(0)) st = 2;
    }
    if (t == 0) sh.flag[g][2] = st;
    __syncthreads();
    bool all = true;
#pragma unroll
    for (int gg = 0; gg < G; ++gg) all = all && sh.flag[gg][2] != 0;
    if (all || sw == maxsw) {
      if constexpr (!WANTV) {
        if (sh.flag[g][2] == 2) {
          LHF_FOR_ENTRIES {
            if (r == c) sh.A[g][r][r].x += corr[k];
          }
        }
        __syncthreads();
      }
      break;
    }
#pragma unroll 1
    for (int s = 0; s < M - 1; ++s) {
      int pi, qi, pj, qj;
      pair_of<M>(bi, s, pi, qi);
      pair_of<M>(bj, s, pj, qj);
      C a00 = sh.A[g][pi][pj], a01 = sh.A[g][pi][qj], a10 = sh.A[g][qi][pj], a11 = sh.A[g][qi][qj];
      C vp, vq;   // wide layout: V entries (row, p_j), (row, q_j) of this lane's row
      const int row = ea ? qi : pi;
      if constexpr (W == 1 && WANTV) {
        vp = sh.V[g][row][pj];
        vq = sh.V[g][row][qj];
      }
      if (bi == bj && ea == 0 && eb == 0) {
        R cs, dp, dq;
        C sv;
        rotation<R, C>(a00.x, a11.x, a01, cs, sv, dp, dq);
        sh.jc[g][bi] = cs;
        sh.js[g][bi] = sv;
        sh.dn[g][pi] = dp;
        sh.dn[g][qi] = dq;
      }
      __syncthreads();
      const R ci = sh.jc[g][bi], cj = sh.jc[g][bj];
      const C si = sh.js[g][bi], sj = sh.js[g][bj];
      const C msj = cmk<C>(-sj.x, sj.y);   // J_qp of pair j = -conj(s_j)
      if constexpr (W == 4) {
        if (bi == bj) {
          a00 = cmk<C>(sh.dn[g][pi], R(0));
          a11 = cmk<C>(sh.dn[g][qi], R(0));
          a01 = cmk<C>(R(0), R(0));
          a10 = cmk<C>(R(0), R(0));
        } else {
          // T = A J_j, then A' = J_i^H T
          const C t00 = cadd(cscale(a00, cj), cmul(a01, msj));
          const C t01 = cadd(cmul(a00, sj), cscale(a01, cj));
          const C t10 = cadd(cscale(a10, cj), cmul(a11, msj));
          const C t11 = cadd(cmul(a10, sj), cscale(a11, cj));
          a00 = csub(cscale(t00, ci), cmul(si, t10));
          a01 = csub(cscale(t01, ci), cmul(si, t11));
          a10 = cadd(cmulc(si, t00), cscale(t10, ci));
          a11 = cadd(cmulc(si, t01), cscale(t11, ci));
        }
        sh.A[g][pi][pj] = a00; sh.A[g][pi][qj] = a01; sh.A[g][qi][pj] = a10; sh.A[g][qi][qj] = a11;
        if constexpr (WANTV) {
          // columns {pj, qj} of rows {pi, qi}: V <- V J_j
          C up = sh.V[g][pi][pj], uq = sh.V[g][pi][qj];
          sh.V[g][pi][pj] = cadd(cscale(up, cj), cmul(uq, msj));
          sh.V[g][pi][qj] = cadd(cmul(up, sj), cscale(uq, cj));
          up = sh.V[g][qi][pj]; uq = sh.V[g][qi][qj];
          sh.V[g][qi][pj] = cadd(cscale(up, cj), cmul(uq, msj));
          sh.V[g][qi][qj] = cadd(cmul(up, sj), cscale(uq, cj));
        }
      } else {
        // this lane's entry (ea, eb) of J_i^H A J_j: column eb of J_j is
        // (j0, j1) = (cj, -conj(sj)) or (sj, cj); row ea of J_i^H is
        // (ci, -si) or (conj(si), ci)
        const C j0 = cmk<C>(eb ? sj.x : cj, eb ? sj.y : R(0));
        const C j1 = cmk<C>(eb ? cj : msj.x, eb ? R(0) : msj.y);
        const C t0 = cadd(cmul(a00, j0), cmul(a01, j1)), t1 = cadd(cmul(a10, j0), cmul(a11, j1));
        const C r0 = cmk<C>(ea ? si.x : ci, ea ? -si.y : R(0));   // coefficient of t0
        const C r1 = cmk<C>(ea ? ci : -si.x, ea ? R(0) : -si.y);  // coefficient of t1
        C res = cadd(cmul(r0, t0), cmul(r1, t1));
        if (bi == bj) {
          const R dv = sh.dn[g][row];
          res = cmk<C>(ea == eb ? dv : R(0), R(0));
        }
        sh.A[g][row][eb ? qj : pj] = res;
        if constexpr (WANTV) sh.V[g][row][eb ? qj : pj] = cadd(cmul(vp, j0), cmul(vq, j1));
      }
      __syncthreads();
    }
  }
  return 0;
}

// 4. Eigenvalues (diagonal of A) and their ascending ranks among the first m.
template <typename R, int M, int G, bool HASU, bool HASV>
__device__ void eig_rank(Smem<R, M, G, HASU, HASV>& sh, int g, int t, int m, int cur) {
  if (t < M) sh.lam[g][t] = (cur ? sh.B[g] : sh.A[g])[t][t].x;
  __syncthreads();
  if (t < m) {
    const R lr = sh.lam[g][t];
    int k = 0;
    for (int y = 0; y < m; ++y) {
      const R ly = sh.lam[g][y];
      k += (ly < lr || (ly == lr && y < t)) ? 1 : 0;
    }
    sh.rank[g][t] = k;
  }
  __syncthreads();
}

// (re, im) = W Y with the unit lower triangular W held in the strictly upper
// triangle of B (W_rk at B[k][r], r > k)
template <int M>
__device__ __forceinline__ void mf_product_wup(const MfTile<M>& f, const double2 (&B)[M][M + 1],
                                               const double2 (&Y)[M][M + 1], mf4& re, mf4& im) {
  re = mf4{0.0, 0.0, 0.0, 0.0};
  im = mf4{0.0, 0.0, 0.0, 0.0};
  const int r = f.r0 + f.lr;
#pragma unroll
  for (int k0 = 0; k0 < M; k0 += 4) {
    const int k = k0 + f.lk;
    const double2 b = B[k][r];
    const double2 x = r == k ? make_double2(1.0, 0.0) : (r > k ? b : make_double2(0.0, 0.0));
    const double2 y = Y[k][f.c0 + f.lr];
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, re, 0, 0, 0);
    re = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.y, y.y, re, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.y, im, 0, 0, 0);
    im = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.x, im, 0, 0, 0);
  }
}

// 1-2'. Reduction to standard form without the W array (FP64 eigenvalues):
// the same elimination as chol_reduce, run on the lower triangle
// of B (the trailing block stays Hermitian, so row j right of the diagonal is
// the conjugate of column j below it), with W = L^-1 kept in the strictly
// upper triangle of B (W_rc, r > c, at B[c][r]; the unit diagonal implied).
// Within step j the lower entries of columns > j and the upper entries of
// columns > j are written while column j is read: no entry is both.  Then
// A <- D^-1/2 W A W^H D^-1/2, on the matrix cores as in chol_reduce when one
// matrix fills the workgroup (M >= 16), else per entry on the vector units,
// with a barrier before B is overwritten by the product.
template <int W, int M, int G>
__device__ void chol_reduce_wup(Smem<double, M, G, false, false, true>& sh, int g, int t) {
  typedef double2 C;
  typedef double R;
  constexpr int TPM = M * M / W;
  auto& B = sh.B[g];
  auto& A = sh.A[g];
  LHF_FOR_ENTRIES {
    if (c > r) B[r][c] = cmk<C>(R(0), R(0));   // W = I below the diagonal
  }
  __syncthreads();
  const int c = t % M;   // the W entries of a thread share this column
  // Steps in pairs (j, j1 = j + 1), one barrier per pair: with f_r = B_rj / d_j,
  // row j1 after step j is known to every thread from column j and j1
  // (d1 = B_j1j1 - |B_j1j|^2 / d_j, g_r = (B_rj1 - f_r conj(B_j1j)) / d1), so
  // rows r > j1 take both steps at once, x -= f_r p_j + g_r p_j1.  Row j1's
  // own new entries (its W row and d1) are read in this pass by others, so
  // they are written after the barrier, at the start of the next pass, when
  // no one reads column j1 any more.
  bool pend = false;
  int pa = 0, pb = 0;
  C pv = cmk<C>(R(0), R(0));
  int j = 0;
#pragma unroll 1
  for (; j + 1 < M - 1; j += 2) {
    if (pend) {
      B[pa][pb] = pv;
      pend = false;
    }
    const int j1 = j + 1;
    const R d = B[j][j].x;
    const bool ok = d > R(0);
    const R dinv = ok ? rcp_(d) : R(1);
    const C bj1 = B[j1][j];
    const C f1 = cscale(bj1, dinv);
    const R d1 = B[j1][j1].x - (bj1.x * bj1.x + bj1.y * bj1.y) * dinv;
    const bool ok1 = d1 > R(0);
    const R d1inv = ok1 ? rcp_(d1) : R(1);
    if (t == 0 && sh.flag[g][0] == 0) {
      if (!ok) sh.flag[g][0] = j + 1;
      else if (!ok1) sh.flag[g][0] = j1 + 1;
    }
    // rows j and j1 (after step j) of [B | W] in column c
    const C bcj = B[c][j], bcj1 = B[c][j1];
    C pj, pj1;
    if (c > j1) {
      pj = cconj(bcj);
      pj1 = cconj(csub(bcj1, cmul(bcj, cconj(f1))));
    } else if (c == j1) {
      pj = cconj(bj1);
      pj1 = cmk<C>(R(1), R(0));
    } else if (c == j) {
      pj = cmk<C>(R(1), R(0));
      pj1 = cmk<C>(-f1.x, -f1.y);
    } else {
      pj = bcj;
      pj1 = csub(bcj1, cmul(f1, bcj));
    }
    C xv[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      xv[k] = cmk<C>(R(0), R(0));
      if (r > j1 && (c <= j1 || c <= r)) {
        const C fr = cscale(B[r][j], dinv);
        const C gr = cscale(csub(B[r][j1], cmul(fr, cconj(bj1))), d1inv);
        if (c == j1) {
          xv[k] = cmk<C>(-gr.x, -gr.y);
        } else {
          xv[k] = csub(csub(c > j1 ? B[r][c] : B[c][r], cmul(fr, pj)), cmul(gr, pj1));
        }
      } else if (r == j1 && c <= j1) {
        pend = true;
        pa = c == j1 ? j1 : c;
        pb = j1;
        pv = c == j1 ? cmk<C>(d1, R(0)) : pj1;
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      if (r > j1) {
        if (c > j1) {
          if (c <= r) B[r][c] = xv[k];
        } else {
          B[c][r] = xv[k];
        }
      }
    }
    __syncthreads();
  }
  if (pend) B[pa][pb] = pv;
  __syncthreads();
  // the last step when M - 1 is odd
#pragma unroll 1
  for (; j < M - 1; ++j) {
    const R d = B[j][j].x;
    const bool ok = d > R(0);
    const R dinv = ok ? rcp_(d) : R(1);
    if (t == 0 && !ok && sh.flag[g][0] == 0) sh.flag[g][0] = j + 1;
    const C bc = B[c][j];
    const C pj = c > j ? cconj(bc) : (c == j ? cmk<C>(R(1), R(0)) : bc);
    C xv[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      xv[k] = cmk<C>(R(0), R(0));
      if (r > j && (c <= j || c <= r)) {
        const C f = cscale(B[r][j], dinv);
        xv[k] = csub(c > j ? B[r][c] : B[c][r], cmul(f, pj));
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int r = (t + k * TPM) / M;
      if (r > j) {
        if (c > j) {
          if (c <= r) B[r][c] = xv[k];
        } else {
          B[c][r] = xv[k];
        }
      }
    }
    __syncthreads();
  }
  if (t < M) {
    const R d = B[t][t].x;
    sh.dsc[g][t] = d > R(0) ? rsq_(d) : R(1);
    if (t == M - 1 && !(d > R(0)) && sh.flag[g][0] == 0) sh.flag[g][0] = M;
  }
  if constexpr (M >= 16 && G == 1) {
    const MfTile<M> mft;
    mf4 re, im;
    if (mft.on) mf_product_wup<M>(mft, B, A, re, im);   // W A
    __syncthreads();
    if (mft.on) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mft.r0 + mft.lk + 4 * v, cc = mft.c0 + mft.lr;
        A[cc][r] = cmk<C>(re[v], -im[v]);   // (W A)^H = A W^H
      }
    }
    __syncthreads();
    if (mft.on) mf_product_wup<M>(mft, B, A, re, im);   // W A W^H
    __syncthreads();                                   // every read of W in B done
    if (mft.on) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mft.r0 + mft.lk + 4 * v, cc = mft.c0 + mft.lr;
        const R sc = sh.dsc[g][r] * sh.dsc[g][cc];
        B[r][cc] = cmk<C>(re[v] * sc, im[v] * sc);
      }
    }
    __syncthreads();
  } else {
    // T = A W^H (W_ck at B[k][c] for k < c), then W T (W_rk at B[k][r])
    C tv[W];
    LHF_FOR_ENTRIES {
      C acc = A[r][c];
#pragma unroll
      for (int q = 0; q < M - 1; ++q)
        if (q < c) acc = cadd(acc, cmul(A[r][q], cconj(B[q][c])));
      tv[k] = acc;
    }
    __syncthreads();
    LHF_FOR_ENTRIES { A[r][c] = tv[k]; }
    __syncthreads();
    LHF_FOR_ENTRIES {
      C acc = A[r][c];
#pragma unroll
      for (int q = 0; q < M - 1; ++q)
        if (q < r) acc = cadd(acc, cmul(B[q][r], A[q][c]));
      tv[k] = cscale(acc, sh.dsc[g][r] * sh.dsc[g][c]);
    }
    __syncthreads();   // every read of W in B done
    LHF_FOR_ENTRIES { B[r][c] = tv[k]; }
    __syncthreads();
  }
  LHF_FOR_ENTRIES {
    const C x = B[r][c], y = B[c][r];
    C s2 = cmk<C>(R(0.5) * (x.x + y.x), R(0.5) * (x.y - y.y));
    if (r == c) s2.y = R(0);
    A[r][c] = s2;
  }
  __syncthreads();
}

// 3'-4'. Eigenvalues only: Householder reduction of the Hermitian A (its
// leading n x n block) to tridiagonal form, then bisection on Sturm counts.
// Step h reflects rows and columns h+1..n-1 with P = I - beta u u^H,
// u = x + phase(x_0) |x| e_0 (x: column h below the diagonal), so the new
// subdiagonal entry has modulus |x|; the trailing block is updated as
// A <- A - u q^H - q u^H with p = beta A u, q = p - (beta u^H p / 2) u.  The
// tridiagonal matrix with complex subdiagonal has the spectrum of the real one
// with the moduli (a diagonal unitary similarity), so only d_i and e_i^2 are
// kept.  Eigenvalue i (ascending) is found by the P = M / W lanes of row
// group i: each counts the eigenvalues below interior points of the current
// interval and the group keeps the sub-interval holding it, until its width is
// a few ulps of the interval or of the matrix norm.  The count at x is the
// number of sign changes of the leading minors p_j of T - x I, from the
// division-free recurrence p_j = (d_j - x) p_(j-1) - e_(j-1)^2 p_(j-2)
// (sturm_row: a zero taken as positive; a matrix with a zero interior
// coupling takes the row that restarts the recurrence there, the others the
// plain one), on T scaled by a power of two to norm below 1 and rescaled by
// 2^-+256 every eighth row against overflow and underflow (exact,
// sign-preserving).  Each lane runs one
// sequence (P + 1 sections per pass), or two in groups of one or two lanes.
// The points of a pass increase along the group's lanes and the counts are
// monotone in x, so the points with count <= i form a prefix: its length k,
// from ballots, gives the new interval [point k, point k + 1] directly.  The
// eigenvalues land sorted: rank i = i.
template <int W, typename R, int M, int G, bool HASU, bool HASV, bool NOF>
__device__ void tridiag_eigs(Smem<R, M, G, HASU, HASV, NOF>& sh, int g, int t, int n) {
  typedef typename Cx<R>::T C;
  constexpr int TPM = M * M / W, P = TPM / M;
  static_assert(P >= 1 && (P & (P - 1)) == 0 && P <= 64, "row group of one wavefront");
  static_assert(M >= 4, "size classes start at 4");
  R* dg = sh.dsc[g];        // diagonal d
  R* e2 = sh.dn[g];         // squared subdiagonal moduli
  C* de = &sh.B[g][2][0];   // (d_j, e_(j-1)^2) per row, one LDS word for the Sturm pass
  const int gi = t / P, gc = t % P;   // row group and lane within it
  auto add = [](double x, double y) { return x + y; };
  // The reduction keeps the matrix in registers, column by column: lane gc of
  // group gi holds column gi, rows gc + P k (k < W), so the column norm and
  // (A^H u)_c are all-reduces over the group's P lanes (an aligned DPP
  // group).  Per step h: the group owning column h forms u and beta; barrier;
  // every group forms p_c = beta sum_r conj(A_rc) u_r (= (beta A u)_c, A
  // Hermitian) and publishes p_c and Re(conj(u_c) p_c); barrier; every lane
  // updates its entries, and the owner of column h + 1 goes straight on to
  // the next reflector, its column being current (with several wavefronts
  // per matrix its wavefront updates at raised priority).  u, p, those
  // products and beta are double-buffered in LDS by the parity of h, so two
  // barriers per step keep every read ahead of the next overwrite.
  C* const lb = &sh.B[g][0][0];   // B is free after the reduction
  C* const ubuf = lb;             // u: [2][M]
  C* const pbuf = lb + 2 * M;     // p: [2][M]
  R* const upbuf = reinterpret_cast<R*>(lb + 4 * M);   // Re(conj(u_i) p_i): [2][M]
  R* const bbuf = sh.red[g];      // beta = 2 / u^H u (0: no reflection): [2]
  C a[W];
#pragma unroll
  for (int k = 0; k < W; ++k) a[k] = sh.A[g][gc + P * k][gi];
#pragma unroll 1
  for (int h = 0; h < M - 2; ++h) {
    const int bsel = h & 1;
    const bool act = h < n - 2;
    C* const u = ubuf + bsel * M;
    C* const pv = pbuf + bsel * M;
    R* const upv = upbuf + bsel * M;
    if (gi == h) {
      // x: column h below the diagonal; a2 = |x_0|^2 (row h + 1), x2 the rest
      R a2 = R(0), x2 = R(0);
      C al = cmk<C>(R(0), R(0));
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const int r = gc + P * k;
        const R v = a[k].x * a[k].x + a[k].y * a[k].y;
        if (r == h + 1) {
          a2 += v;
          al = a[k];
        } else if (r > h + 1 && r < n) {
          x2 += v;
        }
      }
      lane_reduce2<P>(a2, x2, add);
      const R ar = sqrt(a2), nrm = sqrt(a2 + x2);
      // u = phase(x_0) (|x_0| + |x|) e_0 + x scaled by sc = |x_0| (1 when
      // x_0 = 0), which needs no division: u_(h+1) = x_0 (|x_0| + |x|),
      // u_r = |x_0| x_r below, zero elsewhere; hh = u^H u / 2 =
      // sc^2 |x| (|x| + |x_0|), published as beta = 1 / hh
      const R sc = ar > R(0) ? ar : R(1);
      const C u1 = ar > R(0) ? cscale(al, ar + nrm) : cmk<C>(nrm, R(0));
      const R hh = act && x2 > R(0) ? sc * sc * (nrm * (nrm + ar)) : R(0);
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const int r = gc + P * k;
        const bool in = act && r > h && r < n;
        u[r] = in ? (r == h + 1 ? u1 : cscale(a[k], sc)) : cmk<C>(R(0), R(0));
      }
      if (gc == 0) {
        bbuf[bsel] = hh != R(0) ? rcp_fast(hh) : R(0);
        if (act) e2[h] = a2 + x2;
      }
    }
    if constexpr (TPM > 64) __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    const R beta = bbuf[bsel];
    const bool refl = beta != R(0);
    const bool colok = gi > h && gi < n;
    C ur[W], pc = cmk<C>(R(0), R(0));
#pragma unroll
    for (int k = 0; k < W; ++k) ur[k] = u[gc + P * k];
    const C uc = u[gi];
    if (refl) {
      C sacc = cmulc(a[0], ur[0]);   // conj(A_rc) u_r
#pragma unroll
      for (int k = 1; k < W; ++k) sacc = cadd(sacc, cmulc(a[k], ur[k]));
      lane_reduce2<P>(sacc.x, sacc.y, add);
      pc = cscale(sacc, beta);
      if (gc == 0) {
        pv[gi] = pc;
        upv[gi] = colok ? uc.x * pc.x + uc.y * pc.y : R(0);
      }
    }
    __syncthreads();
    if (refl) {
      // several wavefronts per matrix: the one owning the next column goes
      // first, so that its reflector work overlaps the others' updates
      if constexpr (TPM > 64) {
        if ((t >> 6) == ((h + 1) * P >> 6)) __builtin_amdgcn_s_setprio(1);
      }
      // K = beta u^H p / 2, four partial sums over the rows
      R ks4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) ks4[i] = upv[i];
#pragma unroll
      for (int i = 4; i < M; ++i) ks4[i & 3] += upv[i];
      const R kk = R(0.5) * beta * ((ks4[0] + ks4[1]) + (ks4[2] + ks4[3]));
      C pr[W];
#pragma unroll
      for (int k = 0; k < W; ++k) pr[k] = pv[gc + P * k];
      const C qc = csub(pc, cscale(uc, kk));
      if (colok) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int r = gc + P * k;
          if (r > h && r < n) {
            const C qr = csub(pr[k], cscale(ur[k], kk));
            // A_rc -= u_r conj(q_c) + q_r conj(u_c)
            a[k] = csub(a[k], cadd(cmulc(qc, ur[k]), cmulc(uc, qr)));
          }
        }
      }
    }
  }
  // d and the last squared coupling |A_(n-1, n-2)|^2 from the registers
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int r = gc + P * k;
    if (r == gi && gi < n) dg[gi] = a[k].x;
    if (n >= 2 && gi == n - 2 && r == n - 1) e2[n - 2] = a[k].x * a[k].x + a[k].y * a[k].y;
  }
  __syncthreads();
  // Gershgorin interval of the tridiagonal matrix, one row per lane t < M of
  // the group's first wavefront (the M lanes are an aligned DPP group), then
  // lo, hi and the largest e^2 by all-reduces over them; rows past n are
  // neutral
  constexpr R eps = R(1.1102230246251565e-16);
  constexpr R kHuge = R(1.79e308);
  const bool rowl = t < n;
  const R er = rowl && t < n - 1 ? e2[t < M ? t : 0] : R(0);
  const R erm = rowl && t > 0 ? e2[t > 0 && t <= M ? t - 1 : 0] : R(0);
  const R dr = rowl ? dg[t < M ? t : 0] : R(0);
  const R rad = sqrt(er) + sqrt(erm);
  R lo = lane_reduce<M>(rowl ? dr - rad : kHuge, [](double x, double y) { return fmin(x, y); });
  R hi = lane_reduce<M>(rowl ? dr + rad : -kHuge, [](double x, double y) { return fmax(x, y); });
  R emax = lane_reduce<M>(er, [](double x, double y) { return fmax(x, y); });
  // the pass runs on T scaled by sc = 2^-ex (exact), |T| < 1, so the minors
  // grow at most 3x per row and a rescale every eighth row suffices
  int ex = 0;
  (void)frexp(fmax(fabs(lo), fabs(hi)), &ex);
  const R sc = ldexp(R(1), -ex);
  lo *= sc;
  hi *= sc;
  emax *= sc * sc;
  R tnorm = fmax(fabs(lo), fabs(hi));
  R tiny = R(2.2250738585072014e-308) * fmax(R(1), emax);   // absolute floor of the widths
  const R widen = R(4) * R(n) * eps * tnorm + R(2) * tiny;
  lo -= widen;
  hi += widen;
  // rows past n: d beyond the interval (d - x > 0, bounded) and e = 0, so
  // they change no sign and the pass runs over all M rows without selects
  // (the plain row keeps p_j = (d - x) p_(j-1) there, the restarting one
  // starts a positive sequence)
  const R dpad = R(2) * fmax(fabs(lo), fabs(hi)) + R(1);
  const R e2s = erm * sc * sc;
  // a zero interior coupling after scaling (the same for the whole matrix)
  const unsigned long long zb = __ballot(t >= 1 && t < n && e2s == R(0));
  if (t < M) {
    de[t] = t < n ? cmk<C>(dr * sc, e2s) : cmk<C>(dpad, R(0));
    const int base = (int)(threadIdx.x & 63) - t;   // lane of row 0
    const unsigned long long rmask = M >= 64 ? ~0ull : (((1ull << M) - 1ull) << base);
    if (t == 0) {
      R* b = sh.red[g];
      b[0] = lo;
      b[1] = hi;
      b[2] = tnorm;
      b[3] = tiny;
      b[4] = R(ex);
      b[5] = (zb & rmask) ? R(1) : R(0);
    }
  }
  __syncthreads();
  {
    const R* b = sh.red[g];
    lo = b[0];
    hi = b[1];
    tnorm = b[2];
    tiny = b[3];
    ex = (int)b[4];
  }
  const bool split = sh.red[g][5] != R(0);
  const bool live = gi < n;
  // (d_j, e_(j-1)^2) in registers for M <= 16, read from LDS per row for M = 32
  constexpr int ND = M <= 16 ? M : 1;
  C drr[ND];
  if constexpr (M <= 16) {
#pragma unroll
    for (int j = 0; j < M; ++j) drr[j] = de[j];
  }
  auto dr_at = [&](int j) -> C {
    if constexpr (M <= 16) return drr[j]; else return de[j];
  };
  // SH sequences per lane, NPT = SH P points per pass: one sequence when the
  // group has four or more lanes (the passes are issue-bound, and one point
  // per lane costs fewer row evaluations to the bit), two for smaller groups,
  // where the fixed cost of a pass dominates.  Point i (1..NPT): the same
  // expression where it is evaluated and where it becomes an end of the new
  // interval
  constexpr int SH = P >= 4 ? 1 : 2, NPT = SH * P;
  const R inv = R(1) / R(NPT + 1);
  auto point = [&](int i) { return fma(hi - lo, R(i) * inv, lo); };
  const int gbase = ((int)(threadIdx.x & 63) / P) * P;   // first lane of the group in its wavefront
  const unsigned long long gmask = P >= 64 ? ~0ull : ((1ull << P) - 1ull);
  constexpr R kBig = R(1.157920892373162e77), kSmall = R(8.636168555094445e-78);   // 2^256, 2^-256
  auto passes = [&](auto splitc) {
  constexpr bool SPLIT = decltype(splitc)::value;
#pragma unroll 1
  for (int it = 0; it < 96; ++it) {
    const bool conv = !live || hi - lo <= R(2) * eps * fmax(fabs(lo), fabs(hi)) + eps * tnorm + R(4) * tiny;
    if (__all(conv)) break;
    const R xa = point(SH * gc + 1), xb = SH == 2 ? point(SH * gc + 2) : xa;
    int ca = 0, cb = 0;
    if (live) {
      const C d0 = dr_at(0);
      R pa2 = R(1), pb2 = R(1), pa1 = d0.x - xa, pb1 = d0.x - xb;
      int na = sign_bit(pa1), nb = sign_bit(pb1);
      ca = na;
      cb = nb;
      // row j of the pass; rescale after rows 7, 15, 23, ... (RS: j % 8 == 7,
      // known at compile time in every caller)
      auto row = [&](int j, auto rs) {
        constexpr bool RS = decltype(rs)::value;
        const C dj = dr_at(j);
        sturm_row<SPLIT>(dj.x, dj.y, xa, pa1, pa2, na, ca);
        if constexpr (SH == 2) sturm_row<SPLIT>(dj.x, dj.y, xb, pb1, pb2, nb, cb);
        if constexpr (RS) {
          const R sa = fabs(pa1) > kBig ? kSmall : (fabs(pa1) < kSmall ? kBig : R(1));
          pa1 *= sa;
          pa2 *= sa;
          if constexpr (SH == 2) {
            const R sb = fabs(pb1) > kBig ? kSmall : (fabs(pb1) < kSmall ? kBig : R(1));
            pb1 *= sb;
            pb2 *= sb;
          }
        }
      };
      using RsYes = std::integral_constant<bool, true>;
      using RsNo = std::integral_constant<bool, false>;
      // rows 1 to min(M, 8) - 1, then blocks of eight rows with the rescale
      // after the last (rows past n count nothing)
      row(1, RsNo{});
      row(2, RsNo{});
      row(3, RsNo{});
      if constexpr (M >= 8) {
        row(4, RsNo{});
        row(5, RsNo{});
        row(6, RsNo{});
        row(7, RsYes{});
      }
      auto block8 = [&](int jb) {
        row(jb, RsNo{});
        row(jb + 1, RsNo{});
        row(jb + 2, RsNo{});
        row(jb + 3, RsNo{});
        row(jb + 4, RsNo{});
        row(jb + 5, RsNo{});
        row(jb + 6, RsNo{});
        row(jb + 7, RsYes{});
      };
      if constexpr (M == 16) {
        block8(8);
      } else if constexpr (M > 16) {
        // rolled over blocks (d and e come from LDS)
#pragma unroll 1
        for (int jb = 8; jb < M; jb += 8) block8(jb);
      }
    }
    const unsigned long long ba = __ballot(ca <= gi);
    int k = __popcll((ba >> gbase) & gmask);
    if constexpr (SH == 2) k += __popcll((__ballot(cb <= gi) >> gbase) & gmask);
    if (!conv) {
      const R nlo = k == 0 ? lo : point(k);
      const R nhi = k == NPT ? hi : point(k + 1);
      lo = nlo;
      hi = nhi;
    }
  }
  };
  if (split) passes(std::true_type{}); else passes(std::false_type{});
  if (live && gc == 0) {
    sh.lam[g][gi] = ldexp(R(0.5) * (lo + hi), ex);
    sh.rank[g][gi] = gi;
  }
  if (t == 0) sh.flag[g][2] = 1;
  __syncthreads();
}

// Eigenvectors C^-H V = W^H D^-1/2 V into A (one tiled product).
template <int W, typename R, int M, int G, bool HASU, bool HASV>
__device__ void backsub_vectors(Smem<R, M, G, HASU, HASV>& sh, int g, int t) {
  typedef typename Cx<R>::T C;
  constexpr int NT = TileOf<W>::NT;
  int ti, tj;
  tile_coords<M, NT>(t, ti, tj);
  C p[NT][NT];
  mm_tile_lh_diag<M, NT>(sh.F[g], sh.dsc[g], sh.V[g], ti, tj, p);
  store_tile<M, NT>(sh.A[g], ti, tj, p);
  __syncthreads();
}

// Threads per matrix TPM = M^2 / W (W = 4 entries per thread, or 1: the
// wide layout for batches too small to fill the device), G matrices per
// workgroup (one wavefront when TPM < 64).
template <int M, int W>
struct Shape {
  static constexpr int TPM = M * M / W;
  static constexpr int G = TPM >= 64 ? 1 : 64 / TPM;
  static constexpr int THREADS = G * TPM;
};

// Solve in precision R from Fourier blocks of complex type CIN (rounded to R
// on load).  VMODE: 0 none, 1 write vectors to V (caller, sorted columns),
// 2 write vectors to U (FP32 workspace).
template <typename R, int M, int VMODE, int W, typename CIN>
__global__ void __launch_bounds__((Shape<M, W>::THREADS)) heev_kernel(const LatDev* __restrict__ lats,
                                                                 const int2* __restrict__ canon, int ncanon,
                                                                 const CIN* __restrict__ Hb,
                                                                 const CIN* __restrict__ Sb,
                                                                 double* __restrict__ w,
                                                                 typename Cx<R>::T* __restrict__ Vout,
                                                                 int32_t* __restrict__ info, int maxsw, R tol) {
  typedef typename Cx<R>::T C;
  constexpr int G = Shape<M, W>::G, TPM = Shape<M, W>::TPM;
  constexpr bool WANTV = VMODE != 0;
  // FP64 eigenvalues at M = 8 and 32: W in the upper triangle of B (no F
  // array), so more workgroups fit a CU's LDS (at M = 16 registers, not LDS,
  // bound the residency, and the full-matrix elimination is faster)
  constexpr bool NOF = VMODE == 0 && sizeof(R) == 8 && (M == 8 || M == 32);
  __shared__ Smem<R, M, G, false, WANTV, NOF> sh;
  const int g = threadIdx.x / TPM, t = threadIdx.x % TPM;
  const int slot = blockIdx.x * G + g;
  const bool valid = slot < ncanon;
  const int2 cb = canon[valid ? slot : ncanon - 1];   // a spare group repeats a block of its class, unwritten
  const LatDev& L = lats[cb.x];
  const int m = L.m0;
  const int blk = cb.y;
  const int cblk = conj_block(L, blk);
  const int64_t base = L.gen_off + (int64_t)blk * m * m;
  // every global load first (padding entries read entry 0 and discard it;
  // a spare group reads a valid block)
  C av[W], bv[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int e = t + k * TPM, r = e / M, c = e % M;
    const int64_t o = base + (r < m && c < m ? r * m + c : 0);
    const CIN hx = Hb[o], sx = Sb[o];
    av[k] = cmk<C>((R)hx.x, (R)hx.y);
    bv[k] = cmk<C>((R)sx.x, (R)sx.y);
  }
  if (t < 4) sh.flag[g][t] = 0;
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int e = t + k * TPM, r = e / M, c = e % M;
    C a = cmk<C>(R(0), R(0)), b = cmk<C>(r == c ? R(1) : R(0), R(0));
    if (valid && r < m && c < m) {
      a = av[k];
      b = bv[k];
      if (!(isfinite(a.x) && isfinite(a.y) && isfinite(b.x) && isfinite(b.y))) {
        bad = true;
        a = cmk<C>(R(0), R(0));
        b = cmk<C>(r == c ? R(1) : R(0), R(0));
      }
    }
    sh.A[g][r][c] = a;
    sh.B[g][r][c] = b;
  }
  if (bad) sh.flag[g][1] = 1;
  __syncthreads();
  if constexpr (NOF) chol_reduce_wup<W, M, G>(sh, g, t); else chol_reduce<W, false>(sh, g, t);
  if constexpr (VMODE == 0 && sizeof(R) == 8) {
    tridiag_eigs<W>(sh, g, t, m);
  } else {
    const int cur = jacobi<W, R, M, G, false, WANTV, WANTV>(sh, g, t, maxsw, tol);
    eig_rank(sh, g, t, m, cur);
  }
  if constexpr (WANTV) backsub_vectors<W>(sh, g, t);
  if (!valid) return;   // no barrier follows
  const int64_t wb = L.w_off + (int64_t)blk * m, wc = L.w_off + (int64_t)cblk * m;
  if (t < m) {
    const double lv = (double)sh.lam[g][t];
    w[wb + sh.rank[g][t]] = lv;
    if (cblk != blk) w[wc + sh.rank[g][t]] = lv;
  }
  if (WANTV) {
    const int64_t cb0 = L.gen_off + (int64_t)cblk * m * m;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int e = t + k * TPM, r = e / M, c = e % M;
      if (r < m && c < m) {
        const C v = sh.A[g][r][c];
        Vout[base + r * m + sh.rank[g][c]] = v;
        if (VMODE == 1 && cblk != blk) Vout[cb0 + r * m + sh.rank[g][c]] = cconj(v);
      }
    }
  }
  if (t == 0) {
    const int st = sh.flag[g][1] ? -2 : (sh.flag[g][0] ? sh.flag[g][0] : (sh.flag[g][2] ? 0 : -1));
    info[L.blk_off + blk] = st;
    if (cblk != blk) info[L.blk_off + cblk] = st;
  }
}

template <typename SM>
__device__ __forceinline__ auto& xbuf(SM& sh, int g) {
  if constexpr (SM::HASF) return sh.F[g]; else return sh.U[g];
}

// Refinement in FP64 from FP32 eigenvectors U (layout [blk][row][col]).
// Blocks from H64/S64 (complex128) or regenerated from the FP64 generator band.
template <int M, bool WANTV, int W>
__global__ void __launch_bounds__((Shape<M, W>::THREADS)) __attribute__((amdgpu_waves_per_eu(2))) refine_kernel(const LatDev* __restrict__ lats,
                                                                   const int2* __restrict__ canon, int ncanon,
                                                                   const double2* __restrict__ tw,
                                                                   const double2* __restrict__ H64,
                                                                   const double2* __restrict__ S64,
                                                                   const double* __restrict__ Hg,
                                                                   const double* __restrict__ Sg,
                                                                   const float2* __restrict__ U32,
                                                                   const int32_t* __restrict__ info32,
                                                                   double* __restrict__ w, double2* __restrict__ Vout,
                                                                   int32_t* __restrict__ info, int maxsw, double tol) {
  typedef double2 C;
  typedef double R;
  constexpr int G = Shape<M, W>::G, TPM = Shape<M, W>::TPM;
  // eigenvalues only: no V; the products' scratch is F (Rayleigh-Ritz) and
  // the dead U (congruence), so four matrices per group instead of five
  __shared__ Smem<R, M, G, true, WANTV> sh;
  const int g = threadIdx.x / TPM, t = threadIdx.x % TPM;
  const int slot = blockIdx.x * G + g;
  const bool valid = slot < ncanon;
  const int2 cb = canon[valid ? slot : ncanon - 1];   // a spare group repeats a block of its class, unwritten
  const LatDev& L = lats[cb.x];
  const int m = L.m0;
  const int blk = cb.y;
  const int cblk = conj_block(L, blk);
  const int64_t base = L.gen_off + (int64_t)blk * m * m;
  // every global load of the block first (padding entries read entry 0 and
  // discard it; a spare group reads a valid block; U of a block whose FP32
  // solve failed is discarded)
  C hv[W], sv[W];
  float2 uv[W];
  const int32_t st32 = info32[L.blk_off + blk];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int e = t + k * TPM, r = e / M, c = e % M;
    const int64_t o = base + (r < m && c < m ? r * m + c : 0);
    if (H64) {
      hv[k] = H64[o];
      sv[k] = S64[o];
    }
    uv[k] = U32[o];
  }
  if (t < 4) sh.flag[g][t] = 0;
  const bool fresh = !valid || st32 != 0;
  auto cell_of = [&](const DimDev& D, int s) -> int {
    if (D.full) return s;
    const int k = s - D.L0;
    return k < 0 ? k + D.L : k;
  };
  // regeneration path only (a uniform branch: with complex128 blocks none of
  // the band descriptors is read, so no load waits behind the block loads)
  int j1 = 0, j2 = 0, j3 = 0, ns1 = 1, ns2 = 1, ns3 = 1, ncell = 0;
  bool twl = false;
  // band-cell twiddles w^(j.k) of this block, cached in the storage of F
  // (free until the series) or, without F, of A until every lane has formed
  // its block entries
  C* twc = Smem<R, M, G, true, WANTV>::HASF ? &xbuf(sh, g)[0][0] : &sh.A[g][0][0];
  if (!H64) {
    j3 = blk % L.L[2];
    j2 = (blk / L.L[2]) % L.L[1];
    j1 = blk / (L.L[2] * L.L[1]);
    ns1 = L.dim[0].L == 1 ? 1 : L.dim[0].nshift;
    ns2 = L.dim[1].L == 1 ? 1 : L.dim[1].nshift;
    ns3 = L.dim[2].L == 1 ? 1 : L.dim[2].nshift;
    ncell = ns1 * ns2 * ns3;
    twl = ncell <= M * (M + 1);
    if (twl) {
      for (int q = t; q < ncell; q += TPM) {
        const int t3 = q % ns3, t2 = (q / ns3) % ns2, t1 = q / (ns3 * ns2);
        const int k1 = cell_of(L.dim[0], t1), k2 = cell_of(L.dim[1], t2), k3 = cell_of(L.dim[2], t3);
        C ww = cmul(tw[L.dim[0].tw_off + (j1 * k1) % L.L[0]], tw[L.dim[1].tw_off + (j2 * k2) % L.L[1]]);
        twc[q] = cmul(ww, tw[L.dim[2].tw_off + (j3 * k3) % L.L[2]]);
      }
    }
  }
  __syncthreads();
  C ue[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int e = t + k * TPM, r = e / M, c = e % M;
    C h = cmk<C>(0.0, 0.0), s = cmk<C>(r == c ? 1.0 : 0.0, 0.0), u = cmk<C>(r == c ? 1.0 : 0.0, 0.0);
    if (valid && r < m && c < m) {
      if (H64) {
        h = hv[k];
        s = sv[k];
      } else {
        // regenerate: sum over band cells k of w^(j.k) A_k
        h = cmk<C>(0.0, 0.0);
        s = cmk<C>(0.0, 0.0);
#pragma unroll 4
        for (int q = 0; q < ncell; ++q) {
          const int t3 = q % ns3, t2 = (q / ns3) % ns2, t1 = q / (ns3 * ns2);
          const int k1 = cell_of(L.dim[0], t1), k2 = cell_of(L.dim[1], t2), k3 = cell_of(L.dim[2], t3);
          C ww;
          if (twl) {
            ww = twc[q];
          } else {
            ww = cmul(cmul(tw[L.dim[0].tw_off + (j1 * k1) % L.L[0]], tw[L.dim[1].tw_off + (j2 * k2) % L.L[1]]),
                      tw[L.dim[2].tw_off + (j3 * k3) % L.L[2]]);
          }
          const int64_t o = L.gen_off + ((int64_t)(k1 * L.L[1] + k2) * L.L[2] + k3) * m * m + r * m + c;
          h = cadd(h, cscale(ww, Hg[o]));
          s = cadd(s, cscale(ww, Sg[o]));
        }
      }
      if (!fresh) u = cmk<C>((double)uv[k].x, (double)uv[k].y);
    }
    if constexpr (Smem<R, M, G, true, WANTV>::HASF) {
      sh.A[g][r][c] = h;
      sh.B[g][r][c] = s;
      sh.U[g][r][c] = u;
    } else {
      hv[k] = h;
      sv[k] = s;
      ue[k] = u;
    }
  }
  if constexpr (!Smem<R, M, G, true, WANTV>::HASF) {
    __syncthreads();   // the twiddle cache in A is no longer read
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int e = t + k * TPM, r = e / M, c = e % M;
      sh.A[g][r][c] = hv[k];
      sh.B[g][r][c] = sv[k];
      sh.U[g][r][c] = ue[k];
    }
  }
  __syncthreads();
  // Rayleigh-Ritz pair: A <- U^H Hbar U, B <- U^H Sbar U (two fused passes)
  constexpr int NT = TileOf<W>::NT;
  int ti, tj;
  tile_coords<M, NT>(t, ti, tj);
  // X = (I + E)^-1/2, or the reduction's W: F where it exists, else U, dead
  // after the Rayleigh-Ritz products
  constexpr bool HASF = Smem<R, M, G, true, WANTV>::HASF;
  auto& Xm = xbuf(sh, g);
  // products on the matrix cores for one matrix per workgroup of size >= 16
  constexpr bool kMf = M >= 16 && G == 1;
  const MfTile<M> mft;
  if constexpr (kMf) {
    mf4 ar, ai, br, bi;
    if (mft.on) {
      mf_product<M, false>(mft, sh.A[g], sh.U[g], ar, ai);
      mf_product<M, false>(mft, sh.B[g], sh.U[g], br, bi);
    }
    __syncthreads();
    if (mft.on) {
      mf_store<M>(mft, sh.A[g], ar, ai, 0.0);
      mf_store<M>(mft, sh.B[g], br, bi, 0.0);
    }
    __syncthreads();
    if (mft.on) {
      mf_product<M, true>(mft, sh.U[g], sh.A[g], ar, ai);
      mf_product<M, true>(mft, sh.U[g], sh.B[g], br, bi);
    }
    __syncthreads();
    if (mft.on) {
      mf_store<M>(mft, sh.A[g], ar, ai, 0.0);
      mf_store<M>(mft, sh.B[g], br, bi, 0.0);
    }
    __syncthreads();
  } else {
    C p1[NT][NT], p2[NT][NT];
    mm_shared_right<M, NT>(sh.A[g], sh.B[g], sh.U[g], ti, tj, p1, p2);
    __syncthreads();
    store_tile<M, NT>(sh.A[g], ti, tj, p1);
    store_tile<M, NT>(sh.B[g], ti, tj, p2);
    __syncthreads();
    mm_shared_left_h<M, NT>(sh.U[g], sh.A[g], sh.B[g], ti, tj, p1, p2);
    __syncthreads();
    store_tile<M, NT>(sh.A[g], ti, tj, p1);
    store_tile<M, NT>(sh.B[g], ti, tj, p2);
    __syncthreads();
  }
  // B = I + E with E small when U is S-orthonormal to FP32 accuracy (E is
  // about kappa(Sbar) times the FP32 rounding): then
  // X = (I + E)^-1/2 = I - E/2 + 3/8 E^2 - 5/16 E^3 + 35/128 E^4 - 63/256 E^5
  // + O(E^6), summed by Horner's rule, and A <- X A X.  Otherwise Cholesky
  // reduction.
  R eloc = R(0);
  LHF_FOR_ENTRIES {
    const C b = sh.B[g][r][c];
    const R br = b.x - (r == c ? R(1) : R(0));
    eloc += br * br + b.y * b.y;
  }
  const R e2 = group_sum<W>(sh, g, t, eloc);
  // series degree: the first neglected term ||E||^(deg+1) stays below ~1e-16
  if (t == 0) sh.flag[g][3] = e2 <= R(1e-12) ? 2 : e2 <= R(1e-9) ? 3 : e2 <= R(1e-7) ? 4 : e2 <= R(4e-6) ? 5 : 0;
  __syncthreads();
  int deg = 0;
  bool series = true;
#pragma unroll
  for (int gg = 0; gg < G; ++gg) {
    series = series && sh.flag[gg][3] != 0;
    deg = max(deg, sh.flag[gg][3]);
  }
  // Z <- X Y + d I (X, Y, Z in LDS); when Z aliases X or Y (alias) every read
  // of the product precedes a barrier before the store
  auto prod_store = [&](const C (&X)[M][M + 1], const C (&Y)[M][M + 1], C (&Z)[M][M + 1], R d, bool alias) {
    if constexpr (kMf) {
      mf4 re, im;
      if (mft.on) mf_product<M, false>(mft, X, Y, re, im);
      if (alias) __syncthreads();
      if (mft.on) mf_store<M>(mft, Z, re, im, d);
    } else {
      C q[NT][NT];
      if (d != R(0)) mm_tile<M, NT, true>(X, Y, ti, tj, d, q); else mm_tile<M, NT, false>(X, Y, ti, tj, R(0), q);
      if (alias) __syncthreads();
      store_tile<M, NT>(Z, ti, tj, q);
    }
    __syncthreads();
  };
  if (series) {
    // coefficients of (1 + E)^-1/2 = sum_k cf(k) E^k
    auto cf = [](int k) -> R {
      return k == 0 ? R(1.0) : k == 1 ? R(-0.5) : k == 2 ? R(0.375) : k == 3 ? R(-0.3125)
             : k == 4 ? R(0.2734375) : R(-0.24609375);
    };
    // E in B; X <- cf_deg E + cf_(deg-1) I, then X <- E X + cf_k I for k = deg-2 .. 0
    LHF_FOR_ENTRIES {
      C ev = sh.B[g][r][c];
      if (r == c) ev.x -= R(1);
      sh.B[g][r][c] = ev;
      C f = cscale(ev, cf(deg));
      if (r == c) f.x += cf(deg - 1);
      Xm[r][c] = f;
    }
    __syncthreads();
#pragma unroll 1
    for (int h = deg - 2; h >= 0; --h) prod_store(sh.B[g], Xm, Xm, cf(h), true);
    if constexpr (WANTV) {
      // T <- A X into V, then B <- X T (E is dead), then A <- the Hermitian
      // part of B and V <- I
      prod_store(sh.A[g], Xm, sh.V[g], R(0), false);
      prod_store(Xm, sh.V[g], sh.B[g], R(0), false);
      LHF_FOR_ENTRIES {
        const C x = sh.B[g][r][c], y = sh.B[g][c][r];
        C s2 = cmk<C>(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
        if (r == c) s2.y = 0.0;
        sh.A[g][r][c] = s2;
        sh.V[g][r][c] = cmk<C>(r == c ? 1.0 : 0.0, 0.0);
      }
      __syncthreads();
    } else if constexpr (HASF) {
      // T <- A X into the dead U, then B <- X T (E is dead), then A <- the
      // Hermitian part of B
      prod_store(sh.A[g], Xm, sh.U[g], R(0), false);
      prod_store(Xm, sh.U[g], sh.B[g], R(0), false);
      LHF_FOR_ENTRIES {
        const C x = sh.B[g][r][c], y = sh.B[g][c][r];
        sh.A[g][r][c] = cmk<C>(0.5 * (x.x + y.x), r == c ? 0.0 : 0.5 * (x.y - y.y));
      }
      __syncthreads();
    } else {
      // X is in U: T <- A X into B (E is dead), A <- X T, then A <- its
      // Hermitian part
      prod_store(sh.A[g], Xm, sh.B[g], R(0), false);
      prod_store(Xm, sh.B[g], sh.A[g], R(0), false);
      C hs[W];
      LHF_FOR_ENTRIES {
        const C x = sh.A[g][r][c], y = sh.A[g][c][r];
        hs[k] = cmk<C>(0.5 * (x.x + y.x), r == c ? 0.0 : 0.5 * (x.y - y.y));
      }
      __syncthreads();
      LHF_FOR_ENTRIES { sh.A[g][r][c] = hs[k]; }
      __syncthreads();
    }
  } else {
    chol_reduce<W, !HASF>(sh, g, t);
  }
  const int cur = jacobi<W, R, M, G, true, WANTV, WANTV>(sh, g, t, maxsw, tol);
  eig_rank(sh, g, t, m, cur);
  C vfin[NT][NT];
  if constexpr (WANTV) {
    if (series) {
      // A <- X V
      C p[NT][NT];
      mm_tile<M, NT, false>(sh.F[g], sh.V[g], ti, tj, R(0), p);
      store_tile<M, NT>(sh.A[g], ti, tj, p);
      __syncthreads();
    } else {
      backsub_vectors<W>(sh, g, t);
    }
    mm_tile<M, NT, false>(sh.U[g], sh.A[g], ti, tj, R(0), vfin);
  }
  if (!valid) return;
  const int64_t wb = L.w_off + (int64_t)blk * m, wc = L.w_off + (int64_t)cblk * m;
  if (t < m) {
    w[wb + sh.rank[g][t]] = sh.lam[g][t];
    if (cblk != blk) w[wc + sh.rank[g][t]] = sh.lam[g][t];
  }
  if constexpr (WANTV) {
    const int64_t cb0 = L.gen_off + (int64_t)cblk * m * m;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const int r = ti + a * (M / NT), c = tj + b * (M / NT);
        if (r < m && c < m) {
          Vout[base + r * m + sh.rank[g][c]] = vfin[a][b];
          if (cblk != blk) Vout[cb0 + r * m + sh.rank[g][c]] = cconj(vfin[a][b]);
        }
      }
  }
  if (t == 0) {
    const int st = sh.flag[g][1] ? -2 : (sh.flag[g][0] ? sh.flag[g][0] : (sh.flag[g][2] ? 0 : -1));
    info[L.blk_off + blk] = st;
    if (cblk != blk) info[L.blk_off + cblk] = st;
  }
}

template <typename R, int M, int W, typename CIN>
hipError_t launch_heev_mw(const lhf_plan_s* p, int vmode, const void* Hb, const void* Sb, double* w, void* V,
                          int32_t* info, int maxsw, R tol, hipStream_t s) {
  typedef typename Cx<R>::T C;
  const int cls = M == 4 ? 0 : M == 8 ? 1 : M == 16 ? 2 : 3;
  const int nc = p->ncanon[cls];
  const int2* canon = p->d_canon[cls];
  const dim3 grid((nc + Shape<M, W>::G - 1) / Shape<M, W>::G), block(Shape<M, W>::THREADS);
  const CIN* h = (const CIN*)Hb;
  const CIN* sm = (const CIN*)Sb;
  if (vmode == 0)
    hipLaunchKernelGGL((heev_kernel<R, M, 0, W, CIN>), grid, block, 0, s, p->d_lat, canon, nc, h, sm, w, (C*)V,
                       info, maxsw, tol);
  else if (vmode == 1)
    hipLaunchKernelGGL((heev_kernel<R, M, 1, W, CIN>), grid, block, 0, s, p->d_lat, canon, nc, h, sm, w, (C*)V,
                       info, maxsw, tol);
  else
    hipLaunchKernelGGL((heev_kernel<R, M, 2, W, CIN>), grid, block, 0, s, p->d_lat, canon, nc, h, sm, w, (C*)V,
                       info, maxsw, tol);
  return hipGetLastError();
}

// One launch for the class of size M, in the wide layout when the plan
// chose it for that class.
// (in64: the FP32 solve reads complex128 blocks)
template <typename R, int M>
hipError_t launch_heev_m(const lhf_plan_s* p, int vmode, const void* Hb, const void* Sb, double* w, void* V,
                         int32_t* info, int maxsw, R tol, hipStream_t s, bool in64 = false) {
  typedef typename Cx<R>::T C;
  const int cls = M == 4 ? 0 : M == 8 ? 1 : M == 16 ? 2 : 3;
  if (p->ncanon[cls] == 0) return hipSuccess;
  if constexpr (sizeof(R) == 4) {
    if (in64) {
      if (p->heev_wide[cls]) return launch_heev_mw<R, M, 1, double2>(p, vmode, Hb, Sb, w, V, info, maxsw, tol, s);
      return launch_heev_mw<R, M, 4, double2>(p, vmode, Hb, Sb, w, V, info, maxsw, tol, s);
    }
  }
  if (p->heev_wide[cls]) return launch_heev_mw<R, M, 1, C>(p, vmode, Hb, Sb, w, V, info, maxsw, tol, s);
  return launch_heev_mw<R, M, 4, C>(p, vmode, Hb, Sb, w, V, info, maxsw, tol, s);
}

template <int M, int W>
hipError_t launch_refine_mw(const lhf_plan_s* p, bool wantv, const void* H64, const void* S64, const double* Hg,
                            const double* Sg, const float2* U, const int32_t* info32, double* w, void* V,
                            int32_t* info, hipStream_t s) {
  const int cls = M == 4 ? 0 : M == 8 ? 1 : M == 16 ? 2 : 3;
  const int nc = p->ncanon[cls];
  const int2* canon = p->d_canon[cls];
  const dim3 grid((nc + Shape<M, W>::G - 1) / Shape<M, W>::G), block(Shape<M, W>::THREADS);
  // eigenvalues only: stop at an off-diagonal norm of 1e-11 of the norm (the
  // eigenvalue error is at most that, even for a degenerate pair); with
  // vectors: 4 M eps
  const double tol = wantv ? 4.0 * M * 1.1102230246251565e-16 : 1e-11;
  if (wantv)
    hipLaunchKernelGGL((refine_kernel<M, true, W>), grid, block, 0, s, p->d_lat, canon, nc, p->d_tw64,
                       (const double2*)H64, (const double2*)S64, Hg, Sg, U, info32, w, (double2*)V, info, 30, tol);
  else
    hipLaunchKernelGGL((refine_kernel<M, false, W>), grid, block, 0, s, p->d_lat, canon, nc, p->d_tw64,
                       (const double2*)H64, (const double2*)S64, Hg, Sg, U, info32, w, (double2*)V, info, 30, tol);
  return hipGetLastError();
}

template <int M>
hipError_t launch_refine_m(const lhf_plan_s* p, bool wantv, const void* H64, const void* S64, const double* Hg,
                           const double* Sg, const float2* U, const int32_t* info32, double* w, void* V,
                           int32_t* info, hipStream_t s) {
  const int cls = M == 4 ? 0 : M == 8 ? 1 : M == 16 ? 2 : 3;
  if (p->ncanon[cls] == 0) return hipSuccess;
  if (p->heev_wide[cls]) return launch_refine_mw<M, 1>(p, wantv, H64, S64, Hg, Sg, U, info32, w, V, info, s);
  return launch_refine_mw<M, 4>(p, wantv, H64, S64, Hg, Sg, U, info32, w, V, info, s);
}

}  // namespace

int heev_class(int m0) { return m0 <= 4 ? 0 : m0 <= 8 ? 1 : m0 <= 16 ? 2 : 3; }

// One launch per size class M = 4, 8, 16, 32 that has blocks; in the mixed
// pipeline all FP32 solves run before the FP64 refinements.
hipError_t launch_heev(const lhf_plan_s* p, uint32_t flags, const void* Hbar, const void* Sbar,
                       const void* Hbar64, const void* Sbar64, const double* Hgen64, const double* Sgen64,
                       double* w, void* V, int32_t* info, float2* U, int32_t* info32, hipStream_t s) {
  const bool wantv = (flags & LHF_HEEV_VECTORS) != 0;
  const bool refine = p->prec == LHF_PREC_MIXED && (flags & LHF_HEEV_REFINE_FP64);
  hipError_t e = hipSuccess;
  if (p->prec == LHF_PREC_FP64) {
    const int vm = wantv ? 1 : 0;
    const double eps = 1.1102230246251565e-16;
    if (e == hipSuccess) e = launch_heev_m<double, 4>(p, vm, Hbar, Sbar, w, V, info, 30, 16 * eps, s);
    if (e == hipSuccess) e = launch_heev_m<double, 8>(p, vm, Hbar, Sbar, w, V, info, 30, 32 * eps, s);
    if (e == hipSuccess) e = launch_heev_m<double, 16>(p, vm, Hbar, Sbar, w, V, info, 30, 64 * eps, s);
    if (e == hipSuccess) e = launch_heev_m<double, 32>(p, vm, Hbar, Sbar, w, V, info, 30, 128 * eps, s);
    return e;
  }
  // mixed: FP32 solve, then FP64 refinement; with complex128 blocks, the
  // classes the plan marks take the FP64 solve alone instead
  const bool any64 = refine && Hbar64 && !(flags & LHF_HEEV_FP32_SOLVE);
  const bool f64[4] = {any64 && p->heev_fp64[0], any64 && p->heev_fp64[1], any64 && p->heev_fp64[2],
                       any64 && p->heev_fp64[3]};
  if (f64[0] || f64[1] || f64[2] || f64[3]) {
    const int vm = wantv ? 1 : 0;
    const double eps = 1.1102230246251565e-16;
    if (e == hipSuccess && f64[0]) e = launch_heev_m<double, 4>(p, vm, Hbar64, Sbar64, w, V, info, 30, 16 * eps, s);
    if (e == hipSuccess && f64[1]) e = launch_heev_m<double, 8>(p, vm, Hbar64, Sbar64, w, V, info, 30, 32 * eps, s);
    if (e == hipSuccess && f64[2]) e = launch_heev_m<double, 16>(p, vm, Hbar64, Sbar64, w, V, info, 30, 64 * eps, s);
    if (e == hipSuccess && f64[3]) e = launch_heev_m<double, 32>(p, vm, Hbar64, Sbar64, w, V, info, 30, 128 * eps, s);
  }
  const int vm = refine ? 2 : (wantv ? 1 : 0);
  void* vdst = refine ? (void*)U : V;
  int32_t* i32 = refine ? info32 : info;
  const float eps = 5.9604645e-08f * (float)p->tol32_scale;
  // without complex64 blocks the FP32 solve reads the complex128 ones
  const bool in64 = refine && !Hbar;
  const void* h32 = in64 ? Hbar64 : Hbar;
  const void* s32 = in64 ? Sbar64 : Sbar;
  if (e == hipSuccess && !f64[0]) e = launch_heev_m<float, 4>(p, vm, h32, s32, w, vdst, i32, 20, 16 * eps, s, in64);
  if (e == hipSuccess && !f64[1]) e = launch_heev_m<float, 8>(p, vm, h32, s32, w, vdst, i32, 20, 32 * eps, s, in64);
  if (e == hipSuccess && !f64[2]) e = launch_heev_m<float, 16>(p, vm, h32, s32, w, vdst, i32, 20, 64 * eps, s, in64);
  if (e == hipSuccess && !f64[3]) e = launch_heev_m<float, 32>(p, vm, h32, s32, w, vdst, i32, 20, 128 * eps, s, in64);
  if (e != hipSuccess || !refine) return e;
  if (e == hipSuccess && !f64[0]) e = launch_refine_m<4>(p, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  if (e == hipSuccess && !f64[1]) e = launch_refine_m<8>(p, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  if (e == hipSuccess && !f64[2]) e = launch_refine_m<16>(p, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  if (e == hipSuccess && !f64[3]) e = launch_refine_m<32>(p, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  return e;
}

}  // namespace lhf
