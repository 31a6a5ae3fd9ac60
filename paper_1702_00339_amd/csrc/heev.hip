// Batched generalized Hermitian eigensolver for the Fourier blocks
// (eq. HF-FSpace-Block; union of block spectra, Prop. 5.1 eq. lambdAbc).
//
// Per block j, in LDS, one thread per matrix entry:
//   1. Cholesky  Sbar = C C^H (right-looking, one column per step);
//   2. reduction A = C^-1 Hbar C^-H by two forward substitutions;
//   3. cyclic Jacobi sweeps with the parallel round-robin ordering: in each of
//      the M-1 rounds of a sweep, M/2 disjoint index pairs (p, q) are rotated
//      at once by J = [[c, s b/|b|], [-s conj(b)/|b|, c]] (b = A_pq; c, s from
//      the stable tangent formula), every entry updated from its 2 x 2 block;
//      sweeps stop when the off-diagonal Frobenius norm is below
//      4 M eps times the norm of A;
//   4. eigenvalues sorted ascending; eigenvectors back-transformed C^-H V.
// Blocks j and -j are complex conjugates (real symmetric generators), so each
// conjugate pair is solved once and written twice.
//
// Refinement (mixed precision): the FP32 solve leaves eigenvectors U; in FP64
// the block pair is rebuilt accurately (from complex128 Fourier blocks, or
// regenerated from the FP64 generator band) and the Rayleigh-Ritz pair
// (U^H Hbar U, U^H Sbar U) -- nearly diagonal -- is solved by the same FP64
// steps, which converge in one or two sweeps.  If the FP32 solve failed for a
// block, U = I and the FP64 solve does the whole work.
//
// Sizes: M in {4, 8, 16, 32} >= m0 (padded rows/columns are decoupled: unit
// overlap, zero Hamiltonian, never written out); M = 4 packs 4 blocks per
// workgroup.
#include <algorithm>

#include "plan.h"

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

__device__ __forceinline__ int partner_of(int x, int s, int M) {
  const int m = M - 1;
  if (x == 0) return 1 + s;
  const int u = x - 1;
  if (u == s) return 0;
  int v = (2 * s - u) % m;
  if (v < 0) v += m;
  return 1 + v;
}

__device__ __forceinline__ int conj_block(const LatDev& L, int b) {
  const int k3 = b % L.L[2];
  const int k2 = (b / L.L[2]) % L.L[1];
  const int k1 = b / (L.L[2] * L.L[1]);
  const int c1 = k1 ? L.L[0] - k1 : 0, c2 = k2 ? L.L[1] - k2 : 0, c3 = k3 ? L.L[2] - k3 : 0;
  return (c1 * L.L[1] + c2) * L.L[2] + c3;
}

template <typename R, int M, int G>
struct Shared {
  typedef typename Cx<R>::T C;
  C A[G][M][M + 1];
  C B[G][M][M + 1];
  C V[G][M][M + 1];
  C U[G][M][M + 1];
  R jd[G][M];        // J[x][x]
  C jo[G][M];        // J[partner(x)][x]
  R dnew[G][M];      // rotated diagonal
  R red[G * M * M];
  R lam[G][M];
  int rank[G][M];
  int flag[G][4];    // 0: Cholesky failure column, 1: non-finite, 2: converged
};

// Group-wide sum of one value per thread (all threads of the workgroup call it).
template <typename R, int M, int G>
__device__ R group_sum(Shared<R, M, G>& sh, int g, int loc, R v) {
  constexpr int MM = M * M;
  sh.red[g * MM + loc] = v;
  __syncthreads();
#pragma unroll 1
  for (int st = MM / 2; st > 0; st >>= 1) {
    if (loc < st) sh.red[g * MM + loc] += sh.red[g * MM + loc + st];
    __syncthreads();
  }
  R r = sh.red[g * MM];
  __syncthreads();
  return r;
}

// Cholesky of B, reduction of A, Jacobi on A (with V if WANTV).  Returns the
// number of sweeps; flags in sh.flag.
template <typename R, int M, int G, bool WANTV>
__device__ void solve_pair(Shared<R, M, G>& sh, int g, int r, int c, int maxsw, R tol) {
  typedef typename Cx<R>::T C;
  const int loc = r * M + c;
  // 1. Cholesky B = L L^H (lower triangle)
#pragma unroll 1
  for (int j = 0; j < M; ++j) {
    if (r == j && c == j) {
      R d = sh.B[g][j][j].x;
      if (!(d > R(0)) && sh.flag[g][0] == 0) sh.flag[g][0] = j + 1;
      sh.B[g][j][j] = cmk<C>(sqrt(d > R(0) ? d : R(1)), R(0));
    }
    __syncthreads();
    if (c == j && r > j) sh.B[g][r][j] = cscale(sh.B[g][r][j], R(1) / sh.B[g][j][j].x);
    __syncthreads();
    if (r > j && c > j && c <= r) sh.B[g][r][c] = csub(sh.B[g][r][c], cmul(sh.B[g][r][j], cconj(sh.B[g][c][j])));
    __syncthreads();
  }
  // 2. A <- L^-1 A, then A <- L^-1 A^H (= L^-1 H L^-H, Hermitian)
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll 1
    for (int j = 0; j < M; ++j) {
      if (r == j) sh.A[g][j][c] = cscale(sh.A[g][j][c], R(1) / sh.B[g][j][j].x);
      __syncthreads();
      if (r > j) sh.A[g][r][c] = csub(sh.A[g][r][c], cmul(sh.B[g][r][j], sh.A[g][j][c]));
      __syncthreads();
    }
    C t = cconj(sh.A[g][c][r]);
    __syncthreads();
    sh.A[g][r][c] = t;
    __syncthreads();
  }
  {
    C t = sh.A[g][r][c], u = sh.A[g][c][r];
    __syncthreads();
    C s = cmk<C>(R(0.5) * (t.x + u.x), R(0.5) * (t.y - u.y));
    if (r == c) s.y = R(0);
    sh.A[g][r][c] = s;
    if (WANTV) sh.V[g][r][c] = cmk<C>(r == c ? R(1) : R(0), R(0));
    __syncthreads();
  }
  // 3. Jacobi sweeps
  const R nrm2 = group_sum<R, M, G>(sh, g, loc, sh.A[g][r][c].x * sh.A[g][r][c].x + sh.A[g][r][c].y * sh.A[g][r][c].y);
#pragma unroll 1
  for (int sw = 0;; ++sw) {
    {
      // every group tests its own convergence; the workgroup stops when all
      // groups have converged (barriers stay uniform); converged groups keep
      // rotating by near-identity rotations meanwhile
      const C a = sh.A[g][r][c];
      const R off = group_sum<R, M, G>(sh, g, loc, r != c ? a.x * a.x + a.y * a.y : R(0));
      if (r == 0 && c == 0) sh.flag[g][2] = (off <= tol * tol * nrm2) ? 1 : 0;
      __syncthreads();
      bool all = true;
#pragma unroll
      for (int gg = 0; gg < G; ++gg) all = all && sh.flag[gg][2] != 0;
      __syncthreads();
      if (all || sw == maxsw) break;
    }
#pragma unroll 1
    for (int s = 0; s < M - 1; ++s) {
      // rotation parameters, one thread per pair (p < q)
      if (r < M && c == 0) {
        const int p = r, q = partner_of(r, s, M);
        if (p < q) {
          const R app = sh.A[g][p][p].x, aqq = sh.A[g][q][q].x;
          const C b = sh.A[g][p][q];
          const R ab = sqrt(b.x * b.x + b.y * b.y);
          if (ab > R(0)) {
            const R tau = (aqq - app) / (R(2) * ab);
            const R t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + sqrt(R(1) + tau * tau));
            const R cs = R(1) / sqrt(R(1) + t * t);
            const R sn = t * cs;
            const C ph = cscale(b, R(1) / ab);          // b / |b|
            sh.jd[g][p] = cs; sh.jd[g][q] = cs;
            sh.jo[g][p] = cscale(cconj(ph), -sn);       // J[q][p]
            sh.jo[g][q] = cscale(ph, sn);               // J[p][q]
            sh.dnew[g][p] = app - t * ab;
            sh.dnew[g][q] = aqq + t * ab;
          } else {
            sh.jd[g][p] = R(1); sh.jd[g][q] = R(1);
            sh.jo[g][p] = cmk<C>(R(0), R(0)); sh.jo[g][q] = cmk<C>(R(0), R(0));
            sh.dnew[g][p] = app; sh.dnew[g][q] = aqq;
          }
        }
      }
      __syncthreads();
      const int rb = partner_of(r, s, M), cb = partner_of(c, s, M);
      C na;
      if (r == c) {
        na = cmk<C>(sh.dnew[g][r], R(0));
      } else if (c == rb) {
        na = cmk<C>(R(0), R(0));
      } else {
        const R jrr = sh.jd[g][r], jcc = sh.jd[g][c];
        const C jbr = sh.jo[g][r], jbc = sh.jo[g][c];
        // (A J)[x][c] for x in {r, rb}
        const C x0 = cadd(cscale(sh.A[g][r][c], jcc), cmul(sh.A[g][r][cb], jbc));
        const C x1 = cadd(cscale(sh.A[g][rb][c], jcc), cmul(sh.A[g][rb][cb], jbc));
        na = cadd(cscale(x0, jrr), cmulc(jbr, x1));
      }
      C nv;
      if (WANTV) nv = cadd(cscale(sh.V[g][r][c], sh.jd[g][c]), cmul(sh.V[g][r][cb], sh.jo[g][c]));
      __syncthreads();
      sh.A[g][r][c] = na;
      if (WANTV) sh.V[g][r][c] = nv;
      __syncthreads();
    }
  }
}

// Eigenvalues, ranks and (optionally) back-transformed eigenvectors.
template <typename R, int M, int G, bool WANTV>
__device__ void finish(Shared<R, M, G>& sh, int g, int r, int c, int m) {
  typedef typename Cx<R>::T C;
  if (c == 0) sh.lam[g][r] = sh.A[g][r][r].x;
  __syncthreads();
  if (c == 0 && r < m) {
    const R lr = sh.lam[g][r];
    int k = 0;
    for (int y = 0; y < m; ++y) {
      const R ly = sh.lam[g][y];
      k += (ly < lr || (ly == lr && y < r)) ? 1 : 0;
    }
    sh.rank[g][r] = k;
  }
  if (WANTV) {
    // V <- L^-H V
#pragma unroll 1
    for (int j = M - 1; j >= 0; --j) {
      __syncthreads();
      if (r == j) sh.V[g][j][c] = cscale(sh.V[g][j][c], R(1) / sh.B[g][j][j].x);
      __syncthreads();
      if (r < j) sh.V[g][r][c] = csub(sh.V[g][r][c], cmulc(sh.B[g][j][r], sh.V[g][j][c]));
    }
  }
  __syncthreads();
}

// MODE 0: solve from Fourier blocks of precision R.  VMODE: 0 none, 1 write
// vectors to V (caller), 2 write vectors to U (FP32 workspace for refinement).
template <typename R, int M, int G, int VMODE>
__global__ void __launch_bounds__(G * M * M) heev_kernel(const LatDev* __restrict__ lats, int li,
                                                         const typename Cx<R>::T* __restrict__ Hb,
                                                         const typename Cx<R>::T* __restrict__ Sb,
                                                         double* __restrict__ w,
                                                         typename Cx<R>::T* __restrict__ Vout,
                                                         int32_t* __restrict__ info, int maxsw, R tol) {
  typedef typename Cx<R>::T C;
  constexpr bool WANTV = VMODE != 0;
  __shared__ Shared<R, M, G> sh;
  const LatDev& L = lats[li];
  const int m = L.m0;
  const int tid = threadIdx.x;
  const int g = tid / (M * M), r = (tid / M) % M, c = tid % M;
  const int blk = blockIdx.x * G + g;
  const bool valid = blk < L.nblk;
  const int cblk = valid ? conj_block(L, blk) : 0;
  const bool writer = valid && cblk >= blk;
  if (G == 1 && !writer) return;   // uniform over the workgroup
  const int64_t base = L.gen_off + (int64_t)(valid ? blk : 0) * m * m;
  if (c == 0 && r < 4) sh.flag[g][r] = 0;
  __syncthreads();
  C a, b;
  if (valid && r < m && c < m) {
    a = Hb[base + r * m + c];
    b = Sb[base + r * m + c];
  } else {
    a = cmk<C>(R(0), R(0));
    b = cmk<C>(r == c ? R(1) : R(0), R(0));
  }
  if (!(isfinite(a.x) && isfinite(a.y) && isfinite(b.x) && isfinite(b.y))) {
    sh.flag[g][1] = 1;
    a = cmk<C>(R(0), R(0));
    b = cmk<C>(r == c ? R(1) : R(0), R(0));
  }
  sh.A[g][r][c] = a;
  sh.B[g][r][c] = b;
  __syncthreads();
  solve_pair<R, M, G, WANTV>(sh, g, r, c, maxsw, tol);
  finish<R, M, G, WANTV>(sh, g, r, c, m);
  if (!writer) return;   // no barrier follows
  const int64_t wb = L.w_off + (int64_t)blk * m, wc = L.w_off + (int64_t)cblk * m;
  if (c == 0 && r < m) {
    const double lv = (double)sh.lam[g][r];
    w[wb + sh.rank[g][r]] = lv;
    if (cblk != blk) w[wc + sh.rank[g][r]] = lv;
  }
  if (WANTV && r < m && c < m) {
    const C v = sh.V[g][r][c];
    const int64_t cb0 = L.gen_off + (int64_t)cblk * m * m;
    Vout[base + r * m + sh.rank[g][c]] = v;
    if (cblk != blk) Vout[cb0 + r * m + sh.rank[g][c]] = cconj(v);
  }
  if (r == 0 && c == 0) {
    int st = sh.flag[g][1] ? -2 : (sh.flag[g][0] ? sh.flag[g][0] : (sh.flag[g][2] ? 0 : -1));
    info[L.blk_off + blk] = st;
    if (cblk != blk) info[L.blk_off + cblk] = st;
  }
}

// Refinement in FP64 from FP32 eigenvectors U (layout [blk][row][col]).
// Blocks from H64/S64 (complex128) or regenerated from the FP64 generator band.
template <int M, int G, bool WANTV>
__global__ void __launch_bounds__(G * M * M) refine_kernel(const LatDev* __restrict__ lats, int li,
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
  __shared__ Shared<R, M, G> sh;
  const LatDev& L = lats[li];
  const int m = L.m0;
  const int tid = threadIdx.x;
  const int g = tid / (M * M), r = (tid / M) % M, c = tid % M;
  const int blk = blockIdx.x * G + g;
  const bool valid = blk < L.nblk;
  const int cblk = valid ? conj_block(L, blk) : 0;
  const bool writer = valid && cblk >= blk;
  if (G == 1 && !writer) return;
  const int64_t base = L.gen_off + (int64_t)(valid ? blk : 0) * m * m;
  if (c == 0 && r < 4) sh.flag[g][r] = 0;
  __syncthreads();
  C h = cmk<C>(0.0, 0.0), s = cmk<C>(r == c ? 1.0 : 0.0, 0.0);
  if (valid && r < m && c < m) {
    if (H64) {
      h = H64[base + r * m + c];
      s = S64[base + r * m + c];
    } else {
      // regenerate: sum over band cells k of w^(j.k) A_k
      const int j3 = blk % L.L[2], j2 = (blk / L.L[2]) % L.L[1], j1 = blk / (L.L[2] * L.L[1]);
      auto cell_of = [&](const DimDev& D, int t) -> int {
        if (D.full) return t;
        const int k = t - D.L0;
        return k < 0 ? k + D.L : k;
      };
      const int ns1 = L.dim[0].L == 1 ? 1 : L.dim[0].nshift;
      const int ns2 = L.dim[1].L == 1 ? 1 : L.dim[1].nshift;
      const int ns3 = L.dim[2].L == 1 ? 1 : L.dim[2].nshift;
      C hs = cmk<C>(0.0, 0.0), ss = cmk<C>(0.0, 0.0);
      for (int t1 = 0; t1 < ns1; ++t1)
        for (int t2 = 0; t2 < ns2; ++t2)
          for (int t3 = 0; t3 < ns3; ++t3) {
            const int k1 = cell_of(L.dim[0], t1), k2 = cell_of(L.dim[1], t2), k3 = cell_of(L.dim[2], t3);
            const C w1 = tw[L.dim[0].tw_off + (int)(((int64_t)j1 * k1) % L.L[0])];
            const C w2 = tw[L.dim[1].tw_off + (int)(((int64_t)j2 * k2) % L.L[1])];
            const C w3 = tw[L.dim[2].tw_off + (int)(((int64_t)j3 * k3) % L.L[2])];
            const C ww = cmul(cmul(w1, w2), w3);
            const int64_t cell = ((int64_t)k1 * L.L[1] + k2) * L.L[2] + k3;
            const int64_t o = L.gen_off + cell * m * m + r * m + c;
            hs = cadd(hs, cscale(ww, Hg[o]));
            ss = cadd(ss, cscale(ww, Sg[o]));
          }
      h = hs;
      s = ss;
    }
  }
  const bool fresh = !valid || info32[L.blk_off + blk] != 0;
  C u = cmk<C>(r == c ? 1.0 : 0.0, 0.0);
  if (!fresh && r < m && c < m) {
    const float2 uf = U32[base + r * m + c];
    u = cmk<C>((double)uf.x, (double)uf.y);
  }
  sh.A[g][r][c] = h;
  sh.B[g][r][c] = s;
  sh.U[g][r][c] = u;
  __syncthreads();
  // Rayleigh-Ritz pair: A <- U^H Hbar U, B <- U^H Sbar U
#pragma unroll 1
  for (int which = 0; which < 2; ++which) {
    C acc = cmk<C>(0.0, 0.0);
    for (int k = 0; k < M; ++k) acc = cadd(acc, cmul(which == 0 ? sh.A[g][r][k] : sh.B[g][r][k], sh.U[g][k][c]));
    sh.V[g][r][c] = acc;
    __syncthreads();
    C acc2 = cmk<C>(0.0, 0.0);
    for (int k = 0; k < M; ++k) acc2 = cadd(acc2, cmulc(sh.U[g][k][r], sh.V[g][k][c]));
    __syncthreads();
    if (which == 0) sh.A[g][r][c] = acc2; else sh.B[g][r][c] = acc2;
    __syncthreads();
  }
  solve_pair<R, M, G, WANTV>(sh, g, r, c, maxsw, tol);
  finish<R, M, G, WANTV>(sh, g, r, c, m);
  C vfin = cmk<C>(0.0, 0.0);
  if (WANTV) {
    for (int k = 0; k < M; ++k) vfin = cadd(vfin, cmul(sh.U[g][r][k], sh.V[g][k][c]));
  }
  if (!writer) return;
  const int64_t wb = L.w_off + (int64_t)blk * m, wc = L.w_off + (int64_t)cblk * m;
  if (c == 0 && r < m) {
    w[wb + sh.rank[g][r]] = sh.lam[g][r];
    if (cblk != blk) w[wc + sh.rank[g][r]] = sh.lam[g][r];
  }
  if (WANTV && r < m && c < m) {
    const int64_t cb0 = L.gen_off + (int64_t)cblk * m * m;
    Vout[base + r * m + sh.rank[g][c]] = vfin;
    if (cblk != blk) Vout[cb0 + r * m + sh.rank[g][c]] = cconj(vfin);
  }
  if (r == 0 && c == 0) {
    int st = sh.flag[g][1] ? -2 : (sh.flag[g][0] ? sh.flag[g][0] : (sh.flag[g][2] ? 0 : -1));
    info[L.blk_off + blk] = st;
    if (cblk != blk) info[L.blk_off + cblk] = st;
  }
}

template <typename R, int M, int G>
hipError_t launch_heev_m(const lhf_plan_s* p, int li, int vmode, const void* Hb, const void* Sb, double* w,
                         void* V, int32_t* info, int maxsw, R tol, hipStream_t s) {
  typedef typename Cx<R>::T C;
  const LatDev& L = p->lat[li];
  const dim3 grid((L.nblk + G - 1) / G), block(G * M * M);
  const C* h = (const C*)Hb;
  const C* sm = (const C*)Sb;
  if (vmode == 0)
    hipLaunchKernelGGL((heev_kernel<R, M, G, 0>), grid, block, 0, s, p->d_lat, li, h, sm, w, (C*)V, info, maxsw, tol);
  else if (vmode == 1)
    hipLaunchKernelGGL((heev_kernel<R, M, G, 1>), grid, block, 0, s, p->d_lat, li, h, sm, w, (C*)V, info, maxsw, tol);
  else
    hipLaunchKernelGGL((heev_kernel<R, M, G, 2>), grid, block, 0, s, p->d_lat, li, h, sm, w, (C*)V, info, maxsw, tol);
  return hipGetLastError();
}

template <int M, int G>
hipError_t launch_refine_m(const lhf_plan_s* p, int li, bool wantv, const void* H64, const void* S64,
                           const double* Hg, const double* Sg, const float2* U, const int32_t* info32,
                           double* w, void* V, int32_t* info, hipStream_t s) {
  const LatDev& L = p->lat[li];
  const dim3 grid((L.nblk + G - 1) / G), block(G * M * M);
  const double tol = 4.0 * M * 1.1102230246251565e-16;
  if (wantv)
    hipLaunchKernelGGL((refine_kernel<M, G, true>), grid, block, 0, s, p->d_lat, li, p->d_tw64,
                       (const double2*)H64, (const double2*)S64, Hg, Sg, U, info32, w, (double2*)V, info, 30, tol);
  else
    hipLaunchKernelGGL((refine_kernel<M, G, false>), grid, block, 0, s, p->d_lat, li, p->d_tw64,
                       (const double2*)H64, (const double2*)S64, Hg, Sg, U, info32, w, (double2*)V, info, 30, tol);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_heev(const lhf_plan_s* p, int li, uint32_t flags, const void* Hbar, const void* Sbar,
                       const void* Hbar64, const void* Sbar64, const double* Hgen64, const double* Sgen64,
                       double* w, void* V, int32_t* info, float2* U, int32_t* info32, hipStream_t s) {
  const LatDev& L = p->lat[li];
  const int m = L.m0;
  const bool wantv = (flags & LHF_HEEV_VECTORS) != 0;
  const bool refine = p->prec == LHF_PREC_MIXED && (flags & LHF_HEEV_REFINE_FP64);
  hipError_t e;
  if (p->prec == LHF_PREC_FP64) {
    const int vm = wantv ? 1 : 0;
    const double tol = 1.1102230246251565e-16;
    if (m <= 4) e = launch_heev_m<double, 4, 4>(p, li, vm, Hbar, Sbar, w, V, info, 30, 16 * tol, s);
    else if (m <= 8) e = launch_heev_m<double, 8, 1>(p, li, vm, Hbar, Sbar, w, V, info, 30, 32 * tol, s);
    else if (m <= 16) e = launch_heev_m<double, 16, 1>(p, li, vm, Hbar, Sbar, w, V, info, 30, 64 * tol, s);
    else e = launch_heev_m<double, 32, 1>(p, li, vm, Hbar, Sbar, w, V, info, 30, 128 * tol, s);
    return e;
  }
  // mixed: FP32 solve, then FP64 refinement
  const int vm = refine ? 2 : (wantv ? 1 : 0);
  void* vdst = refine ? (void*)U : V;
  int32_t* i32 = refine ? info32 : info;
  const float tol = 5.9604645e-08f;
  if (m <= 4) e = launch_heev_m<float, 4, 4>(p, li, vm, Hbar, Sbar, w, vdst, i32, 20, 16 * tol, s);
  else if (m <= 8) e = launch_heev_m<float, 8, 1>(p, li, vm, Hbar, Sbar, w, vdst, i32, 20, 32 * tol, s);
  else if (m <= 16) e = launch_heev_m<float, 16, 1>(p, li, vm, Hbar, Sbar, w, vdst, i32, 20, 64 * tol, s);
  else e = launch_heev_m<float, 32, 1>(p, li, vm, Hbar, Sbar, w, vdst, i32, 20, 128 * tol, s);
  if (e != hipSuccess || !refine) return e;
  if (m <= 4) return launch_refine_m<4, 4>(p, li, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  if (m <= 8) return launch_refine_m<8, 1>(p, li, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  if (m <= 16) return launch_refine_m<16, 1>(p, li, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
  return launch_refine_m<32, 1>(p, li, wantv, Hbar64, Sbar64, Hgen64, Sgen64, U, info32, w, V, info, s);
}

}  // namespace lhf
