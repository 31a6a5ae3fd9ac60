// Lowest k eigenpairs of a small dense real symmetric matrix (m <= kMaxSmall),
// in one workgroup: the Rayleigh-Ritz problem of the block LOBPCG that finds
// the lowest eigenpairs of the Dirichlet operators (Sec. 3; Remark 3.2).
//
//  1. Householder tridiagonalisation with the matrix in registers, column by
//     column: the kRrP lanes of group g (one DPP row) hold columns 2g and
//     2g + 1 at the rows of reversed index idx = m - 1 - r = gc + kRrP j.
//     Step h: the group owning column h forms the reflector
//     u = x + sign(x_0) |x| e_0 (x: column h below the diagonal; the new
//     coupling is -sign(x_0) |x|) and publishes u and beta = 1 / hh,
//     hh = u^T u / 2 = |x| (|x| + |x_0|); barrier; every group forms
//     p_c = beta sum_r A_rc u_r (A symmetric) for its two columns by DPP
//     all-reduces and publishes them; barrier; every group forms u^T p over
//     its rows by one more all-reduce and updates
//     A_rc -= u_r q_c + q_r u_c, q = p - (beta u^T p / 2) u; the wavefront
//     owning the next column runs its update at raised priority, so that its
//     reflector work overlaps the other wavefronts' updates.
//     Only rows and columns after h change: in reversed order those rows are
//     the first J = ceil((m - 1 - h) / kRrP) blocks, and the steps run in
//     phases of equal J compiled for that J, so a step touches J blocks only;
//     wavefronts without a column after h skip the step; inside the last
//     block u and p read zero at the rows up to h, and columns up to h see
//     u_c = q_c = 0, so the update needs no masks.  u and p are
//     double-buffered in LDS by the parity of h; the reflectors
//     (reversed, padded with zeros to whole blocks) and beta stay in LDS for
//     step 4.
//  2. Bisection on Sturm counts (csrc/sturm.h) for the lowest k eigenvalues
//     of the tridiagonal T on four wavefronts, P lanes (P as large as the
//     wavefronts allow) per eigenvalue, one point per lane per pass, on T
//     scaled by a power of two to norm below 1 (minors rescaled by 2^-+256
//     every eighth row; rows padded to a multiple of eight with a diagonal
//     beyond the interval and no coupling; each half block is read while the
//     other is counted), to a few ulps of the interval or of the norm.  The
//     points with count <= i form a prefix of the group's lanes; its length
//     (a ballot) gives the new interval, 1 / (P + 1) of the old one.
//  3. Inverse iteration on T for each eigenvalue, one lane per eigenvector,
//     kRrChunk at a time: T - lambda I = L D L^T (a pivot below eps |T| is
//     replaced by +-eps |T|), two solves from a fixed start vector, each
//     followed by Gram-Schmidt against the eigenvectors of the same tight
//     cluster (consecutive eigenvalues closer than kRrClusterTol |T|; a
//     vector's rank in its cluster, from ballots, orders the work) and
//     normalisation.  The recurrences carry their last value in registers and
//     read each block of eight rows before its first use; the normalisation
//     is folded into the next pass and, at the end, into a per-vector scale.
//     Vectors of eigenvalues farther apart are orthogonal to about
//     eps |T| / gap, which the caller's next orthonormalisation absorbs.
//  4. Back-transform z = H_0 H_1 ... H_(m-3) y, kRrVecLanes lanes per vector
//     in the reversed row order of step 1, reflectors applied from the last
//     (z -= beta u (u^T z)) out of LDS over their nonzero blocks only (phases
//     of equal block count, as in step 1), the next reflector read while the
//     current one is applied.
// Eigenvalues ascending in w, eigenvector i in column i of V (row-major, ldv).
#include <string>
#include <type_traits>

#include "dpp.h"
#include "plan.h"
#include "sturm.h"
#include "toeplitz.h"

namespace lhf {
namespace {

constexpr int kRrThreads = 1024;
constexpr int kRrP = 16;                               // lanes per column pair in step 1 (a DPP row)
constexpr int kRrCols = 2 * kRrThreads / kRrP;         // column slots (> m: the last one stays zero)
constexpr int kRrW = (kMaxSmall + kRrP - 1) / kRrP;    // rows per lane in step 1
constexpr int kRrRows = kRrW * kRrP;                   // rows padded to whole blocks
// reflector rows, each reflector padded to whole blocks of kRrP
constexpr int kRrRefl = kMaxSmall * (kMaxSmall - 1) / 2 + (kRrP - 1) * kMaxSmall;
constexpr int kRrBisWaves = 4;                         // wavefronts of step 2
constexpr int kRrChunk = 40;                           // eigenvectors per chunk in step 3
constexpr int kRrVecLanes = kRrP;                      // lanes per eigenvector in step 4 (step 1's row blocks)
constexpr int kRrVecPass = kRrThreads / kRrVecLanes;   // eigenvectors per pass of step 4
constexpr double kRrClusterTol = 1e-8;
static_assert(kRrCols > kMaxSmall, "one column slot per column and a zero slot");
static_assert(kRrRows % 8 == 0 && kRrRows >= kMaxSmall, "rows in blocks of eight");
static_assert(kMaxSmall <= kRrBisWaves * 64, "every eigenvalue has a lane");
static_assert(kMaxSmall <= 128, "cluster ranks from two ballots");
static_assert(kRrChunk <= 64, "one wavefront runs the inverse iterations");

// 1 / x for a normal x, to within a few ulps: the hardware estimate refined
// by two Newton steps.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

template <int N>
using IC = std::integral_constant<int, N>;
static_assert(kRrW == 7, "the dispatch below names every block count");
// F(IC<J>{}) for a block count 1 <= J <= kRrW known only at run time
#define RR_DISPATCH(J, F)                                                                                     \
  switch (J) {                                                                                                \
    case 1: F(IC<1>{}); break;   case 2: F(IC<2>{}); break;   case 3: F(IC<3>{}); break;                      \
    case 4: F(IC<4>{}); break;   case 5: F(IC<5>{}); break;   case 6: F(IC<6>{}); break;                      \
    case 7: F(IC<7>{}); break;   default: break;                                                              \
  }

__global__ void __launch_bounds__(kRrThreads) rr_syev_kernel(int m, int k, const double* __restrict__ A, int lda,
                                                             double* __restrict__ w, double* __restrict__ V,
                                                             int ldv) {
  __shared__ double ubuf[2][kRrCols], pbuf[2][kRrCols];
  __shared__ double Us[kRrRefl], bet[kMaxSmall];
  __shared__ double dd[kRrRows], ee[kRrRows + 1], lam[kMaxSmall], sv[kRrRows];
  __shared__ double2 de[kRrRows];
  __shared__ double xv[kRrChunk][kRrRows + 1], ivp[kRrChunk][kRrRows + 1], xsc[kRrChunk];
  __shared__ double red[3][kRrThreads / 64];
  __shared__ int rank_s[kMaxSmall], info[4];
  const int t = threadIdx.x, wv = t >> 6;
  auto add = [](double x, double y) { return x + y; };
  auto fmin_ = [](double x, double y) { return fmin(x, y); };
  auto fmax_ = [](double x, double y) { return fmax(x, y); };
  constexpr double eps = 1.1102230246251565e-16;
  for (int q = t; q < 2 * kRrCols; q += kRrThreads) {
    ubuf[q / kRrCols][q % kRrCols] = 0.0;
    pbuf[q / kRrCols][q % kRrCols] = 0.0;
  }
  __syncthreads();

  // ---- 1. tridiagonalisation ----
  // group g = t / kRrP (one DPP row) holds columns 2 g and 2 g + 1; lane gc of
  // the group the reversed rows idx = gc + kRrP j (row m - 1 - idx)
  const int g = t / kRrP, gc = t % kRrP;
  double a[2][kRrW];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int c = 2 * g + e;
#pragma unroll
    for (int j = 0; j < kRrW; ++j) {
      const int idx = gc + kRrP * j, r = m - 1 - idx;
      a[e][j] = (c < m && idx < m) ? 0.5 * (A[(int64_t)r * lda + c] + A[(int64_t)c * lda + r]) : 0.0;
    }
  }
  int offh = 0;   // start of reflector h in Us
  // steps hb .. he - 1, whose rows after h fill J blocks of kRrP
  auto tri_steps = [&](auto Jc, int hb, int he) {
    constexpr int J = decltype(Jc)::value;
#pragma unroll 1
    for (int h = hb; h < he; ++h) {
      const int bs = h & 1, nh = m - 1 - h;   // rows after h
      if (g == h / 2) {
        // blocks before the last lie wholly after row h + 1; the last block
        // holds row h + 1 (idx = nh - 1) and the rows up to h (idx >= nh)
        auto own = [&](double(&col)[kRrW]) {
          const int il = gc + kRrP * (J - 1);
          double x2a = 0.0, x2b = 0.0;
#pragma unroll
          for (int j = 0; j + 1 < J; ++j) {
            if (j & 1) x2b = fma(col[j], col[j], x2b);
            else x2a = fma(col[j], col[j], x2a);
          }
          const double vl = col[J - 1];
          double al = il == nh - 1 ? vl : 0.0;
          double x2 = (il < nh - 1 ? vl * vl : 0.0) + (x2a + x2b);
          lane_reduce2<kRrP>(x2, al, add);
          const double nrm = sqrt(al * al + x2);
          const double sg = al >= 0.0 ? 1.0 : -1.0;
          if (x2 > 0.0) {   // the same on every lane of the group
#pragma unroll
            for (int j = 0; j + 1 < J; ++j) {
              const int idx = gc + kRrP * j;
              ubuf[bs][idx] = col[j];
              Us[offh + idx] = col[j];
            }
            const double uv = il < nh ? (il == nh - 1 ? al + sg * nrm : vl) : 0.0;
            ubuf[bs][il] = uv;
            Us[offh + il] = uv;
            if (gc == 0) {
              bet[h] = recip(nrm * (nrm + fabs(al)));
              ee[h] = -sg * nrm;
            }
          } else {          // column already reduced: no reflector
#pragma unroll
            for (int j = 0; j < J; ++j) {
              const int idx = gc + kRrP * j;
              ubuf[bs][idx] = 0.0;
              Us[offh + idx] = 0.0;
            }
            if (gc == 0) {
              bet[h] = 0.0;
              ee[h] = al;
            }
          }
          if (il >= nh) pbuf[bs][il] = 0.0;   // rows up to h: p reads zero there
        };
        if (h & 1) own(a[1]);
        else own(a[0]);
      }
      __builtin_amdgcn_s_setprio(0);
      __syncthreads();
      const double beta = bet[h];
      const bool refl = beta != 0.0;                       // the same for every thread
      const bool wlive = 8 * wv + 7 > h && 8 * wv < m;     // the wavefront holds a column in (h, m)
      bool colok[2];
      int ci[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int c = 2 * g + e;
        colok[e] = c > h && c < m;
        ci[e] = colok[e] ? m - 1 - c : kRrCols - 1;        // column's reversed slot; the zero slot otherwise
      }
      double ur[J], pc[2] = {0.0, 0.0}, uc[2] = {0.0, 0.0};
      if (refl && wlive) {
#pragma unroll
        for (int j = 0; j < J; ++j) ur[j] = ubuf[bs][gc + kRrP * j];
        uc[0] = ubuf[bs][ci[0]];
        uc[1] = ubuf[bs][ci[1]];
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          s0 = fma(a[0][j], ur[j], s0);
          s1 = fma(a[1][j], ur[j], s1);
        }
        lane_reduce2<kRrP>(s0, s1, add);
        pc[0] = beta * s0;
        pc[1] = beta * s1;
        if (gc == 0 && colok[0]) pbuf[bs][ci[0]] = pc[0];
        if (gc == 0 && colok[1]) pbuf[bs][ci[1]] = pc[1];
      }
      __syncthreads();
      if (refl && wlive) {
        // the wavefront that owns the next column goes first, so that its
        // reflector work overlaps the other wavefronts' updates
        if (wv == (h + 1) / 8) __builtin_amdgcn_s_setprio(1);
        // every LDS read of the update is issued before the first use; p is
        // complete over the group's rows (zero up to h), so u^T p is a
        // 16-lane reduction of what the lane holds
        double pr[J];
#pragma unroll
        for (int j = 0; j < J; ++j) pr[j] = pbuf[bs][gc + kRrP * j];
        double utp = 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) utp = fma(ur[j], pr[j], utp);
        const double K = 0.5 * beta * lane_reduce<kRrP>(utp, add);
        const double q0 = colok[0] ? pc[0] - K * uc[0] : 0.0, q1 = colok[1] ? pc[1] - K * uc[1] : 0.0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const double qr = fma(-K, ur[j], pr[j]);
          a[0][j] = fma(-ur[j], q0, fma(-qr, uc[0], a[0][j]));
          a[1][j] = fma(-ur[j], q1, fma(-qr, uc[1], a[1][j]));
        }
      }
      offh += kRrP * J;
    }
  };
  for (int h0 = 0; h0 < m - 2;) {
    const int J = (m - 1 - h0 + kRrP - 1) / kRrP;
    const int he = min(m - 2, m - 1 - kRrP * (J - 1));   // the first step with fewer blocks
    RR_DISPATCH(J, [&](auto Jc) { tri_steps(Jc, h0, he); });
    h0 = he;
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int c = 2 * g + e;
#pragma unroll
    for (int j = 0; j < kRrW; ++j) {
      const int idx = gc + kRrP * j, r = m - 1 - idx;
      if (c < m && idx < m && r == c) dd[c] = a[e][j];
      if (m >= 2 && c == m - 2 && idx == 0) ee[m - 2] = a[e][j];
    }
  }
  // rows past m: no coupling (their diagonal is set once |T| is known); the
  // start vector of step 3
  if (t >= m - 1 && t <= kRrRows) ee[t] = 0.0;
  if (t < kRrRows) sv[t] = 1.0 + (double)((t * 37) % 11) * (0.25 / 11.0);
  __syncthreads();

  // ---- 2. bisection for the lowest k eigenvalues ----
  // Gershgorin interval and the largest coupling, one row per thread, reduced
  // over each wavefront and then over the sixteen wavefront results
  {
    double lo = 1.79e308, hi = -1.79e308, e2 = 0.0;
    if (t < m) {
      const double rad = (t > 0 ? fabs(ee[t - 1]) : 0.0) + fabs(ee[t]);   // ee[m - 1] = 0
      lo = dd[t] - rad;
      hi = dd[t] + rad;
      e2 = ee[t] * ee[t];
    }
    lo = lane_reduce<64>(lo, fmin_);
    hi = lane_reduce<64>(hi, fmax_);
    e2 = lane_reduce<64>(e2, fmax_);
    if ((t & 63) == 0) {
      red[0][wv] = lo;
      red[1][wv] = hi;
      red[2][wv] = e2;
    }
  }
  __syncthreads();
  double lo = lane_reduce<16>(red[0][t & 15], fmin_);
  double hi = lane_reduce<16>(red[1][t & 15], fmax_);
  int ex = 0;
  (void)frexp(fmax(fabs(lo), fabs(hi)), &ex);
  const double sc = ldexp(1.0, -ex);
  lo *= sc;
  hi *= sc;
  const double tnorm = fmax(fabs(lo), fabs(hi));
  // largest scaled coupling squared (absolute floor of the widths)
  const double emax = lane_reduce<16>(red[2][t & 15], fmax_) * sc * sc;
  const double tiny = 2.2250738585072014e-308 * fmax(1.0, emax);
  const double widen = 4.0 * m * eps * tnorm + 2.0 * tiny;
  lo -= widen;
  hi += widen;
  const double dpad = 2.0 * fmax(fabs(lo), fabs(hi)) + 1.0;
  const double tn = ldexp(tnorm, ex);            // |T| bound, unscaled
  if (t < kRrRows) {
    const double e2 = t > 0 && t < m ? ee[t - 1] * ee[t - 1] * sc * sc : 0.0;
    de[t] = t < m ? make_double2(dd[t] * sc, e2) : make_double2(dpad, 0.0);
    if (t == 0) info[0] = 0;
  }
  __syncthreads();
  if (t >= 1 && t < m && de[t].y == 0.0) info[0] = 1;   // a zero coupling: split
  // rows past m for step 3: a diagonal far above every eigenvalue
  if (t >= m && t < kRrRows) dd[t] = 4.0 * tn + 1.0;
  __syncthreads();
  const bool split = info[0] != 0;
  if (wv < kRrBisWaves) {
    const int gpw = (k + kRrBisWaves - 1) / kRrBisWaves;   // eigenvalues per wavefront
    const int P = min(32, 64 / gpw);                        // lanes (points) per eigenvalue
    const int ln = t & 63, gl = ln % P, gw = ln / P;
    const int gi = wv * gpw + gw;
    const bool live = gw < gpw && gi < k;
    const int gbase = gw * P;
    const unsigned long long gmask = (1ull << P) - 1ull;
    constexpr double kBig = 1.157920892373162e77, kSmall = 8.636168555094445e-78;   // 2^256, 2^-256
    const double inv = 1.0 / (P + 1);
    double blo = lo, bhi = hi;
    auto point = [&](int i) { return fma(bhi - blo, (double)i * inv, blo); };
    auto passes = [&](auto splitc) {
      constexpr bool SPLIT = decltype(splitc)::value;
#pragma unroll 1
      for (int it = 0; it < 256; ++it) {
        const bool conv = !live || bhi - blo <= 2.0 * eps * fmax(fabs(blo), fabs(bhi)) + eps * tnorm + 4.0 * tiny;
        if (__all(conv)) break;
        const double x = point(gl + 1);
        double2 ra[4], rb[4];   // the two halves of a block of eight rows
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = de[q];
        double p1 = ra[0].x - x, p2 = 1.0;
        int neg = sign_bit(p1);
        int cnt = neg;
#pragma unroll 1
        for (int jb = 0; jb < m; jb += 8) {
#pragma unroll
          for (int q = 0; q < 4; ++q) rb[q] = de[jb + 4 + q];
          // the reads above stay here, in flight while the first half is counted
          // (an empty asm that may change memory: they cannot move below it, and
          // the next iteration cannot read the same rows afresh)
          asm volatile("" ::: "memory");
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (jb + q > 0) sturm_row<SPLIT>(ra[q].x, ra[q].y, x, p1, p2, neg, cnt);
          const int jn = jb + 8 < kRrRows ? jb + 8 : jb;   // the next block
#pragma unroll
          for (int q = 0; q < 4; ++q) ra[q] = de[jn + q];
          asm volatile("" ::: "memory");
#pragma unroll
          for (int q = 0; q < 4; ++q) sturm_row<SPLIT>(rb[q].x, rb[q].y, x, p1, p2, neg, cnt);
          const double s = fabs(p1) > kBig ? kSmall : (fabs(p1) < kSmall ? kBig : 1.0);
          p1 *= s;
          p2 *= s;
        }
        const int kk = __popcll((__ballot(cnt <= gi) >> gbase) & gmask);
        if (!conv) {
          const double nlo = kk == 0 ? blo : point(kk);
          const double nhi = kk == P ? bhi : point(kk + 1);
          blo = nlo;
          bhi = nhi;
        }
      }
    };
    if (split) passes(std::true_type{}); else passes(std::false_type{});
    if (live && gl == 0) lam[gi] = ldexp(0.5 * (blo + bhi), ex);
  }
  __syncthreads();

  // ---- 3. inverse iteration ----
  const double ctol = kRrClusterTol * tn, ptiny = eps * tn + 1e-300;
  // rank of each eigenvalue in its tight cluster: the count of consecutive
  // predecessors closer than ctol (bit i of the ballots: lam_i - lam_(i-1) < ctol)
  if (wv == 0) {
    const bool f0 = t > 0 && t < k && lam[t < k ? t : 0] - lam[t > 0 && t < k ? t - 1 : 0] < ctol;
    const int t1 = t + 64;
    const bool f1 = t1 < k && lam[t1 < k ? t1 : 0] - lam[t1 < k ? t1 - 1 : 0] < ctol;
    const unsigned long long b0 = __ballot(f0), b1 = __ballot(f1);   // bit 0 of b0 is clear
    const unsigned long long below = t == 63 ? ~0ull : (2ull << t) - 1ull;   // bits 0 .. t
    if (t < k) rank_s[t] = t - (63 - __clzll(~b0 & below));
    if (t1 < k) {
      const unsigned long long z1 = ~b1 & below;
      const int pos = z1 ? 64 + 63 - __clzll(z1) : 63 - __clzll(~b0);
      rank_s[t1] = t1 - pos;
    }
  }
  __syncthreads();
  const int jlast = (m - 1) / 8 * 8;   // first row of the last block
  for (int i0 = 0; i0 < k; i0 += kRrChunk) {
    const int i = i0 + t;
    const bool mine = t < kRrChunk && i < k;
    const int rank = mine ? rank_s[i] : 0;
    const int rmax = (int)lane_reduce<64>((double)rank, fmax_);   // wavefront 0 holds the chunk
    const int rmax_all = __shfl(rmax, 0, 64);
    if (wv == 0 && t == 0) info[1] = rmax_all;
    __syncthreads();
    const int nsteps = info[1];
    double* x = xv[t < kRrChunk ? t : 0];
    double* iv = ivp[t < kRrChunk ? t : 0];
    for (int step = 0; step <= nsteps; ++step) {
      if (mine && rank == step) {
        const double li = lam[i];
        // T - li I = L D L^T: iv_j = 1 / D_j, D_j = (d_j - li) - e_(j-1)^2 iv_(j-1)
        double ivl = 0.0;
        for (int jb = 0; jb < m; jb += 8) {
          double dl[8], el[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            dl[q] = dd[jb + q];
            el[q] = jb + q > 0 ? ee[jb + q - 1] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            double D = fma(-el[q] * el[q], ivl, dl[q] - li);
            if (fabs(D) < ptiny) D = D >= 0.0 ? ptiny : -ptiny;
            ivl = recip(D);
            iv[jb + q] = ivl;
          }
        }
        double s = 1.0;   // the vector in x is s times the stored values
        for (int pass = 0; pass < 2; ++pass) {
          // L z = x (z_j = x_j - e_(j-1) iv_(j-1) z_(j-1))
          double zp = 0.0, ivq = 0.0;
          for (int jb = 0; jb < m; jb += 8) {
            double el[8], ivb[8], xb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              el[q] = jb + q > 0 ? ee[jb + q - 1] : 0.0;
              ivb[q] = iv[jb + q];
              xb[q] = pass == 0 ? sv[jb + q] : s * x[jb + q];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              zp = fma(-(el[q] * ivq), zp, xb[q]);
              x[jb + q] = zp;
              ivq = ivb[q];
            }
          }
          // D L^T y = z (y_j = iv_j z_j - iv_j e_j y_(j+1)), last block first
          double yn = 0.0, nn = 0.0;
          for (int jb = jlast; jb >= 0; jb -= 8) {
            double el[8], ivb[8], zb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              el[q] = ee[jb + q];
              ivb[q] = iv[jb + q];
              zb[q] = x[jb + q];
            }
#pragma unroll
            for (int q = 7; q >= 0; --q) {
              yn = fma(-(ivb[q] * el[q]), yn, ivb[q] * zb[q]);
              x[jb + q] = yn;
              nn = jb + q < m ? fma(yn, yn, nn) : nn;
            }
          }
          if (rank > 0) {
            // Gram-Schmidt against the cluster's earlier eigenvectors
            for (int q = 1; q <= rank; ++q) {
              const int jv = i - q;
              const bool inchunk = jv >= i0;
              const double* y = inchunk ? xv[jv - i0] : nullptr;
              const double ys = inchunk ? xsc[jv - i0] : 1.0;
              double dot = 0.0;
              for (int j = 0; j < m; ++j) dot += (inchunk ? ys * y[j] : V[(int64_t)j * ldv + jv]) * x[j];
              for (int j = 0; j < m; ++j) x[j] -= dot * (inchunk ? ys * y[j] : V[(int64_t)j * ldv + jv]);
            }
            nn = 0.0;
            for (int j = 0; j < m; ++j) nn = fma(x[j], x[j], nn);
          }
          s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        }
        xsc[t] = s;
      }
      __syncthreads();
    }
    // eigenvectors of T of this chunk into V (transformed in step 4)
    for (int e = t; e < kRrChunk * m; e += kRrThreads) {
      const int q = e / m, j = e % m;
      if (i0 + q < k) V[(int64_t)j * ldv + i0 + q] = xsc[q] * xv[q][j];
    }
    __syncthreads();
  }
  for (int q = t; q < k; q += kRrThreads) w[q] = lam[q];

  // ---- 4. back-transform ----
  // lane l of a vector holds the reversed rows idx = l + kRrP q; reflector h
  // is nonzero in its first ceil((m - 1 - h) / kRrP) blocks, stored padded in Us
  for (int p0 = 0; p0 < k; p0 += kRrVecPass) {
    const int iv_ = p0 + t / kRrVecLanes, l = t % kRrVecLanes;
    const bool live = iv_ < k;
    double z[kRrW];
#pragma unroll
    for (int q = 0; q < kRrW; ++q) {
      const int idx = l + kRrVecLanes * q;
      z[q] = live && idx < m ? V[(int64_t)(m - 1 - idx) * ldv + iv_] : 0.0;
    }
    // reflectors hhi down to hlo, each nonzero in its first J blocks, in two
    // register sets so that each is read while the other is applied
    auto back_steps = [&](auto Jc, int hhi, int hlo, int off) {
      constexpr int J = decltype(Jc)::value;
      auto load_u = [&](double* u, int o) {
#pragma unroll
        for (int q = 0; q < J; ++q) u[q] = Us[o + l + kRrVecLanes * q];
      };
      auto apply = [&](const double* u, double b) {
        double sd = 0.0;
#pragma unroll
        for (int q = 0; q < J; ++q) sd = fma(u[q], z[q], sd);
        sd = b * lane_reduce<kRrVecLanes>(sd, add);
#pragma unroll
        for (int q = 0; q < J; ++q) z[q] = fma(-sd, u[q], z[q]);
      };
      double ua[J], ub[J];
      load_u(ua, off);
#pragma unroll 1
      for (int h = hhi; h >= hlo; h -= 2) {
        const double ba = bet[h];
        if (h - 1 >= hlo) load_u(ub, off - kRrP * J);
        apply(ua, ba);
        if (h - 1 < hlo) break;
        const double bb = bet[h - 1];
        off -= 2 * kRrP * J;
        if (h - 2 >= hlo) load_u(ua, off);
        apply(ub, bb);
      }
    };
    // phases of equal block count J, from the last reflector down
    int offp = offh;
    for (int J = 1; kRrP * (J - 1) + 1 <= m - 1; ++J) {
      const int hhi = min(m - 3, m - 2 - kRrP * (J - 1)), hlo = max(0, m - 1 - kRrP * J);
      if (hhi < hlo) continue;
      offp -= kRrP * J * (hhi - hlo + 1);
      const int off_hi = offp + kRrP * J * (hhi - hlo);   // start of reflector hhi
      RR_DISPATCH(J, [&](auto Jc) { back_steps(Jc, hhi, hlo, off_hi); });
    }
    __syncthreads();   // every read of V's columns of this pass done before the writes
#pragma unroll
    for (int q = 0; q < kRrW; ++q) {
      const int idx = l + kRrVecLanes * q;
      if (live && idx < m) V[(int64_t)(m - 1 - idx) * ldv + iv_] = z[q];
    }
  }
}

}  // namespace

hipError_t dense_syev_low(int m, int k, const double* A, int lda, double* w, double* V, int ldv, hipStream_t s) {
  if (m < 1 || m > kMaxSmall || k < 1 || k > m || !A || !w || !V || lda < m || ldv < k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rr_syev_kernel, dim3(1), dim3(kRrThreads), 0, s, m, k, A, lda, w, V, ldv);
  return hipGetLastError();
}

}  // namespace lhf

extern "C" {

int32_t lhf_dense_syev(int32_t m, int32_t k, const double* d_A, int32_t lda, double* d_w, double* d_V, int32_t ldv,
                       lhf_stream_t stream) {
  if (m < 1 || m > lhf::kMaxSmall || k < 1 || k > m || lda < m || ldv < k || !d_A || !d_w || !d_V) {
    lhf::set_error("lhf_dense_syev: need 1 <= k <= m <= " + std::to_string(lhf::kMaxSmall) +
                   ", lda >= m, ldv >= k and every pointer");
    return LHF_ERR_INVALID;
  }
  const hipError_t e = lhf::dense_syev_low(m, k, d_A, lda, d_w, d_V, ldv, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    lhf::set_error(std::string("lhf_dense_syev: ") + hipGetErrorString(e));
    return LHF_ERR_HIP;
  }
  return LHF_OK;
}

}  // extern "C"
