// Three-level block-Toeplitz operator of a lattice in a box (Sec. 2.3, item
// (A): the central cell's potential replicated to every cell makes the box
// matrix shift invariant; Def. 5.4: symmetric three-level block-Toeplitz
// class) and its action through the three-level block-circulant embedding of
// Remark 3.2 (double size at each level).
//
// Assembly.  The generators A_s = <g_(0,mu), H_rep g_(s,nu)>, s signed in
// every dimension, are Hadamard combinations of 1D Grams G_l[s_l] (Prop. 2.2),
// with G_l[-s] = G_l[s]^T.  The embedding's per-frequency blocks
//   C_f = sum_d B_d w^(f.d),  B_d = T(k, k - d) = A_(-d),
// are therefore the same Hadamard combination of the 1D transforms
//   Gh_l[f] = sum_d G_l[-d] w_l^(f d)
// (the separable route of Theorem 3.3 applied to the embedding): no 3D
// generator array is formed to build them.
//
// Matvec.  x (cell-major [L1][L2][L3][m0], ncols columns) is zero-padded and
// transformed level by level, each pass a batch of radix-2 line transforms in
// LDS that reads only the planes holding data (pruned: level 3 over the L1 L2
// occupied lines, level 2 over L1 P3, level 1 over P2 P3), one m0 x m0
// product per frequency, and the inverse passes in reverse order keeping only
// the first L_l outputs of each level.
#include <algorithm>

#include "gauss.h"
#include "toeplitz3.h"
#include "../../include/lhf.h"

namespace lhf {
namespace {

template <typename R> struct Cx3;
template <> struct Cx3<double> { typedef double2 T; };
template <> struct Cx3<float> { typedef float2 T; };

__device__ __forceinline__ double gto3(const Toep3Dev& D, int mu, int ell, double x, double c) {
  const double al = D.alpha[mu];
  const double u = x - c;
  const int pw = D.lpow[mu][ell];
  double nrm = sqrt(sqrt(2.0 * al / 3.14159265358979323846));
  if (pw) nrm *= 2.0 * sqrt(al);
  const double g = nrm * exp(-al * u * u);
  return pw ? g * u : g;
}

__device__ __forceinline__ double centre3(const Toep3Dev& D, int ell, int k) {
  return -0.5 * D.L[ell] * D.a + (k + 0.5) * D.a;
}

// Potential factors per dimension and term t = nu R + q (Z_nu w_q folded into
// dimension 1): on a multi-cell dimension the lattice-window sum of the
// central cell at the nc node offsets of a cell (window of L cells, odd L
// symmetric, even L with half weights at the two ends), on a one-cell
// dimension the nucleus's own factor on the box nodes 1..n.
// Grid: (term, dimension); thread j covers node offsets j, j + 256, ...
__global__ void __launch_bounds__(256) vpot3_kernel(const Toep3Dev* __restrict__ dp, double* __restrict__ vpot) {
  const Toep3Dev& D = *dp;
  const int t = blockIdx.x, ell = blockIdx.y, nu = t / D.R, q = t % D.R;
  const double coef = ell == 0 ? D.Z[nu] * D.wq[q] : 1.0;
  const int L = D.L[ell];
  const double h = D.h[ell];
  double* out = vpot + D.vpot_off[ell] + (int64_t)t * D.vpot_len[ell];
  for (int j = threadIdx.x; j < D.vpot_len[ell]; j += 256) {
    double acc = 0.0;
    if (L >= 2) {
      int klo, khi;
      if (L & 1) { klo = -(L - 1) / 2; khi = (L - 1) / 2; }
      else { klo = -L / 2; khi = L / 2; }
      const double y = -0.5 * D.a + (j + 0.5) * h;
      for (int k = klo; k <= khi; ++k) {
        const double wk = ((L & 1) == 0 && (k == klo || k == khi)) ? 0.5 : 1.0;
        acc += wk * cell_gauss(y, h, D.tq[q], D.nuc[nu][ell] + k * D.a);
      }
    } else {
      const double x = D.x0[ell] + (j + 1) * h;
      acc = cell_gauss(x, h, D.tq[q], centre3(D, ell, 0) + D.nuc[nu][ell]);
    }
    out[j] = coef * acc;
  }
}

// 1D Grams of one (dimension, shift s >= 0) per workgroup: rows mu of cell 0,
// columns nu of cell s, terms 0 mass, 1 stiffness, 2 + t potential.  The node
// window [ilo - 1, ihi + 1] of both cells' factors is staged in LDS (wall-free
// on multi-cell dimensions; the box nodes 1..n with zero values outside on a
// one-cell dimension).
__global__ void __launch_bounds__(256) grams3_kernel(const Toep3Dev* __restrict__ dp, const Gram3Job* __restrict__ jobs,
                                                     const double* __restrict__ vpot, double* __restrict__ grams) {
  extern __shared__ double lds[];
  const Toep3Dev& D = *dp;
  const Gram3Job jb = jobs[blockIdx.x];
  const int ell = jb.dim, s = jb.shift, m0 = D.m0, T = 2 + D.M0 * D.R;
  const int W = jb.ihi - jb.ilo + 1, WS = W + 2;
  const bool multi = D.L[ell] >= 2;
  const double h = D.h[ell];
  double* g0 = lds;                 // [m0][WS]
  double* gs = g0 + m0 * WS;        // [m0][WS]
  double* pot = gs + m0 * WS;       // [W]
  const double c0 = centre3(D, ell, 0), cs = centre3(D, ell, s);
  for (int e = threadIdx.x; e < m0 * WS; e += 256) {
    const int mu = e / WS, i = jb.ilo - 1 + e % WS;
    double v0 = 0.0, vs = 0.0;
    if (multi || (i >= 1 && i <= D.n[ell])) {
      const double x = D.x0[ell] + i * h;
      v0 = gto3(D, mu, ell, x, c0 + D.cen[mu][ell]);
      vs = gto3(D, mu, ell, x, cs + D.cen[mu][ell]);
    }
    g0[e] = v0;
    gs[e] = vs;
  }
  __syncthreads();
  double* out = grams + D.gram_off[ell] + (int64_t)s * T * m0 * m0;
  for (int e = threadIdx.x; e < m0 * m0; e += 256) {
    const int mu = e / m0, nu = e % m0;
    const double* a = g0 + mu * WS + 1;
    const double* b = gs + nu * WS + 1;
    double sm = 0.0, km = 0.0;
    for (int i = 0; i < W; ++i) {
      sm += a[i] * (b[i - 1] + 4.0 * b[i] + b[i + 1]);
      km += a[i] * (2.0 * b[i] - b[i - 1] - b[i + 1]);
    }
    out[e] = sm * (h / 6.0);
    out[m0 * m0 + e] = km / h;
  }
  const int nc = multi ? D.n[ell] / D.L[ell] : 0;
  for (int t = 0; t < D.M0 * D.R; ++t) {
    __syncthreads();
    const double* vp = vpot + D.vpot_off[ell] + (int64_t)t * D.vpot_len[ell];
    for (int i = threadIdx.x; i < W; i += 256) {
      const int node = jb.ilo + i;
      double v = 0.0;
      if (multi) {
        int j = (node - 1) % nc;
        if (j < 0) j += nc;
        v = vp[j];
      } else if (node >= 1 && node <= D.n[ell]) {
        v = vp[node - 1];
      }
      pot[i] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < m0 * m0; e += 256) {
      const int mu = e / m0, nu = e % m0;
      const double* a = g0 + mu * WS + 1;
      const double* b = gs + nu * WS + 1;
      double v = 0.0;
      for (int i = 0; i < W; ++i) v += a[i] * pot[i] * b[i];
      out[(int64_t)(2 + t) * m0 * m0 + e] = v;
    }
  }
}

// G_l[t][s] for a signed shift (G[-s] = G[s]^T), entry (mu, nu).
__device__ __forceinline__ double gram_signed(const Toep3Dev& D, const double* grams, int ell, int t, int s, int mu,
                                              int nu) {
  const int m0 = D.m0, T = 2 + D.M0 * D.R;
  const int as = s >= 0 ? s : -s;
  const int e = s >= 0 ? mu * m0 + nu : nu * m0 + mu;
  return grams[D.gram_off[ell] + ((int64_t)as * T + t) * m0 * m0 + e];
}

// 1D transforms onto the embedding frequencies:
//   Gh_l[t][f] = sum_(d = -L0..L0) G_l[t][-d] exp(-2 pi i f d / P_l).
// One thread per (dimension, term, frequency, entry); grid x over all of them.
__global__ void __launch_bounds__(256) ghat3_kernel(const Toep3Dev* __restrict__ dp, const double* __restrict__ grams,
                                                    double2* __restrict__ gh, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const Toep3Dev& D = *dp;
  const int m0 = D.m0, mm = m0 * m0, T = 2 + D.M0 * D.R;
  int ell = 0;
  int64_t r = idx;
  while (ell < 2 && r >= (int64_t)T * D.P[ell] * mm) {
    r -= (int64_t)T * D.P[ell] * mm;
    ++ell;
  }
  const int e = (int)(r % mm), f = (int)((r / mm) % D.P[ell]), t = (int)(r / ((int64_t)mm * D.P[ell]));
  const int mu = e / m0, nu = e % m0, P = D.P[ell], L0 = D.L0[ell];
  double re = 0.0, im = 0.0;
  for (int d = -L0; d <= L0; ++d) {
    const double g = gram_signed(D, grams, ell, t, -d, mu, nu);
    int rr = (int)(((int64_t)f * (d < 0 ? d + P : d)) % P);
    double sn, cs;
    sincospi(-2.0 * rr / P, &sn, &cs);
    re += g * cs;
    im += g * sn;
  }
  gh[D.gh_off[ell] + ((int64_t)t * P + f) * mm + e] = make_double2(re, im);
}

__device__ __forceinline__ double2 cmul3(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Per-frequency blocks of the embedding, f = (f1 P2 + f2) P3 + f3:
//   C_S = Sh1 o Sh2 o Sh3,
//   C_H = 1/2 (Kh1 o Sh2 o Sh3 + Sh1 o Kh2 o Sh3 + Sh1 o Sh2 o Kh3) - sum_t Mh1_t o Mh2_t o Mh3_t.
__global__ void __launch_bounds__(256) chat3_kernel(const Toep3Dev* __restrict__ dp, const double2* __restrict__ gh,
                                                    double2* __restrict__ cH, double2* __restrict__ cS, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const Toep3Dev& D = *dp;
  const int mm = D.m0 * D.m0, T = 2 + D.M0 * D.R;
  const int e = (int)(idx % mm);
  const int64_t f = idx / mm;
  const int f3 = (int)(f % D.P[2]), f2 = (int)((f / D.P[2]) % D.P[1]), f1 = (int)(f / ((int64_t)D.P[2] * D.P[1]));
  const int fl[3] = {f1, f2, f3};
  auto at = [&](int ell, int t) { return gh[D.gh_off[ell] + ((int64_t)t * D.P[ell] + fl[ell]) * mm + e]; };
  const double2 s1 = at(0, 0), s2 = at(1, 0), s3 = at(2, 0);
  const double2 k1 = at(0, 1), k2 = at(1, 1), k3 = at(2, 1);
  const double2 s23 = cmul3(s2, s3);
  double2 hsum = cmul3(k1, s23);
  const double2 b = cmul3(s1, cmul3(k2, s3)), c = cmul3(cmul3(s1, s2), k3);
  hsum = make_double2(0.5 * (hsum.x + b.x + c.x), 0.5 * (hsum.y + b.y + c.y));
  for (int t = 2; t < T; ++t) {
    const double2 v = cmul3(cmul3(at(0, t), at(1, t)), at(2, t));
    hsum.x -= v.x;
    hsum.y -= v.y;
  }
  cH[idx] = hsum;
  cS[idx] = cmul3(s1, s23);
}

// Generators A_s, s + L0 in [0, 2 L0_l], layout [s1][s2][s3][mu][nu] (for
// read-back; the matvec does not use them).
__global__ void __launch_bounds__(256) gen3_kernel(const Toep3Dev* __restrict__ dp, const double* __restrict__ grams,
                                                   double* __restrict__ gH, double* __restrict__ gS, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const Toep3Dev& D = *dp;
  const int m0 = D.m0, mm = m0 * m0, T = 2 + D.M0 * D.R;
  const int e = (int)(idx % mm), mu = e / m0, nu = e % m0;
  const int64_t g = idx / mm;
  const int n3 = 2 * D.L0[2] + 1, n2 = 2 * D.L0[1] + 1;
  const int s3 = (int)(g % n3) - D.L0[2], s2 = (int)((g / n3) % n2) - D.L0[1], s1 = (int)(g / (n3 * n2)) - D.L0[0];
  auto G = [&](int ell, int t, int s) { return gram_signed(D, grams, ell, t, s, mu, nu); };
  const double S1 = G(0, 0, s1), S2 = G(1, 0, s2), S3 = G(2, 0, s3);
  double h = 0.5 * (G(0, 1, s1) * S2 * S3 + S1 * G(1, 1, s2) * S3 + S1 * S2 * G(2, 1, s3));
  for (int t = 2; t < T; ++t) h -= G(0, t, s1) * G(1, t, s2) * G(2, t, s3);
  gH[idx] = h;
  gS[idx] = S1 * S2 * S3;
}

__device__ __forceinline__ int bitrev3(int x, int bits) {
  return bits == 0 ? 0 : (int)(__brev((unsigned)x) >> (32 - bits));
}

// One level of the embedding transform for a batch of lines: line (o, c),
// o < nouter, c < ninner, input entries p < pin at in[(o pin + p) ninner + c]
// (zero for pin <= p < P), output entries p < pout at out[(o pout + p) ninner
// + c].  First pass (REAL_IN): the input is x (FP64, [cells][m0][ld]) with
// c = mu ncols + j and (o, p) = (cell / L3, cell % L3).  Last pass (REAL_OUT):
// the real part times `scale` goes to y the same way.  INV: inverse
// transform (conjugate twiddles).  Grid y: operator (H, S) for the passes
// after the product.  CB lines per workgroup, radix 2 in LDS.
template <typename R, bool INV, bool REAL_IN, bool REAL_OUT>
__global__ void __launch_bounds__(256) lines3_kernel(int nouter, int ninner, int pin, int pout, int P, int bits, int CB,
                                                     const typename Cx3<R>::T* __restrict__ tw,
                                                     const void* __restrict__ in0, const void* __restrict__ in1,
                                                     void* __restrict__ out0, void* __restrict__ out1, int m0,
                                                     int ncols, int ld, double scale) {
  typedef typename Cx3<R>::T C;
  extern __shared__ char lraw3[];
  C* a = reinterpret_cast<C*>(lraw3);
  const int64_t nlines = (int64_t)nouter * ninner;
  const int64_t l0 = (int64_t)blockIdx.x * CB;
  const void* in = blockIdx.y == 0 ? in0 : in1;
  void* out = blockIdx.y == 0 ? out0 : out1;
  for (int e = threadIdx.x; e < CB * P; e += 256) {
    const int cc = e / P, p = e % P;
    const int64_t line = l0 + cc;
    C v;
    v.x = 0;
    v.y = 0;
    if (line < nlines && p < pin) {
      const int64_t o = line / ninner;
      const int c = (int)(line % ninner);
      if constexpr (REAL_IN) {
        const int mu = c / ncols, j = c % ncols;
        const int64_t cell = o * pin + p;
        v.x = (R)static_cast<const double*>(in)[(cell * m0 + mu) * ld + j];
      } else {
        v = static_cast<const C*>(in)[(o * pin + p) * ninner + c];
      }
    }
    a[cc * P + bitrev3(p, bits)] = v;
  }
  __syncthreads();
  for (int s = 1; s <= bits; ++s) {
    const int half = 1 << (s - 1);
    const int tstride = P >> s;
    for (int b = threadIdx.x; b < CB * (P / 2); b += 256) {
      const int cc = b / (P / 2), bb = b % (P / 2);
      const int grp = bb / half, pos = bb % half;
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      C w = tw[pos * tstride];
      if (INV) w.y = -w.y;
      C* col = a + cc * P;
      const C u = col[i0], v0 = col[i1];
      C v;
      v.x = v0.x * w.x - v0.y * w.y;
      v.y = v0.x * w.y + v0.y * w.x;
      col[i0].x = u.x + v.x;
      col[i0].y = u.y + v.y;
      col[i1].x = u.x - v.x;
      col[i1].y = u.y - v.y;
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < CB * pout; e += 256) {
    const int cc = e / pout, p = e % pout;
    const int64_t line = l0 + cc;
    if (line >= nlines) continue;
    const int64_t o = line / ninner;
    const int c = (int)(line % ninner);
    if constexpr (REAL_OUT) {
      const int mu = c / ncols, j = c % ncols;
      const int64_t cell = o * pout + p;
      static_cast<double*>(out)[(cell * m0 + mu) * ld + j] = (double)a[cc * P + p].x * scale;
    } else {
      static_cast<C*>(out)[(o * pout + p) * ninner + c] = a[cc * P + p];
    }
  }
}

// Per-frequency products yhat_f = op_f xhat_f (op_f m0 x m0, xhat_f m0 x
// ncols), one or two operators (grid y).
template <typename R>
__global__ void __launch_bounds__(256) fmul3_kernel(int m0, int ncols, const typename Cx3<R>::T* __restrict__ opH,
                                                    const typename Cx3<R>::T* __restrict__ opS,
                                                    const typename Cx3<R>::T* __restrict__ xhat,
                                                    typename Cx3<R>::T* __restrict__ yH,
                                                    typename Cx3<R>::T* __restrict__ yS) {
  typedef typename Cx3<R>::T C;
  extern __shared__ char lraw3m[];
  C* op = reinterpret_cast<C*>(lraw3m);        // [m0][m0]
  C* xs = op + m0 * m0;                        // [m0][ncols]
  const int64_t f = blockIdx.x;
  const C* o = (blockIdx.y == 0 ? opH : opS) + f * m0 * m0;
  C* y = (blockIdx.y == 0 ? yH : yS) + f * m0 * ncols;
  const C* xf = xhat + f * m0 * ncols;
  for (int e = threadIdx.x; e < m0 * m0; e += 256) op[e] = o[e];
  for (int e = threadIdx.x; e < m0 * ncols; e += 256) xs[e] = xf[e];
  __syncthreads();
  for (int e = threadIdx.x; e < m0 * ncols; e += 256) {
    const int mu = e / ncols, j = e % ncols;
    R re = 0, im = 0;
    for (int nu = 0; nu < m0; ++nu) {
      const C av = op[mu * m0 + nu], bv = xs[nu * ncols + j];
      re += av.x * bv.x - av.y * bv.y;
      im += av.x * bv.y + av.y * bv.x;
    }
    C r;
    r.x = re;
    r.y = im;
    y[e] = r;
  }
}

int log2i(int P) {
  int b = 0;
  while ((1 << b) < P) ++b;
  return b;
}

template <typename R, bool INV, bool RI, bool RO>
hipError_t lines(int nouter, int ninner, int pin, int pout, int P, const void* tw, const void* in0, const void* in1,
                 void* out0, void* out1, int nops, int m0, int ncols, int ld, double scale, hipStream_t s) {
  typedef typename Cx3<R>::T C;
  const int CB = std::max(1, std::min(64, 32768 / (P * (int)sizeof(C))));
  const int64_t nl = (int64_t)nouter * ninner;
  const size_t lds = (size_t)CB * P * sizeof(C);
  (void)hipFuncSetAttribute((const void*)lines3_kernel<R, INV, RI, RO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL((lines3_kernel<R, INV, RI, RO>), dim3((unsigned)((nl + CB - 1) / CB), nops), dim3(256), lds, s,
                     nouter, ninner, pin, pout, P, log2i(P), CB, (const C*)tw, in0, in1, out0, out1, m0, ncols, ld,
                     scale);
  return hipGetLastError();
}

template <typename R>
hipError_t apply3_t(const Toep3Dev& H, const void* const* tw, int ncols, const double* x, int ld, const void* opH,
                    const void* opS, double* yH, double* yS, void* ws, hipStream_t s) {
  typedef typename Cx3<R>::T C;
  const int L1 = H.L[0], L2 = H.L[1], L3 = H.L[2], P1 = H.P[0], P2 = H.P[1], P3 = H.P[2], m0 = H.m0;
  const int ncol = m0 * ncols;
  const int64_t nA = (int64_t)L1 * L2 * P3 * ncol, nB = (int64_t)L1 * P2 * P3 * ncol,
                nC = (int64_t)P1 * P2 * P3 * ncol;
  C* base = static_cast<C*>(ws);
  C* A0 = base;               // level-3 transforms [L1][L2][P3][ncol] (and H's inverse)
  C* A1 = A0 + nA;            // S's inverse
  C* B0 = A1 + nA;            // level-2 transforms [L1][P2][P3][ncol]
  C* B1 = B0 + nB;
  C* X = B1 + nB;             // [P][ncol]
  C* YH = X + nC;
  C* YS = YH + nC;
  const int nops = opS ? 2 : 1;
  hipError_t e;
  // forward: level 3 (real input), level 2, level 1
  e = lines<R, false, true, false>(L1 * L2, ncol, L3, P3, P3, tw[2], x, x, A0, A0, 1, m0, ncols, ld, 1.0, s);
  if (e == hipSuccess)
    e = lines<R, false, false, false>(L1, P3 * ncol, L2, P2, P2, tw[1], A0, A0, B0, B0, 1, m0, ncols, ld, 1.0, s);
  if (e == hipSuccess)
    e = lines<R, false, false, false>(1, P2 * P3 * ncol, L1, P1, P1, tw[0], B0, B0, X, X, 1, m0, ncols, ld, 1.0, s);
  if (e != hipSuccess) return e;
  const size_t lm = sizeof(C) * ((size_t)m0 * m0 + (size_t)m0 * ncols);
  (void)hipFuncSetAttribute((const void*)fmul3_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lm);
  hipLaunchKernelGGL((fmul3_kernel<R>), dim3((unsigned)((int64_t)P1 * P2 * P3), nops), dim3(256), lm, s, m0, ncols,
                     (const C*)opH, (const C*)opS, (const C*)X, YH, YS);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // inverse: level 1 (keep L1), level 2 (keep L2), level 3 (keep L3, real part / P)
  const double scale = 1.0 / ((double)P1 * P2 * P3);
  e = lines<R, true, false, false>(1, P2 * P3 * ncol, P1, L1, P1, tw[0], YH, YS, B0, B1, nops, m0, ncols, ld, 1.0, s);
  if (e == hipSuccess)
    e = lines<R, true, false, false>(L1, P3 * ncol, P2, L2, P2, tw[1], B0, B1, A0, A1, nops, m0, ncols, ld, 1.0, s);
  if (e == hipSuccess)
    e = lines<R, true, false, true>(L1 * L2, ncol, P3, L3, P3, tw[2], A0, A1, yH, yS, nops, m0, ncols, ld, scale, s);
  return e;
}

}  // namespace

size_t toep3_apply_ws_bytes(const Toep3Dev& H, int ncols, bool fp64) {
  const int64_t ncol = (int64_t)H.m0 * ncols;
  const int64_t nA = (int64_t)H.L[0] * H.L[1] * H.P[2] * ncol, nB = (int64_t)H.L[0] * H.P[1] * H.P[2] * ncol,
                nC = (int64_t)H.P[0] * H.P[1] * H.P[2] * ncol;
  return (size_t)(2 * nA + 2 * nB + 3 * nC) * (fp64 ? 16 : 8);
}

hipError_t toep3_launch_assembly(const Toep3Dev* d, const Toep3Dev& H, const Gram3Job* jobs, int njobs, int wmax,
                                 double* vpot, double* grams, double2* gh, double2* cH, double2* cS, hipStream_t s) {
  const int M0R = H.M0 * H.R;
  hipLaunchKernelGGL(vpot3_kernel, dim3(M0R, 3), dim3(256), 0, s, d, vpot);
  const size_t lds = sizeof(double) * (2 * (size_t)H.m0 * (wmax + 2) + (size_t)wmax);
  (void)hipFuncSetAttribute((const void*)grams3_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(grams3_kernel, dim3(njobs), dim3(256), lds, s, d, jobs, vpot, grams);
  const int64_t mm = (int64_t)H.m0 * H.m0, T = 2 + M0R;
  const int64_t ngh = T * mm * ((int64_t)H.P[0] + H.P[1] + H.P[2]);
  hipLaunchKernelGGL(ghat3_kernel, dim3((unsigned)((ngh + 255) / 256)), dim3(256), 0, s, d, grams, gh, ngh);
  const int64_t nf = mm * H.P[0] * H.P[1] * H.P[2];
  hipLaunchKernelGGL(chat3_kernel, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, d, gh, cH, cS, nf);
  return hipGetLastError();
}

hipError_t toep3_launch_generators(const Toep3Dev* d, const Toep3Dev& H, const double* grams, double* gH, double* gS,
                                   hipStream_t s) {
  const int64_t n = (int64_t)H.m0 * H.m0 * (2 * H.L0[0] + 1) * (2 * H.L0[1] + 1) * (2 * H.L0[2] + 1);
  hipLaunchKernelGGL(gen3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, grams, gH, gS, n);
  return hipGetLastError();
}

hipError_t toep3_launch_apply(const Toep3Dev& H, int prec, const void* const* tw, int ncols, const double* x, int ld,
                              const void* opH, const void* opS, double* yH, double* yS, void* ws, hipStream_t s) {
  return prec == LHF_PREC_FP64 ? apply3_t<double>(H, tw, ncols, x, ld, opH, opS, yH, yS, ws, s)
                               : apply3_t<float>(H, tw, ncols, x, ld, opH, opS, yH, yS, ws, s);
}

}  // namespace lhf
