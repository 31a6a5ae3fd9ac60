// Dirichlet chain with defect cells as a perturbed block-Toeplitz operator
// (Sec. 3, the box-case treatment of defects: replicate the central cell's
// potential, then the matrix is block Toeplitz up to block rows and columns of
// a few cells; Remark 3.2: a block-Toeplitz matrix acts through a
// block-circulant embedding of about twice its size).
//
// Assembly: every block of the model is a Hadamard combination of 1D Grams
// (Prop. 2.2, Lemma 3.4).  Along the chain the Grams are taken over a window
// of nodes that holds every non-negligible factor value (on the wall-free
// grid for the pristine generators, on the box grid with its walls for the
// cross blocks); across the chain, per pair of exponent scales.
//
// Matvec: forward DFT over the cell index of every column (radix-2 in LDS,
// zero-padded to P), one m0 x m0 product per frequency, inverse DFT and the
// first L blocks, then the cross corrections D = H_model - T, block row by
// block row (no atomics).
#include <algorithm>
#include <type_traits>

#include "gauss.h"
#include "toeplitz.h"
#include "../../include/lhf.h"

namespace lhf {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { typedef double2 T; };
template <> struct Cx<float> { typedef float2 T; };

__device__ __forceinline__ double gto(const ToepDev& D, int mu, int ell, double scale, double x, double c) {
  const double al = D.alpha[mu] * scale;
  const double u = x - c;
  const int pw = D.lpow[mu][ell];
  double nrm = sqrt(sqrt(2.0 * al / 3.14159265358979323846));
  if (pw) nrm *= 2.0 * sqrt(al);
  const double g = nrm * exp(-al * u * u);
  return pw ? g * u : g;
}

__device__ __forceinline__ double cell_centre(const ToepDev& D, int k) {
  return -0.5 * D.L * D.a + (k + 0.5) * D.a;
}

// V_rep along the chain: the lattice-window potential of the central cell
// (window of L cells; odd L symmetric, even L with half weights at the ends)
// on the nc node offsets of a cell, Z_nu w_q folded in.  One workgroup per
// term nu R + q; thread t sums images k = klo + t / nc (step 256 / nc) for
// offset t % nc; the partial sums are added in a fixed order.
__global__ void __launch_bounds__(256) vrep_kernel(const ToepDev* __restrict__ dp, double* __restrict__ vrep) {
  __shared__ double part[256];
  const ToepDev& D = *dp;
  const int r = blockIdx.x, nu = r / D.R, q = r % D.R;
  const int nc = D.nc, chunks = 256 / nc, tid = threadIdx.x;
  const int j = tid % nc, c = tid / nc;
  int klo, khi;
  if (D.L & 1) { klo = -(D.L - 1) / 2; khi = (D.L - 1) / 2; }
  else { klo = -D.L / 2; khi = D.L / 2; }
  double acc = 0.0;
  if (c < chunks) {
    const double y = -0.5 * D.a + (j + 0.5) * D.h;
    for (int k = klo + c; k <= khi; k += chunks) {
      const double wk = ((D.L & 1) == 0 && (k == klo || k == khi)) ? 0.5 : 1.0;
      acc += wk * cell_gauss(y, D.h, D.tq[q], D.nuc[nu][0] + k * D.a);
    }
  }
  part[tid] = acc;
  __syncthreads();
  if (tid < nc) {
    double v = 0.0;
    for (int cc = 0; cc < chunks; ++cc) v += part[cc * nc + tid];
    vrep[r * nc + tid] = D.Z[nu] * D.wq[q] * v;
  }
}

// The finite lattice's own potential along the chain (the exact box case,
// eq. EwaldSumE in the factor form of eq. EwaldTensorGl): on box node i,
// sum over cells c = 0..L-1 of Z_(nu, c) phi_q(x_i; X_c + a_nu), times w_q,
// with the defect charge on defect cells.  Cells whose Gaussian term is below
// exp(-1400) at the node are skipped (they add exactly zero); the sum runs in
// ascending cell order.  Grid: (term, node chunk of 256).
__global__ void __launch_bounds__(256) vbox_kernel(const ToepDev* __restrict__ dp, const Defect* __restrict__ defs,
                                                   const int32_t* __restrict__ cell_def, double* __restrict__ vbox) {
  const ToepDev& D = *dp;
  const int r = blockIdx.x, nu = r / D.R, q = r % D.R;
  const int i = blockIdx.y * 256 + threadIdx.x + 1;   // box node 1..n
  if (i > D.n) return;
  const double x = D.x0 + i * D.h, t = D.tq[q];
  const double reach = 37.5 / t + D.h;                // t |x - A| > 37.4: term < exp(-1400)
  const double X0 = -0.5 * D.L * D.a + 0.5 * D.a + D.nuc[nu][0];
  int clo = (int)floor((x - reach - X0) / D.a), chi = (int)ceil((x + reach - X0) / D.a);
  clo = max(clo, 0);
  chi = min(chi, D.L - 1);
  double acc = 0.0;
  for (int c = clo; c <= chi; ++c) {
    const int di = cell_def[c];
    const double z = di >= 0 ? defs[di].Z : D.Z[nu];
    acc += z * cell_gauss(x, D.h, t, X0 + c * D.a);
  }
  vbox[(int64_t)r * D.n + i - 1] = D.wq[q] * acc;
}

constexpr int kTChunk = 64;   // transverse nodes per LDS chunk

// Transverse Grams of one pair of exponent scales and one dimension (2 or 3):
// out[pair][dim][t][mu][nu], t = 0 mass, 1 stiffness, 2 + nu' R + q the
// potential factor of nucleus nu' (no charge or weight).  The box grid of a
// one-cell dimension has nodes 1..nt and zero values outside.  Chunks of
// nodes are staged in LDS; partial sums are accumulated in the output in
// chunk order.
__global__ void __launch_bounds__(256) transverse_kernel(const ToepDev* __restrict__ dp,
                                                         const Defect* __restrict__ defs,
                                                         const ScalePair* __restrict__ pairs,
                                                         double* __restrict__ out) {
  extern __shared__ double lds[];
  const ToepDev& D = *dp;
  const int pr = blockIdx.x, dim = blockIdx.y, ell = 1 + dim;
  const int m0 = D.m0, T2 = 2 + D.M0 * D.R, W = kTChunk + 2;
  double* gk = lds;                    // [m0][W]
  double* gm = gk + m0 * W;            // [m0][W]
  double* pot = gm + m0 * W;           // [M0 R][kTChunk]
  const ScalePair sp = pairs[pr];
  const double sk = sp.dk >= 0 ? defs[sp.dk].scale : 1.0;
  const double sm = sp.dm >= 0 ? defs[sp.dm].scale : 1.0;
  const int nt = D.nt[dim];
  const double ht = D.ht[dim], t0 = D.t0[dim];
  double* o = out + ((int64_t)pr * 2 + dim) * T2 * m0 * m0;
  for (int c0 = 1; c0 <= nt; c0 += kTChunk) {
    // stage nodes c0 - 1 .. c0 + kTChunk (zero outside 1..nt)
    for (int e = threadIdx.x; e < m0 * W; e += 256) {
      const int mu = e / W, i = c0 - 1 + e % W;
      double vk = 0.0, vm = 0.0;
      if (i >= 1 && i <= nt) {
        const double x = t0 + i * ht;
        vk = gto(D, mu, ell, sk, x, D.cen[mu][ell]);
        vm = gto(D, mu, ell, sm, x, D.cen[mu][ell]);
      }
      gk[e] = vk;
      gm[e] = vm;
    }
    for (int e = threadIdx.x; e < D.M0 * D.R * kTChunk; e += 256) {
      const int t = e / kTChunk, i = c0 + e % kTChunk;
      const int nu = t / D.R, q = t % D.R;
      pot[e] = i <= nt ? cell_gauss(t0 + i * ht, ht, D.tq[q], D.nuc[nu][ell]) : 0.0;
    }
    __syncthreads();
    const int cnt = min(kTChunk, nt - c0 + 1);
    for (int e = threadIdx.x; e < m0 * m0; e += 256) {
      const int mu = e / m0, nu = e % m0;
      const double* a = gk + mu * W + 1;
      const double* b = gm + nu * W + 1;
      double s = 0.0, k = 0.0;
      for (int i = 0; i < cnt; ++i) {
        s += a[i] * (b[i - 1] + 4.0 * b[i] + b[i + 1]);
        k += a[i] * (2.0 * b[i] - b[i - 1] - b[i + 1]);
      }
      const bool first = c0 == 1;
      o[e] = (first ? 0.0 : o[e]) + s * (ht / 6.0);
      o[m0 * m0 + e] = (first ? 0.0 : o[m0 * m0 + e]) + k / ht;
      for (int t = 0; t < D.M0 * D.R; ++t) {
        const double* p = pot + t * kTChunk;
        double v = 0.0;
        for (int i = 0; i < cnt; ++i) v += a[i] * p[i] * b[i];
        double* ot = o + (int64_t)(2 + t) * m0 * m0 + e;
        *ot = (first ? 0.0 : *ot) + v;
      }
    }
    __syncthreads();
  }
}

constexpr int kMaxEntries = 4;   // (mu, nu) entries per thread: m0^2 <= 1024

// One block of the model per workgroup (see ToepJob).  The chain window
// [ilo - 1, ihi + 1] of both cells' factors is staged in LDS (zero outside the
// box for cross and exact blocks); then the mass and stiffness Grams, and one
// potential term at a time (V_rep terms, then the defect terms of the block's
// defect cells; for exact blocks the finite-lattice terms, which hold the
// defect charges already) staged in LDS and contracted, times the transverse
// Grams.
__global__ void __launch_bounds__(256) block_kernel(const ToepDev* __restrict__ dp,
                                                    const Defect* __restrict__ defs,
                                                    const ToepJob* __restrict__ jobs,
                                                    const double* __restrict__ vrep,
                                                    const double* __restrict__ vbox,
                                                    const double* __restrict__ trans,
                                                    double* __restrict__ outH, double* __restrict__ outS) {
  extern __shared__ double lds[];
  const ToepDev& D = *dp;
  const ToepJob jb = jobs[blockIdx.x];
  const int m0 = D.m0, M0R = D.M0 * D.R, T2 = 2 + M0R;
  const int W = jb.ihi - jb.ilo + 1, WS = W + 2;
  double* gk = lds;                 // [m0][WS]
  double* gm = gk + m0 * WS;        // [m0][WS]
  double* pot = gm + m0 * WS;       // [W]
  const double sk = jb.dk >= 0 ? defs[jb.dk].scale : 1.0;
  const double sm = jb.dm >= 0 ? defs[jb.dm].scale : 1.0;
  const double ck = cell_centre(D, jb.k), cm = cell_centre(D, jb.m);
  for (int e = threadIdx.x; e < m0 * WS; e += 256) {
    const int mu = e / WS, i = jb.ilo - 1 + e % WS;
    double vk = 0.0, vm = 0.0;
    if (jb.mode == 0 || (i >= 1 && i <= D.n)) {
      const double x = D.x0 + i * D.h;
      vk = gto(D, mu, 0, sk, x, ck + D.cen[mu][0]);
      vm = gto(D, mu, 0, sm, x, cm + D.cen[mu][0]);
    }
    gk[e] = vk;
    gm[e] = vm;
  }
  __syncthreads();
  const double* ty = trans + ((int64_t)jb.pair * 2 + 0) * T2 * m0 * m0;
  const double* tz = trans + ((int64_t)jb.pair * 2 + 1) * T2 * m0 * m0;
  double sx[kMaxEntries], kx[kMaxEntries], hv[kMaxEntries];
#pragma unroll
  for (int u = 0; u < kMaxEntries; ++u) {
    sx[u] = kx[u] = hv[u] = 0.0;
    const int e = threadIdx.x + u * 256;
    if (e < m0 * m0) {
      const int mu = e / m0, nu = e % m0;
      const double* a = gk + mu * WS + 1;
      const double* b = gm + nu * WS + 1;
      double s = 0.0, k = 0.0;
      for (int i = 0; i < W; ++i) {
        s += a[i] * (b[i - 1] + 4.0 * b[i] + b[i + 1]);
        k += a[i] * (2.0 * b[i] - b[i - 1] - b[i + 1]);
      }
      sx[u] = s * (D.h / 6.0);
      kx[u] = k / D.h;
    }
  }
  // potential terms: V_rep (M0 R), then M0 R per defect cell of the block
  const int ndt = (jb.mode == 1 && jb.dk >= 0 ? 1 : 0) + (jb.mode == 1 && jb.dm >= 0 && jb.dm != jb.dk ? 1 : 0);
  const int nterms = M0R * (1 + ndt);
  for (int tt = 0; tt < nterms; ++tt) {
    const int t = tt % M0R, src = tt / M0R;   // src 0: V_rep, 1: first defect, 2: second
    const int nu = t / D.R, q = t % D.R;
    __syncthreads();   // pot[] of the previous term has been consumed
    if (src == 0 && jb.mode == 2) {
      for (int i = threadIdx.x; i < W; i += 256) {
        const int node = jb.ilo + i;
        pot[i] = node >= 1 && node <= D.n ? vbox[(int64_t)t * D.n + node - 1] : 0.0;
      }
    } else if (src == 0) {
      for (int i = threadIdx.x; i < W; i += 256) {
        int j = (jb.ilo + i - 1) % D.nc;
        if (j < 0) j += D.nc;
        pot[i] = vrep[t * D.nc + j];
      }
    } else {
      const int di = (src == 1 && jb.dk >= 0) ? jb.dk : jb.dm;
      const Defect df = defs[di];
      const double coef = (df.Z - D.Z[nu]) * D.wq[q];
      const double A = cell_centre(D, df.cell) + D.nuc[nu][0];
      for (int i = threadIdx.x; i < W; i += 256)
        pot[i] = coef * cell_gauss(D.x0 + (jb.ilo + i) * D.h, D.h, D.tq[q], A);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxEntries; ++u) {
      const int e = threadIdx.x + u * 256;
      if (e < m0 * m0) {
        const int mu = e / m0, nu2 = e % m0;
        const double* a = gk + mu * WS + 1;
        const double* b = gm + nu2 * WS + 1;
        double v = 0.0;
        for (int i = 0; i < W; ++i) v += a[i] * pot[i] * b[i];
        const int64_t tr = (int64_t)(2 + t) * m0 * m0 + e;
        hv[u] -= v * ty[tr] * tz[tr];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kMaxEntries; ++u) {
    const int e = threadIdx.x + u * 256;
    if (e < m0 * m0) {
      const double sy = ty[e], ky = ty[m0 * m0 + e], sz = tz[e], kz = tz[m0 * m0 + e];
      const double h = 0.5 * (kx[u] * sy * sz + sx[u] * ky * sz + sx[u] * sy * kz) + hv[u];
      outH[(int64_t)blockIdx.x * m0 * m0 + e] = h;
      outS[(int64_t)blockIdx.x * m0 * m0 + e] = sx[u] * sy * sz;
    }
  }
}

// Cross corrections D = H_model(k, m) - T(k, m) for every entry of every
// affected block row (one workgroup per row).
__global__ void __launch_bounds__(256) delta_kernel(const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ row_cell,
                                                    const CrossEntry* __restrict__ ent,
                                                    const double* __restrict__ genH, const double* __restrict__ genS,
                                                    const double* __restrict__ crossH,
                                                    const double* __restrict__ crossS, double* __restrict__ dH,
                                                    double* __restrict__ dS, int m0) {
  const int r = blockIdx.x, k = row_cell[r];
  const int mm = m0 * m0;
  for (int j = row_ptr[r]; j < row_ptr[r + 1]; ++j) {
    const CrossEntry ce = ent[j];
    const int s = ce.m >= k ? ce.m - k : k - ce.m;
    for (int e = threadIdx.x; e < mm; e += 256) {
      const int mu = e / m0, nu = e % m0;
      const int eb = ce.trans ? nu * m0 + mu : e;               // model block entry
      const int et = ce.m >= k ? e : nu * m0 + mu;              // T(k, m) = A_s or A_s^T
      const double th = genH ? genH[(int64_t)s * mm + et] : 0.0;
      const double ts = genS ? genS[(int64_t)s * mm + et] : 0.0;
      dH[(int64_t)j * mm + e] = crossH[(int64_t)ce.blk * mm + eb] - th;
      dS[(int64_t)j * mm + e] = crossS[(int64_t)ce.blk * mm + eb] - ts;
    }
  }
}

// Per-frequency blocks of the circulant embedding (generators c_d = A_d^T,
// c_(P-d) = A_d, d <= L0):  C_f = sum_d c_d exp(-2 pi i f d / P).
__global__ void __launch_bounds__(256) chat_kernel(const double* __restrict__ genH, const double* __restrict__ genS,
                                                   double2* __restrict__ cH, double2* __restrict__ cS, int m0, int P,
                                                   int L0) {
  const int f = blockIdx.x, mm = m0 * m0;
  for (int e = threadIdx.x; e < mm; e += 256) {
    const int mu = e / m0, nu = e % m0;
    double hr = 0, hi = 0, sr = 0, si = 0;
    for (int d = 0; d <= L0; ++d) {
      const int r = (int)(((int64_t)f * d) % P);
      double sn, cs;
      sincos(-2.0 * 3.14159265358979323846 * r / P, &sn, &cs);
      const double ah = genH[(int64_t)d * mm + nu * m0 + mu], as = genS[(int64_t)d * mm + nu * m0 + mu];
      hr += ah * cs; hi += ah * sn;
      sr += as * cs; si += as * sn;
      if (d) {
        const double bh = genH[(int64_t)d * mm + e], bs = genS[(int64_t)d * mm + e];
        hr += bh * cs; hi -= bh * sn;
        sr += bs * cs; si -= bs * sn;
      }
    }
    cH[(int64_t)f * mm + e] = make_double2(hr, hi);
    cS[(int64_t)f * mm + e] = make_double2(sr, si);
  }
}

// Preconditioner blocks (H_f - sigma S_f)^-1 = V diag(1 / (w - sigma)) V^H
// from the S_f-orthonormal eigenvectors V of the pencil.
__global__ void __launch_bounds__(256) minv_kernel(const double2* __restrict__ V, const double* __restrict__ w,
                                                   double sigma, double2* __restrict__ m64, float2* __restrict__ m32,
                                                   int m0) {
  const int f = blockIdx.x, mm = m0 * m0;
  const double2* Vf = V + (int64_t)f * mm;
  const double* wf = w + (int64_t)f * m0;
  for (int e = threadIdx.x; e < mm; e += 256) {
    const int mu = e / m0, nu = e % m0;
    double re = 0, im = 0;
    for (int j = 0; j < m0; ++j) {
      const double2 a = Vf[mu * m0 + j], b = Vf[nu * m0 + j];
      const double g = 1.0 / (wf[j] - sigma);
      re += g * (a.x * b.x + a.y * b.y);
      im += g * (a.y * b.x - a.x * b.y);
    }
    m64[(int64_t)f * mm + e] = make_double2(re, im);
    m32[(int64_t)f * mm + e] = make_float2((float)re, (float)im);
  }
}

__global__ void __launch_bounds__(256) to32_kernel(const double2* __restrict__ src, float2* __restrict__ dst,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

__device__ __forceinline__ int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// In-place radix-2 transform of CB columns of length P = 2^bits in LDS, S
// apart (natural-order output from bit-reversed input).  INV: conjugate twiddles.
// Stages go in pairs: a thread takes the four elements i0 + {0, 1, 2, 3} h
// (h = 2^(s-1)) through stage s (pairs (0, 1), (2, 3), twiddle of position p)
// and stage s + 1 (pairs (0, 2), (1, 3), twiddles of p and p + h), one barrier
// and one LDS pass per pair; an odd last stage runs alone.  Every index is a
// shift or a mask.
template <typename C, bool INV>
__device__ __forceinline__ C fft_tw(const C* __restrict__ tw, int k) {
  C w = tw[k];
  if (INV) w.y = -w.y;
  return w;
}
template <typename C>
__device__ __forceinline__ C fft_mul(C a, C w) {
  C v;
  v.x = a.x * w.x - a.y * w.y;
  v.y = a.x * w.y + a.y * w.x;
  return v;
}
template <typename C>
__device__ __forceinline__ void fft_bfly(C& a, C& b, C w) {
  const C v = fft_mul(b, w);
  b.x = a.x - v.x;
  b.y = a.y - v.y;
  a.x = a.x + v.x;
  a.y = a.y + v.y;
}
template <typename C, bool INV>
__device__ void fft_lds(C* a, int P, int S, int bits, int CB, const C* __restrict__ tw) {
  int s = 1;
  for (; s + 1 <= bits; s += 2) {
    const int half = 1 << (s - 1), qb = bits - 2;   // P / 4 = 2^qb groups of four per column
    for (int q = threadIdx.x; q < (CB << qb); q += blockDim.x) {
      const int cc = q >> qb, qq = q & ((1 << qb) - 1);
      const int grp = qq >> (s - 1), pos = qq & (half - 1);
      C* col = a + cc * S + (grp << (s + 1)) + pos;
      C x0 = col[0], x1 = col[half], x2 = col[2 * half], x3 = col[3 * half];
      const C w = fft_tw<C, INV>(tw, pos << (bits - s));
      fft_bfly(x0, x1, w);
      fft_bfly(x2, x3, w);
      fft_bfly(x0, x2, fft_tw<C, INV>(tw, pos << (bits - s - 1)));
      fft_bfly(x1, x3, fft_tw<C, INV>(tw, (pos + half) << (bits - s - 1)));
      col[0] = x0;
      col[half] = x1;
      col[2 * half] = x2;
      col[3 * half] = x3;
    }
    __syncthreads();
  }
  if (s == bits) {
    const int hb = bits - 1, half = 1 << (s - 1);
    for (int b = threadIdx.x; b < (CB << hb); b += blockDim.x) {
      const int cc = b >> hb, bb = b & ((1 << hb) - 1);
      const int grp = bb >> (s - 1), pos = bb & (half - 1);
      C* col = a + cc * S + (grp << s) + pos;
      C x0 = col[0], x1 = col[half];
      fft_bfly(x0, x1, fft_tw<C, INV>(tw, pos << (bits - s)));
      col[0] = x0;
      col[half] = x1;
    }
    __syncthreads();
  }
}

// Forward transform over the cell index of columns c = mu ncols + j of x
// ([N][ld], FP64 or FP32 entries IO) zero-padded to P; output xhat[f][mu][j].
template <typename R, typename IO>
__global__ void __launch_bounds__(256) fft_fwd_kernel(int L, int m0, int P, int bits, int ncols, int CB,
                                                      const IO* __restrict__ x, int ld,
                                                      const typename Cx<R>::T* __restrict__ tw,
                                                      typename Cx<R>::T* __restrict__ xhat) {
  typedef typename Cx<R>::T C;
  extern __shared__ char lraw[];
  C* a = reinterpret_cast<C*>(lraw);
  const int ncol = m0 * ncols;
  const int c0 = blockIdx.x * CB;
  // the workgroup's CB columns are adjacent in x and in xhat, so consecutive
  // threads take consecutive columns (CB is a power of two); columns sit
  // S = P + 1 apart in LDS, off one bank
  const int cbits = __builtin_ctz(CB), S = P + 1;
  for (int e = threadIdx.x; e < CB * P; e += 256) {
    const int cc = e & (CB - 1), k = e >> cbits, c = c0 + cc;
    C v;
    v.x = 0;
    v.y = 0;
    if (c < ncol && k < L) {
      const int mu = c / ncols, j = c % ncols;
      v.x = (R)x[((int64_t)k * m0 + mu) * ld + j];
    }
    a[cc * S + bitrev(k, bits)] = v;
  }
  __syncthreads();
  fft_lds<C, false>(a, P, S, bits, CB, tw);
  for (int e = threadIdx.x; e < CB * P; e += 256) {
    const int cc = e & (CB - 1), f = e >> cbits, c = c0 + cc;
    if (c < ncol) xhat[(int64_t)f * ncol + c] = a[cc * S + f];
  }
}

// Per-frequency products yhat_f = op_f xhat_f (op_f m0 x m0), one or two
// operators (grid y).
template <typename R>
__global__ void __launch_bounds__(256) freq_mul_kernel(int m0, int ncols, const typename Cx<R>::T* __restrict__ opH,
                                                       const typename Cx<R>::T* __restrict__ opS,
                                                       const typename Cx<R>::T* __restrict__ xhat,
                                                       typename Cx<R>::T* __restrict__ yH,
                                                       typename Cx<R>::T* __restrict__ yS) {
  typedef typename Cx<R>::T C;
  extern __shared__ char lraw[];
  C* op = reinterpret_cast<C*>(lraw);          // [m0][m0]
  C* xs = op + m0 * m0;                        // [m0][ncols]
  const int f = blockIdx.x;
  const C* o = (blockIdx.y == 0 ? opH : opS) + (int64_t)f * m0 * m0;
  C* y = (blockIdx.y == 0 ? yH : yS) + (int64_t)f * m0 * ncols;
  const C* xf = xhat + (int64_t)f * m0 * ncols;
  for (int e = threadIdx.x; e < m0 * m0; e += 256) op[e] = o[e];
  for (int e = threadIdx.x; e < m0 * ncols; e += 256) xs[e] = xf[e];
  __syncthreads();
  for (int e = threadIdx.x; e < m0 * ncols; e += 256) {
    const int mu = e / ncols, j = e % ncols;
    R re = 0, im = 0;
    for (int nu = 0; nu < m0; ++nu) {
      const C a = op[mu * m0 + nu], b = xs[nu * ncols + j];
      re += a.x * b.x - a.y * b.y;
      im += a.x * b.y + a.y * b.x;
    }
    C r;
    r.x = re;
    r.y = im;
    y[e] = r;
  }
}

// Inverse transform of yhat[f][mu][j] and the first L blocks, real part / P,
// into y ([N][ld], entries IO); grid y selects the operator.
template <typename R, typename IO>
__global__ void __launch_bounds__(256) fft_inv_kernel(int L, int m0, int P, int bits, int ncols, int CB,
                                                      const typename Cx<R>::T* __restrict__ tw,
                                                      const typename Cx<R>::T* __restrict__ yhH,
                                                      const typename Cx<R>::T* __restrict__ yhS,
                                                      IO* __restrict__ yH, IO* __restrict__ yS, int ld) {
  typedef typename Cx<R>::T C;
  extern __shared__ char lraw[];
  C* a = reinterpret_cast<C*>(lraw);
  const int ncol = m0 * ncols;
  const int c0 = blockIdx.x * CB;
  const C* src = blockIdx.y == 0 ? yhH : yhS;
  IO* y = blockIdx.y == 0 ? yH : yS;
  // consecutive threads take consecutive (adjacent) columns, as in the forward kernel
  const int cbits = __builtin_ctz(CB), S = P + 1;
  for (int e = threadIdx.x; e < CB * P; e += 256) {
    const int cc = e & (CB - 1), f = e >> cbits, c = c0 + cc;
    C v;
    v.x = 0;
    v.y = 0;
    if (c < ncol) v = src[(int64_t)f * ncol + c];
    a[cc * S + bitrev(f, bits)] = v;
  }
  __syncthreads();
  fft_lds<C, true>(a, P, S, bits, CB, tw);
  const double inv = 1.0 / P;
  for (int e = threadIdx.x; e < CB * L; e += 256) {
    const int cc = e & (CB - 1), k = e >> cbits, c = c0 + cc;
    if (c < ncol) {
      const int mu = c / ncols, j = c % ncols;
      y[((int64_t)k * m0 + mu) * ld + j] = (IO)((double)a[cc * S + k].x * inv);
    }
  }
}

constexpr int kCrossJ = 32;                    // columns per workgroup
constexpr int kCrossMG = 8;                    // row groups: thread group g owns rows g, g + 8, ...
constexpr int kCrossAcc = kMaxM0 / kCrossMG;   // rows per thread

// y_k += sum over the entries q of row r of D_q x_{m_q} for the affected block
// row k = row_cell[r] (grid: rows, column chunks of kCrossJ, H / S); SET: y_k =
// the sum (the block-sparse product of the exact box operator).  Per entry
// the workgroup stages D_q (m0 x m0) and the chunk's columns of the m0 rows of
// block m_q of x in LDS; thread (j, g) accumulates rows g, g + 8, ... of
// column j over the entries in order, in FP64 for either I/O type IO.
template <bool SET, typename IO>
__global__ void __launch_bounds__(256) cross_apply_kernel(int m0, int ncols, const IO* __restrict__ x, int ld,
                                                          const int32_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ row_cell,
                                                          const CrossEntry* __restrict__ ent,
                                                          const double* __restrict__ dH,
                                                          const double* __restrict__ dS, IO* __restrict__ yH,
                                                          IO* __restrict__ yS) {
  __shared__ double xs[kMaxM0][kCrossJ];
  __shared__ double ds[kMaxM0][kMaxM0 + 1];
  const int r = blockIdx.x, k = row_cell[r], j0 = blockIdx.y * kCrossJ;
  const double* Dm = blockIdx.z == 0 ? dH : dS;
  IO* y = blockIdx.z == 0 ? yH : yS;
  const int jl = threadIdx.x % kCrossJ, g = threadIdx.x / kCrossJ, j = j0 + jl;
  const int mm = m0 * m0;
  double acc[kCrossAcc];
#pragma unroll
  for (int t = 0; t < kCrossAcc; ++t) acc[t] = 0.0;
  // the next entry's D_q and x block are fetched into registers while the
  // current one is used
  constexpr int kFD = kMaxM0 * kMaxM0 / 256, kFX = kMaxM0 * kCrossJ / 256;
  double rd[kFD], rx[kFX];
  auto fetch = [&](int q) {
    const int m = ent[q].m;
    const double* d = Dm + (int64_t)q * mm;
#pragma unroll
    for (int u = 0; u < kFD; ++u) {
      const int e = threadIdx.x + 256 * u;
      rd[u] = e < mm ? d[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kFX; ++u) {
      const int e = threadIdx.x + 256 * u, nu = e / kCrossJ, jj = e % kCrossJ;
      rx[u] = e < m0 * kCrossJ && j0 + jj < ncols ? (double)x[((int64_t)m * m0 + nu) * ld + j0 + jj] : 0.0;
    }
  };
  const int qa = row_ptr[r], qe = row_ptr[r + 1];
  if (qa < qe) fetch(qa);
  for (int q = qa; q < qe; ++q) {
#pragma unroll
    for (int u = 0; u < kFD; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < mm) ds[e / m0][e % m0] = rd[u];
    }
#pragma unroll
    for (int u = 0; u < kFX; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < m0 * kCrossJ) xs[e / kCrossJ][e % kCrossJ] = rx[u];
    }
    __syncthreads();
    if (q + 1 < qe) fetch(q + 1);
    for (int nu = 0; nu < m0; ++nu) {
      const double xv = xs[nu][jl];
#pragma unroll
      for (int t = 0; t < kCrossAcc; ++t) {
        const int mu = g + kCrossMG * t;
        if (mu < m0) acc[t] += ds[mu][nu] * xv;
      }
    }
    __syncthreads();
  }
  if (j < ncols) {
#pragma unroll
    for (int t = 0; t < kCrossAcc; ++t) {
      const int mu = g + kCrossMG * t;
      if (mu < m0) {
        IO* yp = y + ((int64_t)k * m0 + mu) * ld + j;
        *yp = (IO)(SET ? acc[t] : (double)*yp + acc[t]);
      }
    }
  }
}

template <typename R, typename IO>
hipError_t apply_t(int L, int m0, int P, int ncols, const IO* x, int ld, const void* opH, const void* opS,
                   const void* tw, void* xhat, void* yhH, void* yhS, IO* yH, IO* yS, hipStream_t s) {
  typedef typename Cx<R>::T C;
  int bits = 0;
  while ((1 << bits) < P) ++bits;
  const int CB = std::max(1, std::min(16, 65536 / (P * (int)sizeof(C))));   // a power of two (P is)
  const int ncol = m0 * ncols;
  const unsigned gx = (unsigned)((ncol + CB - 1) / CB);
  const size_t lds = (size_t)CB * (P + 1) * sizeof(C);   // columns P + 1 apart
  const int nops = opS ? 2 : 1;
  (void)hipFuncSetAttribute((const void*)fft_fwd_kernel<R, IO>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)hipFuncSetAttribute((const void*)fft_inv_kernel<R, IO>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((fft_fwd_kernel<R, IO>), dim3(gx), dim3(256), lds, s, L, m0, P, bits, ncols, CB, x, ld,
                     (const C*)tw, (C*)xhat);
  const size_t lm = sizeof(C) * ((size_t)m0 * m0 + (size_t)m0 * ncols);
  (void)hipFuncSetAttribute((const void*)freq_mul_kernel<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lm);
  hipLaunchKernelGGL((freq_mul_kernel<R>), dim3(P, nops), dim3(256), lm, s, m0, ncols, (const C*)opH,
                     (const C*)opS, (const C*)xhat, (C*)yhH, (C*)yhS);
  hipLaunchKernelGGL((fft_inv_kernel<R, IO>), dim3(gx, nops), dim3(256), lds, s, L, m0, P, bits, ncols, CB,
                     (const C*)tw, (const C*)yhH, (const C*)yhS, yH, yS, ld);
  return hipGetLastError();
}

}  // namespace

hipError_t toep_launch_vrep(const ToepDev* d, double* vrep, int M0R, int nc, hipStream_t s) {
  (void)nc;
  hipLaunchKernelGGL(vrep_kernel, dim3(M0R), dim3(256), 0, s, d, vrep);
  return hipGetLastError();
}

hipError_t toep_launch_transverse(const ToepDev* d, const Defect* defs, const ScalePair* pairs, int npairs, int m0,
                                  int M0R, double* trans, hipStream_t s) {
  // LDS: factors of both cells over a chunk with halo, potential rows of a chunk
  const size_t lds = sizeof(double) * (2 * (size_t)m0 * (kTChunk + 2) + (size_t)M0R * kTChunk);
  (void)hipFuncSetAttribute((const void*)transverse_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(transverse_kernel, dim3(npairs, 2), dim3(256), lds, s, d, defs, pairs, trans);
  return hipGetLastError();
}

hipError_t toep_launch_vbox(const ToepDev* d, const Defect* defs, const int32_t* cell_def, double* vbox, int M0R,
                            int n, hipStream_t s) {
  hipLaunchKernelGGL(vbox_kernel, dim3(M0R, (n + 255) / 256), dim3(256), 0, s, d, defs, cell_def, vbox);
  return hipGetLastError();
}

hipError_t toep_launch_blocks(const ToepDev* d, const Defect* defs, const ToepJob* jobs, int njobs, int m0,
                                int wmax, const double* vrep, const double* vbox, const double* trans, double* outH,
                                double* outS, hipStream_t s) {
  const size_t lds = sizeof(double) * (2 * (size_t)m0 * (wmax + 2) + (size_t)wmax);
  (void)hipFuncSetAttribute((const void*)block_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(block_kernel, dim3(njobs), dim3(256), lds, s, d, defs, jobs, vrep, vbox, trans, outH, outS);
  return hipGetLastError();
}

hipError_t toep_launch_delta(const ToepDev* d, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                             const CrossEntry* ent, const double* genH, const double* genS, const double* crossH,
                             const double* crossS, double* dH, double* dS, int m0, hipStream_t s) {
  (void)d;
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(delta_kernel, dim3(nrows), dim3(256), 0, s, row_ptr, row_cell, ent, genH, genS, crossH, crossS,
                     dH, dS, m0);
  return hipGetLastError();
}

hipError_t toep_launch_chat(const ToepDev* d, const double* genH, const double* genS, double2* cH, double2* cS,
                            int m0, int P, int L0, hipStream_t s) {
  (void)d;
  hipLaunchKernelGGL(chat_kernel, dim3(P), dim3(256), 0, s, genH, genS, cH, cS, m0, P, L0);
  return hipGetLastError();
}

hipError_t toep_launch_minv(const double2* V, const double* w, double sigma, double2* minv64, float2* minv32, int P,
                            int m0, hipStream_t s) {
  hipLaunchKernelGGL(minv_kernel, dim3(P), dim3(256), 0, s, V, w, sigma, minv64, minv32, m0);
  return hipGetLastError();
}

hipError_t toep_launch_to32(const double2* src, float2* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename IO>
static hipError_t launch_apply_io(int prec, int L, int m0, int P, int ncols, const IO* x, int ld, const void* opH,
                                  const void* opS, const void* tw, void* xhat, void* yhatH, void* yhatS, IO* yH,
                                  IO* yS, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                                  const CrossEntry* ent, const double* dH, const double* dS, hipStream_t s,
                                  bool exact) {
  const dim3 grid(nrows, (ncols + kCrossJ - 1) / kCrossJ, (exact ? yS : opS) ? 2 : 1);
  if (exact) {
    hipLaunchKernelGGL((cross_apply_kernel<true, IO>), grid, dim3(256), 0, s, m0, ncols, x, ld, row_ptr, row_cell,
                       ent, dH, dS, yH, yS);
    return hipGetLastError();
  }
  hipError_t e = prec == LHF_PREC_FP64
                     ? apply_t<double, IO>(L, m0, P, ncols, x, ld, opH, opS, tw, xhat, yhatH, yhatS, yH, yS, s)
                     : apply_t<float, IO>(L, m0, P, ncols, x, ld, opH, opS, tw, xhat, yhatH, yhatS, yH, yS, s);
  if (e != hipSuccess || nrows == 0) return e;
  hipLaunchKernelGGL((cross_apply_kernel<false, IO>), grid, dim3(256), 0, s, m0, ncols, x, ld, row_ptr, row_cell,
                     ent, dH, dS, yH, yS);
  return hipGetLastError();
}

hipError_t toep_launch_apply(int prec, int L, int m0, int P, int ncols, const double* x, int ld, const void* opH,
                             const void* opS, const void* tw, void* xhat, void* yhatH, void* yhatS, double* yH,
                             double* yS, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                             const CrossEntry* ent, const double* dH, const double* dS, hipStream_t s, bool exact) {
  return launch_apply_io<double>(prec, L, m0, P, ncols, x, ld, opH, opS, tw, xhat, yhatH, yhatS, yH, yS, row_ptr,
                                 row_cell, nrows, ent, dH, dS, s, exact);
}

hipError_t toep_launch_apply32(int L, int m0, int P, int ncols, const float* x, int ld, const void* opH,
                               const void* opS, const void* tw, void* xhat, void* yhatH, void* yhatS, float* yH,
                               float* yS, const int32_t* row_ptr, const int32_t* row_cell, int nrows,
                               const CrossEntry* ent, const double* dH, const double* dS, hipStream_t s, bool exact) {
  return launch_apply_io<float>(LHF_PREC_MIXED, L, m0, P, ncols, x, ld, opH, opS, tw, xhat, yhatH, yhatS, yH, yS,
                                row_ptr, row_cell, nrows, ent, dH, dS, s, exact);
}

}  // namespace lhf
