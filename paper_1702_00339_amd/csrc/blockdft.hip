// Block diagonalisation by a Fourier transform over the lattice index
// (Lemma 3.1, Prop. 5.1):
//   Hbar_j = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) A_k,  w_l = exp(-2 pi i / L_l)
// applied entry-wise to the m0 x m0 generator blocks.
//
// The generators vanish outside the band (offsets beyond L0 in a banded
// dimension), so the transform is done one dimension at a time as a pruned
// DFT: the first pass reads only band cells of the real stack and transforms
// the last non-trivial dimension; each later pass transforms the next
// dimension of a complex intermediate [outer band slots][slots][inner] into
// [outer band slots][L][inner].  Inner indices (the m0^2 block entries and the
// dimensions already transformed) are contiguous, so every load and store is
// coalesced; each output entry costs (band width) complex multiply-adds per
// pass.  H and S are transformed in the same launch (grid y).
//
// Grouped launches: one launch per pass and band-width class covers every
// lattice of the plan through a task table (one task per lattice and pass);
// each task's thread range starts at a multiple of 256, so a workgroup
// serves one task, found by binary search over the table.
#include <algorithm>

#include "plan.h"

namespace lhf {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { typedef double2 T; };
template <> struct Cx<float> { typedef float2 T; };

constexpr int kLdsTwiddles = 2048;   // longest axis whose twiddles are staged in LDS

__host__ __device__ __forceinline__ int slot_cell(const DimDev& D, int s) {
  if (D.full) return s;
  int k = s - D.L0;
  return k < 0 ? k + D.L : k;
}

// Element of the half layout [L1][L2][L3/2+1][m0][m0] (the Hermitian
// half-space along k3: the blocks j3 > L3/2 are conjugates of kept ones) for
// the full-layout element `flat` of lattice L, or -1 for j3 > L3/2.
__device__ __forceinline__ int64_t half_index(const LatDev& L, int64_t flat) {
  const int L3 = L.L[2];
  if (L3 == 1) return flat;
  const int E = L.m0 * L.m0, L3h = L3 / 2 + 1;
  const int64_t q = flat / E, r = q / L3;
  const int e = (int)(flat - q * E), j3 = (int)(q - r * L3);
  return j3 < L3h ? (r * L3h + j3) * E + e : -1;
}

__host__ __device__ __forceinline__ int nslot(const DimDev& D) { return D.L == 1 ? 1 : D.nshift; }

__device__ __forceinline__ int find_task(const DftTask* __restrict__ tasks, int ntasks, int64_t wg0) {
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tbase <= wg0) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One pass of the pruned DFT.  Thread t of a task owns one input column
// (o, i) and a chunk of JC outputs j along the transformed axis: it loads the
// column's B band inputs once into registers and writes
//   Y[o][j][i] = sum_b w^(j k_b) X[o][b][i],  k_b the lattice offset of slot b
// for its JC values of j (twiddle indices advance by k_b per j, 32-bit).
// FIRST: X is the real generator stack, band-gathered over the outer dims
// (o enumerates their slots) with inner index i = block entry.
template <typename R, int BMAX, bool FIRST>
__global__ void __launch_bounds__(256) dft_pass_kernel(const LatDev* __restrict__ lats,
                                                       const DftTask* __restrict__ tasks, int ntasks,
                                                       const typename Cx<R>::T* __restrict__ tw,
                                                       const R* __restrict__ genH, const R* __restrict__ genS,
                                                       typename Cx<R>::T* __restrict__ tmp,
                                                       typename Cx<R>::T* __restrict__ barH,
                                                       typename Cx<R>::T* __restrict__ barS,
                                                       float2* __restrict__ b32H, float2* __restrict__ b32S,
                                                       int half) {
  typedef typename Cx<R>::T C;
  const int64_t wg0 = (int64_t)blockIdx.x * 256;
  const DftTask T = tasks[find_task(tasks, ntasks, wg0)];
  const LatDev& L = lats[T.li];
  const int d = T.d;
  const DimDev& D = L.dim[d];
  const int Ld = D.L, B = T.B, I = T.I, JC = T.JC, njc = T.njc;
  // twiddle table staged in LDS when the launch gives room for it
  extern __shared__ char lds_raw[];
  C* sT = reinterpret_cast<C*>(lds_raw);
  const bool lds_tw = Ld <= kLdsTwiddles;
  if (lds_tw) {
    for (int q = threadIdx.x; q < Ld; q += 256) sT[q] = tw[D.tw_off + q];
    __syncthreads();
  }
  const int tid = (int)(wg0 - T.tbase) + threadIdx.x;
  if (tid >= T.O * njc * I) return;
  const int i = tid % I;
  const int jc = (tid / I) % njc;
  const int o = tid / (I * njc);
  const bool isH = blockIdx.y == 0;
  R xr[BMAX], xi[BMAX];
  int kb[BMAX];
  if constexpr (FIRST) {
    const R* X = (isH ? genH : genS) + L.gen_off;
    const int E = L.m0 * L.m0;
    int kk[3] = {0, 0, 0};
    int oo = o;
    for (int q = d - 1; q >= 0; --q) {
      const int ns = nslot(L.dim[q]);
      kk[q] = slot_cell(L.dim[q], oo % ns);
      oo /= ns;
    }
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
      if (b < B) {
        kk[d] = slot_cell(D, b);
        kb[b] = kk[d];
        const int cell = (kk[0] * L.L[1] + kk[1]) * L.L[2] + kk[2];
        xr[b] = X[cell * E + i];
        xi[b] = R(0);
      }
    }
  } else {
    const C* X = tmp + T.in_off + (isH ? 0 : T.in_half) + (int64_t)o * B * I + i;
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
      if (b < B) {
        kb[b] = slot_cell(D, b);
        const C x = X[(int64_t)b * I];
        xr[b] = x.x;
        xi[b] = x.y;
      }
    }
  }
  const int j0 = jc * JC;
  const int j1 = min(Ld, j0 + JC);
  int idx[BMAX];
#pragma unroll
  for (int b = 0; b < BMAX; ++b)
    if (b < B) idx[b] = (j0 * kb[b]) % Ld;
  const C* Tw = lds_tw ? sT : tw + D.tw_off;
  const bool hout = half && T.out_final;   // final blocks in the half layout
  C* Y = T.out_final ? (isH ? barH : barS) + (hout ? L.half_off : L.gen_off)
                     : tmp + T.out_off + (isH ? 0 : T.out_half);
  const int64_t f0 = (int64_t)o * Ld * I + i;
  C* dst = Y + f0;
  // complex64 copy of final blocks (the FP64 transform of the mixed pipeline)
  float2* d32 = (T.out_final && b32H) ? (isH ? b32H : b32S) + L.gen_off + (int64_t)o * Ld * I + i : nullptr;
  for (int j = j0; j < j1; ++j) {
    R re = 0, im = 0;
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
      if (b < B) {
        const C w = Tw[idx[b]];
        re += w.x * xr[b] - w.y * xi[b];
        im += w.x * xi[b] + w.y * xr[b];
        idx[b] += kb[b];
        if (idx[b] >= Ld) idx[b] -= Ld;
      }
    }
    C r;
    r.x = re;
    r.y = im;
    if (hout) {
      const int64_t h = half_index(L, f0 + (int64_t)j * I);
      if (h >= 0) Y[h] = r;
    } else {
      dst[(int64_t)j * I] = r;
    }
    if (d32) d32[(int64_t)j * I] = make_float2((float)re, (float)im);
  }
}

// Bands wider than 32 slots: one thread per output (tasks with JC = 1).
template <typename R, bool FIRST>
__global__ void __launch_bounds__(256) dft_wide_kernel(const LatDev* __restrict__ lats,
                                                       const DftTask* __restrict__ tasks, int ntasks,
                                                       const typename Cx<R>::T* __restrict__ tw,
                                                       const R* __restrict__ genH, const R* __restrict__ genS,
                                                       typename Cx<R>::T* __restrict__ tmp,
                                                       typename Cx<R>::T* __restrict__ barH,
                                                       typename Cx<R>::T* __restrict__ barS,
                                                       float2* __restrict__ b32H, float2* __restrict__ b32S,
                                                       int half) {
  typedef typename Cx<R>::T C;
  const int64_t wg0 = (int64_t)blockIdx.x * 256;
  const DftTask T = tasks[find_task(tasks, ntasks, wg0)];
  const LatDev& L = lats[T.li];
  const int d = T.d;
  const DimDev& D = L.dim[d];
  const int Ld = D.L, B = T.B, I = T.I;
  const int tid = (int)(wg0 - T.tbase) + threadIdx.x;
  if (tid >= T.O * Ld * I) return;
  const int i = tid % I;
  const int j = (tid / I) % Ld;
  const int o = tid / (I * Ld);
  const bool isH = blockIdx.y == 0;
  const C* Tw = tw + D.tw_off;
  R re = 0, im = 0;
  int kk[3] = {0, 0, 0};
  if (FIRST) {
    int oo = o;
    for (int q = d - 1; q >= 0; --q) {
      const int ns = nslot(L.dim[q]);
      kk[q] = slot_cell(L.dim[q], oo % ns);
      oo /= ns;
    }
  }
  const C* Xc = tmp + T.in_off + (isH ? 0 : T.in_half) + (int64_t)o * B * I + i;
  const R* Xr = (isH ? genH : genS) + L.gen_off;
  for (int b = 0; b < B; ++b) {
    const int k = slot_cell(D, b);
    const C w = Tw[(int)(((int64_t)j * k) % Ld)];
    R xr, xi;
    if (FIRST) {
      kk[d] = k;
      const int cell = (kk[0] * L.L[1] + kk[1]) * L.L[2] + kk[2];
      xr = Xr[(int64_t)cell * L.m0 * L.m0 + i];
      xi = R(0);
    } else {
      const C x = Xc[(int64_t)b * I];
      xr = x.x;
      xi = x.y;
    }
    re += w.x * xr - w.y * xi;
    im += w.x * xi + w.y * xr;
  }
  const bool hout = half && T.out_final;   // final blocks in the half layout
  C* Y = T.out_final ? (isH ? barH : barS) + (hout ? L.half_off : L.gen_off)
                     : tmp + T.out_off + (isH ? 0 : T.out_half);
  C r;
  r.x = re;
  r.y = im;
  if (hout) {
    const int64_t h = half_index(L, tid);
    if (h >= 0) Y[h] = r;
  } else {
    Y[tid] = r;
  }
  if (T.out_final && b32H) ((isH ? b32H : b32S) + L.gen_off)[tid] = make_float2((float)re, (float)im);
}

constexpr int kFusedEC = 8;    // block entries per fused workgroup
constexpr int kFusedJ2 = 16;   // j2 values per fused workgroup

__device__ __forceinline__ int find_fused(const FusedTask* __restrict__ t, int n, int64_t wg) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].wg_base <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Last stage of the fused transforms: the outputs j1 = j + q Q (q < R1,
// Q = L1 / R1, R1 = 4, 2 or 1 as L1 allows) share the twiddles w1^(j k1) up
// to zeta^(q k1), zeta = w1^Q = +-i or -1.  The inputs T2[s1][jj][ec] (LDS)
// are summed by slot residue a = s1 mod 4 (k1 = s1 + off mod R1), and Y_q =
// zeta^(q off) sum_a zeta^(q a) S_a: one complex multiply-add per input for R1
// outputs.  A thread owns one (j2, e) column with its B1 inputs in registers
// and walks groups of R1 outputs j1.  Slot cells are consecutive mod L1
// (k1(s1) = k1(0) + s1), so output j's twiddle index j k1(s1) mod L1 starts
// at j k1(0) mod L1 and steps by j from one slot to the next.
template <typename R, int BM>
__device__ __forceinline__ void fused_last_stage(const LatDev& L, int J2C, int j2lo, int j2n, int j3, int e0, int ecn,
                                                 const typename Cx<R>::T* T2, const typename Cx<R>::T* tw1, bool isH,
                                                 typename Cx<R>::T* __restrict__ barH,
                                                 typename Cx<R>::T* __restrict__ barS, float2* __restrict__ b32H,
                                                 float2* __restrict__ b32S, bool half) {
  typedef typename Cx<R>::T C;
  constexpr int EC = kFusedEC;
  const DimDev& D0 = L.dim[0];
  const int L1 = L.L[0], L2 = L.L[1], L3 = L.L[2], B1 = nslot(D0), E = L.m0 * L.m0;
  const int tid = threadIdx.x, ec = tid & (EC - 1);
  const int ncol = J2C * EC, nrep = 256 / ncol;
  const int col = tid % ncol, rep = tid / ncol;
  const int jj = col / EC;
  if (rep >= nrep || jj >= j2n || ec >= ecn) return;
  const int R1 = (L1 & 3) == 0 ? 4 : (L1 & 1) == 0 ? 2 : 1;
  const int Q = L1 / R1;
  const int off = slot_cell(D0, 0) % R1;
  // inputs past the band are zero, so the sums below may run past it in
  // whole groups of four slots (the twiddle index stays in range regardless)
  R xr[BM], xi[BM];
#pragma unroll
  for (int s1 = 0; s1 < BM; ++s1) {
    const C x = T2[(min(s1, B1 - 1) * J2C + jj) * EC + ec];
    xr[s1] = s1 < B1 ? x.x : R(0);
    xi[s1] = s1 < B1 ? x.y : R(0);
  }
  const int k0 = slot_cell(D0, 0);
  int base = (int)(((int64_t)rep * k0) % L1);   // j k1(0) mod L1 for the current j
  const int bstep = (int)(((int64_t)nrep * k0) % L1);
  // full layout [L1][L2][L3][E], or the half layout with L3 / 2 + 1 planes
  // (the caller runs no workgroup for j3 > L3 / 2 then)
  const int L3o = half ? L3 / 2 + 1 : L3;
  const int64_t yoff = (half ? L.half_off : L.gen_off) + ((int64_t)(j2lo + jj) * L3o + j3) * E + e0 + ec;
  C* Y = (isH ? barH : barS) + yoff;
  float2* Y32 = b32H ? (isH ? b32H : b32S) + yoff : nullptr;
  const int64_t jstride = (int64_t)L2 * L3o * E;
  const R zs = tw1[Q % L1].y < R(0) ? R(-1) : R(1);   // zeta = zs i when R1 = 4
  // output j1 = j + q Q sits (j1 - j) jstride past the base output j
  const int64_t ystep = (int64_t)nrep * jstride, qstep = (int64_t)Q * jstride;
  int64_t ybase = (int64_t)rep * jstride;
  auto put = [&](int q, R re, R im) {
    C v;
    v.x = re;
    v.y = im;
    const int64_t o = ybase + q * qstep;
    Y[o] = v;
    if (Y32) Y32[o] = make_float2((float)re, (float)im);
  };
  for (int j = rep; j < Q; j += nrep, ybase += ystep) {
    R sr[4] = {R(0), R(0), R(0), R(0)}, si[4] = {R(0), R(0), R(0), R(0)};
    int ix = base;   // j k1(s1) mod L1; j < Q <= L1
    // opaque, or the compiler keeps one index register per slot across j
    asm volatile("" : "+v"(ix));
    // groups of four slots up to the band (a uniform branch per group, the
    // group's twiddle reads in flight together)
#pragma unroll
    for (int s0 = 0; s0 < BM; s0 += 4) {
      if (s0 < B1) {
#pragma unroll
        for (int s1 = s0; s1 < s0 + 4 && s1 < BM; ++s1) {
          const C w = tw1[ix];
          sr[s1 & 3] += w.x * xr[s1] - w.y * xi[s1];
          si[s1 & 3] += w.x * xi[s1] + w.y * xr[s1];
          ix += j;
          if (ix >= L1) ix -= L1;
        }
      }
    }
    base += bstep;
    if (base >= L1) base -= L1;
    if (R1 == 4) {
      // U_q = sum_a zeta^(q a) S_a; zeta (x + i y) = zs (-y + i x); Y_q = zeta^(q off) U_q
      const R ar = sr[0] + sr[2], ai = si[0] + si[2], br = sr[0] - sr[2], bi = si[0] - si[2];
      const R cr = sr[1] + sr[3], ci = si[1] + si[3], dr = sr[1] - sr[3], di = si[1] - si[3];
      auto rot = [&](int q, R yr, R yi) {
        const int m = (q * off) & 3;
        if (m == 1) { const R tr = -zs * yi; yi = zs * yr; yr = tr; }
        else if (m == 2) { yr = -yr; yi = -yi; }
        else if (m == 3) { const R tr = zs * yi; yi = -zs * yr; yr = tr; }
        put(q, yr, yi);
      };
      rot(0, ar + cr, ai + ci);
      rot(1, br - zs * di, bi + zs * dr);
      rot(2, ar - cr, ai - ci);
      rot(3, br + zs * di, bi - zs * dr);
    } else if (R1 == 2) {
      const R er = sr[0] + sr[2], ei = si[0] + si[2], orr = sr[1] + sr[3], oi = si[1] + si[3];
      put(0, er + orr, ei + oi);
      const R sg = (off & 1) ? R(-1) : R(1);
      put(1, sg * (er - orr), sg * (ei - oi));
    } else {
      put(0, sr[0] + sr[1] + sr[2] + sr[3], si[0] + si[1] + si[2] + si[3]);
    }
  }
}

// Fused transform of all three dimensions of a lattice (band-pruned):
//   stage 1: T1[s1][s2][e] = sum_s3 w3^(j3 k3) A[k1][k2][k3][e]      (fixed j3)
//   stage 2: T2[s1][j2][e] = sum_s2 w2^(j2 k2) T1[s1][s2][e]          (a chunk of j2)
//   stage 3: Y[j1][j2][j3][e] = sum_s1 w1^(j1 k1) T2[s1][j2][e]      (every j1)
// The intermediates stay in LDS; every Fourier block entry is written once,
// in segments of EC consecutive entries.  In stage 3 a thread owns one
// (j2, e) column with its B1 inputs in registers and walks groups of R1
// outputs j1 (radix-R1 output symmetry) with incrementally updated twiddle
// indices.
template <typename R, int BM>
__global__ void __launch_bounds__(256) dft_fused_kernel(const LatDev* __restrict__ lats,
                                                        const FusedTask* __restrict__ tasks, int ntasks,
                                                        const typename Cx<R>::T* __restrict__ tw,
                                                        const R* __restrict__ genH, const R* __restrict__ genS,
                                                        typename Cx<R>::T* __restrict__ barH,
                                                        typename Cx<R>::T* __restrict__ barS,
                                                        float2* __restrict__ b32H, float2* __restrict__ b32S,
                                                        int half) {
  typedef typename Cx<R>::T C;
  extern __shared__ char lds_raw[];
  const int64_t wg = blockIdx.x;
  const FusedTask T = tasks[find_fused(tasks, ntasks, wg)];
  const LatDev& L = lats[T.li];
  const DimDev& D0 = L.dim[0];
  const DimDev& D1 = L.dim[1];
  const DimDev& D2 = L.dim[2];
  const int L1 = L.L[0], L2 = L.L[1], L3 = L.L[2];
  const int B1 = nslot(D0), B2 = nslot(D1), B3 = nslot(D2);
  constexpr int EC = kFusedEC;   // the planner's entry chunk
  constexpr int PS = 256 / EC;     // (s1, s2) or (s1, j2) rows per pass of the workgroup
  const int E = L.m0 * L.m0, J2C = T.J2C;
  int64_t loc = wg - T.wg_base;
  const int eci = (int)(loc % T.nec);
  loc /= T.nec;
  const int j2c = (int)(loc % T.nj2c);
  const int j3 = (int)(loc / T.nj2c);
  if (half && j3 > L3 / 2) return;   // the conjugate half: the whole workgroup
  const int e0 = eci * EC, ecn = min(EC, E - e0);
  const int j2lo = j2c * J2C, j2n = min(J2C, L2 - j2lo);
  C* T1 = reinterpret_cast<C*>(lds_raw);   // [B1][B2][EC]
  C* T2 = T1 + B1 * B2 * EC;               // [B1][J2C][EC]
  C* tw1 = T2 + B1 * J2C * EC;             // [L1]
  C* tw2 = tw1 + L1;                       // [J2C][B2]
  C* tw3 = tw2 + J2C * B2;                 // [B3]
  const int tid = threadIdx.x;
  for (int q = tid; q < L1; q += 256) tw1[q] = tw[D0.tw_off + q];
  for (int q = tid; q < j2n * B2; q += 256) {
    const int jj = q / B2, s2 = q % B2;
    const int k2 = slot_cell(D1, s2);
    tw2[jj * B2 + s2] = tw[D1.tw_off + ((j2lo + jj) * k2) % L2];
  }
  for (int q = tid; q < B3; q += 256) tw3[q] = tw[D2.tw_off + (j3 * slot_cell(D2, q)) % L3];
  __syncthreads();
  const R* X = (blockIdx.y == 0 ? genH : genS) + L.gen_off;
  // stage 1: a thread keeps entry ec = tid mod EC and steps its (s1, s2)
  // row by PS (no divisions in the loop)
  const int ec = tid & (EC - 1);
  {
    int s1 = (tid / EC) / B2, s2 = (tid / EC) % B2;
    const int d1 = PS / B2, d2 = PS % B2;
    for (int row = tid / EC; row < B1 * B2; row += PS) {
      R re = 0, im = 0;
      if (ec < ecn) {
        const int k1 = slot_cell(D0, s1), k2 = slot_cell(D1, s2);
        const R* xp = X + ((int64_t)(k1 * L2 + k2) * L3) * E + e0 + ec;
        // all band loads first (unrolled to the band bound), then the sums
        R xv[BM];
#pragma unroll
        for (int s3 = 0; s3 < BM; ++s3) xv[s3] = s3 < B3 ? xp[(int64_t)slot_cell(D2, s3) * E] : R(0);
#pragma unroll
        for (int s3 = 0; s3 < BM; ++s3) {
          if (s3 < B3) {
            const C w = tw3[s3];
            re += w.x * xv[s3];
            im += w.y * xv[s3];
          }
        }
      }
      C v;
      v.x = re;
      v.y = im;
      T1[row * EC + ec] = v;
      s2 += d2;
      s1 += d1;
      if (s2 >= B2) { s2 -= B2; ++s1; }
    }
  }
  __syncthreads();
  // stage 2: rows (s1, jj) stepped the same way
  {
    int s1 = (tid / EC) / j2n, jj = (tid / EC) % j2n;
    const int d1 = PS / j2n, d2 = PS % j2n;
    for (int row = tid / EC; row < B1 * j2n; row += PS) {
      R re = 0, im = 0;
      const C* wp = tw2 + jj * B2;
      const C* xp = T1 + s1 * B2 * EC + ec;
      for (int s2 = 0; s2 < B2; ++s2) {
        const C w = wp[s2], x = xp[s2 * EC];
        re += w.x * x.x - w.y * x.y;
        im += w.x * x.y + w.y * x.x;
      }
      C v;
      v.x = re;
      v.y = im;
      T2[(s1 * J2C + jj) * EC + ec] = v;
      jj += d2;
      s1 += d1;
      if (jj >= j2n) { jj -= j2n; ++s1; }
    }
  }
  __syncthreads();
  // stage 3: every j1 of the band's columns
  fused_last_stage<R, BM>(L, J2C, j2lo, j2n, j3, e0, ecn, T2, tw1, blockIdx.y == 0, barH, barS, b32H, b32S,
                          half != 0);
}

int band_class(int B) { return B <= 4 ? 0 : B <= 8 ? 1 : B <= 16 ? 2 : B <= 32 ? 3 : 4; }

template <typename R>
hipError_t dft_launch_all(const lhf_plan_s* p, const R* gH, const R* gS, typename Cx<R>::T* bH,
                          typename Cx<R>::T* bS, typename Cx<R>::T* tmp, const typename Cx<R>::T* tw,
                          float2* b32H, float2* b32S, bool half, hipStream_t s) {
  const int hf = half ? 1 : 0;
  typedef typename Cx<R>::T C;
  if (p->n_fused > 0) {
    const dim3 grid((unsigned)p->fused_wgs, 2);
    const size_t shb = (size_t)p->fused_lds / 16 * sizeof(C);
    if (p->fused_bmax <= 8)
      hipLaunchKernelGGL((dft_fused_kernel<R, 8>), grid, dim3(256), shb, s, p->d_lat, p->d_fused, p->n_fused, tw, gH,
                         gS, bH, bS, b32H, b32S, hf);
    else if (p->fused_bmax <= 16)
      hipLaunchKernelGGL((dft_fused_kernel<R, 16>), grid, dim3(256), shb, s, p->d_lat, p->d_fused, p->n_fused, tw, gH,
                         gS, bH, bS, b32H, b32S, hf);
    else
      hipLaunchKernelGGL((dft_fused_kernel<R, 32>), grid, dim3(256), shb, s, p->d_lat, p->d_fused, p->n_fused, tw, gH,
                         gS, bH, bS, b32H, b32S, hf);
  }
  for (const DftLaunch& l : p->dft_launches) {
    const dim3 grid((unsigned)(l.threads / 256), 2);
    const DftTask* tk = p->d_dft_tasks + l.t0;
    const size_t shb = sizeof(C) * (size_t)l.lds_tw;
    const bool first = l.pass == 0;
#define LHF_PASS(BM)                                                                                      \
  if (first)                                                                                              \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, true>), grid, dim3(256), shb, s, p->d_lat, tk, l.nt, tw,   \
                       gH, gS, tmp, bH, bS, b32H, b32S, hf);                                                           \
  else                                                                                                    \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, false>), grid, dim3(256), shb, s, p->d_lat, tk, l.nt, tw,  \
                       gH, gS, tmp, bH, bS, b32H, b32S, hf);
    switch (l.cls) {
      case 0: LHF_PASS(4) break;
      case 1: LHF_PASS(8) break;
      case 2: LHF_PASS(16) break;
      case 3: LHF_PASS(32) break;
      default:
        if (first)
          hipLaunchKernelGGL((dft_wide_kernel<R, true>), grid, dim3(256), 0, s, p->d_lat, tk, l.nt, tw, gH, gS,
                             tmp, bH, bS, b32H, b32S, hf);
        else
          hipLaunchKernelGGL((dft_wide_kernel<R, false>), grid, dim3(256), 0, s, p->d_lat, tk, l.nt, tw, gH, gS,
                             tmp, bH, bS, b32H, b32S, hf);
    }
#undef LHF_PASS
  }
  return hipGetLastError();
}

// Separable formation of the Fourier blocks (Theorem 3.3, Remark 3.5).  The
// generator is a sum of Hadamard products of 1D Grams (eqs. BC-Core,
// BC-mass, BC-Laplace),
//   S_k = S1[k1] o S2[k2] o S3[k3],
//   H_k = 1/2 (K1 o S2 o S3 + S1 o K2 o S3 + S1 o S2 o K3) - sum_t M1_t o M2_t o M3_t,
// so its transform over dimensions 2 and 3 is the same expression in the
// 1D-transformed Grams G^_l[j] = sum_s w_l^(j k_s) G_l[s] (complex, small):
//   T2[s1](j2, j3) = 1/2 (K1[s1] P_ss + S1[s1] P_ks) - sum_t M1_t[s1] P_t,
//   P_ss = S^2 S^3,  P_ks = K^2 S^3 + S^2 K^3,  P_t = M^2_t M^3_t,
// and the last stage transforms dimension 1 as in the fused kernel.  No
// generator stack is formed or read; every Fourier block is written once.

constexpr int kGhBatch = 16;   // slots of a transformed Gram entry loaded together

// G^ along dimensions 2 and 3: gh[t][j][e] = sum over slots s of w^(j k_s) G[t][s][e]
__global__ void __launch_bounds__(256) gram_dft_kernel(const LatDev* __restrict__ lats,
                                                       const GhItem* __restrict__ items, int nitems,
                                                       const double* __restrict__ grams,
                                                       const double2* __restrict__ tw, double2* __restrict__ gh) {
  const int64_t wg0 = (int64_t)blockIdx.x * 256;
  int lo = 0, hi = nitems - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].start <= wg0) lo = mid; else hi = mid - 1;
  }
  const GhItem it = items[lo];
  const LatDev& L = lats[it.li];
  const DimDev& D = L.dim[it.d];
  const int m2 = L.m0 * L.m0;
  const int64_t idx = wg0 - it.start + threadIdx.x;
  if (idx >= (int64_t)L.T * D.L * m2) return;
  const int e = (int)(idx % m2);
  const int j = (int)((idx / m2) % D.L);
  const int t = (int)(idx / ((int64_t)m2 * D.L));
  double re = 0.0, im = 0.0;
  const int ns = nslot(D);
  const double* gp = grams + D.gram_off + (int64_t)t * D.nshift * m2 + e;
  const double2* wt = tw + D.tw_off;
  // slot cells are consecutive mod L, so the twiddle index j k_s mod L
  // starts at j k_0 mod L and steps by j (< L); the loads of kGhBatch slots
  // are in flight together
  int ix = (int)(((int64_t)j * slot_cell(D, 0)) % D.L);
  for (int s0 = 0; s0 < ns; s0 += kGhBatch) {
    double2 w[kGhBatch];
    double g[kGhBatch];
#pragma unroll
    for (int u = 0; u < kGhBatch; ++u) {
      w[u] = make_double2(0.0, 0.0);
      g[u] = 0.0;
      if (s0 + u < ns) {
        w[u] = wt[ix];
        g[u] = gp[(int64_t)(s0 + u) * m2];
      }
      ix += j;
      if (ix >= D.L) ix -= D.L;
    }
#pragma unroll
    for (int u = 0; u < kGhBatch; ++u) {
      re += w[u].x * g[u];
      im += w[u].y * g[u];
    }
  }
  gh[D.gh_off + idx] = make_double2(re, im);
}

constexpr int kSepLds = 40960;   // LDS per workgroup: four of them per CU

// Bytes after the staged Grams for slot reads past the band: (nsp - 1) kFusedEC
// doubles at most, nsp = 256 / (J2C kFusedEC)
__host__ __device__ inline int sep_pad_bytes(int J2C) { return 256 / J2C * 8; }
constexpr int kSepQR = 4;   // staged products per thread and round (two rounds)
constexpr int kSepGR = 6;   // staged Gram entries per thread and round (two rounds)

// Gram terms per chunk of the separable kernel: each term stages G1_t[s1][ec]
// (B1 kFusedEC doubles) and Q_t[jj][ec] (J2C kFusedEC complex) in LDS; the
// chunk, its padding and the L1 twiddles fit kSepLds, and its entries fit the
// two staging rounds of 256 threads (at least one term: B1 <= 32, J2C <= 16)
__host__ __device__ inline int sep_term_chunk(int B1, int J2C, int L1, int nterm) {
  const int per = B1 * kFusedEC * 8 + J2C * kFusedEC * 16;
  int fit = (kSepLds - sep_pad_bytes(J2C) - L1 * 16) / per;
  const int fg = 2 * kSepGR * 256 / (B1 * kFusedEC), fq = 2 * kSepQR * 256 / (J2C * kFusedEC);
  fit = fit < fg ? fit : fg;
  fit = fit < fq ? fit : fq;
  return fit < 1 ? 1 : (fit < nterm ? fit : nterm);
}
// LDS of the separable kernel before its twiddles: the chunk's products,
// Grams and padding, or T2, whichever is larger
__host__ __device__ inline int sep_stage_bytes(int B1, int J2C, int L1, int nterm) {
  const int g = sep_term_chunk(B1, J2C, L1, nterm) * (B1 * kFusedEC * 8 + J2C * kFusedEC * 16) + sep_pad_bytes(J2C);
  const int t2 = B1 * J2C * kFusedEC * 16;
  return g > t2 ? g : t2;
}

// Asynchronous staging (lattices with m0^2 a multiple of 8: whole, 16-byte
// aligned entry chunks): kSepBufs chunk buffers, each holding per term the
// dimension-1 Grams G1_t[s1][ec] (B1 kFusedEC doubles) and the transformed
// factors F2_t[jj][ec] (J2C kFusedEC complex) and F3_t[ec] (kFusedEC complex),
// copied from global memory to LDS by the 16-byte global_load_lds, every copy
// of a chunk in flight at once.  With two buffers the next chunk is in flight
// while the current one is summed; summing a chunk takes far less than a copy
// round, so one buffer of twice the terms (half the rounds) is faster.
constexpr int kSepBufs = 1;
__host__ __device__ inline int sep_async_term_bytes(int B1, int J2C) {
  return B1 * kFusedEC * 8 + J2C * kFusedEC * 16 + kFusedEC * 16;
}
// terms per buffer, 0 when fewer than two fit (terms 0 and 1 must share a chunk)
__host__ __device__ inline int sep_async_chunk(int B1, int J2C, int L1, int nterm) {
  const int fit = (kSepLds - kSepBufs * sep_pad_bytes(J2C) - L1 * 16) / (kSepBufs * sep_async_term_bytes(B1, J2C));
  if (fit < 2) return 0;
  return fit < nterm ? fit : (nterm > 2 ? nterm : 2);
}
__host__ __device__ inline int sep_async_buf_bytes(int B1, int J2C, int L1, int nterm) {
  return sep_async_chunk(B1, J2C, L1, nterm) * sep_async_term_bytes(B1, J2C) + sep_pad_bytes(J2C);
}
__host__ __device__ inline bool sep_async_ok(int m2, int B1, int J2C, int L1, int nterm) {
  return m2 % kFusedEC == 0 && sep_async_chunk(B1, J2C, L1, nterm) >= 2;
}
// LDS of the separable kernel before its twiddles, for either staging
__host__ __device__ inline int sep_lds_stage(int m2, int B1, int J2C, int L1, int nterm) {
  if (!sep_async_ok(m2, B1, J2C, L1, nterm)) return sep_stage_bytes(B1, J2C, L1, nterm);
  const int g = kSepBufs * sep_async_buf_bytes(B1, J2C, L1, nterm), t2 = B1 * J2C * kFusedEC * 16;
  return g > t2 ? g : t2;
}

// Issue the copies of one chunk (terms t0 .. t0 + tc - 1) into an LDS buffer:
// 16-byte piece P of a region goes to region + 16 P, lane order within a wave
__device__ __forceinline__ void sep_async_issue(char* buf, int tc, int tcap, int B1, int J2C, int j2n,
                                                const double* g1, int64_t rowstep, const double2* f2,
                                                int64_t st2, int m2, const double2* f3, int64_t st3) {
  constexpr int EC = kFusedEC;
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const int tid = threadIdx.x, wb = tid & ~63;
  char* r1 = buf;                                              // G1 [tcap][B1][EC]
  char* r2 = r1 + tcap * B1 * EC * 8;                          // F2 [tcap][J2C][EC]
  char* r3 = r2 + tcap * J2C * EC * 16;                        // F3 [tcap][EC]
  const int n1 = tc * B1 * 4, n2 = tc * J2C * EC, n3 = tc * EC;
  for (int P = tid; P - (tid & 63) < n1; P += 256) {
    // row r = P / 4 of 8 doubles (term t0 + r / B1, slot r mod B1), quarter P mod 4
    if (P < n1)
      __builtin_amdgcn_global_load_lds((const void*)(g1 + (P >> 2) * rowstep + 2 * (P & 3)),
                                       (lds_ptr)(r1 + (P - tid + wb) * 16), 16, 0, 0);
  }
  for (int P = tid; P - (tid & 63) < n2; P += 256) {
    const int tt = P / (J2C * EC), jj = (P / EC) % J2C, ec = P % EC;
    if (P < n2 && jj < j2n)
      __builtin_amdgcn_global_load_lds((const void*)(f2 + tt * st2 + (int64_t)jj * m2 + ec),
                                       (lds_ptr)(r2 + (P - tid + wb) * 16), 16, 0, 0);
  }
  for (int P = tid; P - (tid & 63) < n3; P += 256) {
    if (P < n3)
      __builtin_amdgcn_global_load_lds((const void*)(f3 + (P / EC) * st3 + P % EC),
                                       (lds_ptr)(r3 + (P - tid + wb) * 16), 16, 0, 0);
  }
}

// Workgroup (lattice, entry chunk, j2 chunk, j3) as in dft_fused_kernel;
// grid y: H, S.  With Q_0 = P_ks / 2, Q_1 = P_ss / 2 and Q_t = -P_t (t >= 2)
// for H, and Q_0 = P_ss for S (one term), T2[s1] = sum_t G1_t[s1] Q_t.  The
// terms go in chunks staged in LDS, then thread (column (jj, ec), part sp)
// accumulates the slots s1 = sp, sp + nsp, ... of its column from LDS alone;
// T2 takes the stage's place once every term is in.  ASYNC (the plan's
// choice when every lattice allows it): the chunk's G1_t and the transformed
// factors of dimensions 2 and 3 arrive by global-to-LDS copies
// (sep_async_issue, sep_async_chunk) and the products are formed while
// summing; otherwise the workgroup loads G1_t and the factors in registers,
// forms Q_t, and stores both (sep_term_chunk), two rounds of loads per chunk.
template <int BM, bool ASYNC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BM <= 16 ? 4 : 1)))
sep_fused_kernel(const LatDev* __restrict__ lats,
                                                        const FusedTask* __restrict__ tasks, int ntasks,
                                                        const double2* __restrict__ tw,
                                                        const double* __restrict__ grams,
                                                        const double2* __restrict__ gh, double2* __restrict__ barH,
                                                        double2* __restrict__ barS, int half) {
  typedef double2 C;
  extern __shared__ char lds_raw[];
  const int64_t wg = blockIdx.x;
  const FusedTask T = tasks[find_fused(tasks, ntasks, wg)];
  const LatDev& L = lats[T.li];
  const DimDev& D0 = L.dim[0];
  const DimDev& D1 = L.dim[1];
  const DimDev& D2 = L.dim[2];
  const int L1 = L.L[0], L2 = L.L[1], L3 = L.L[2], B1 = nslot(D0);
  constexpr int EC = kFusedEC;
  const int m2 = L.m0 * L.m0, J2C = T.J2C;
  int64_t loc = wg - T.wg_base;
  const int eci = (int)(loc % T.nec);
  loc /= T.nec;
  const int j2c = (int)(loc % T.nj2c);
  const int j3 = (int)(loc / T.nj2c);
  if (half && j3 > L3 / 2) return;   // the conjugate half: the whole workgroup
  const int e0 = eci * EC, ecn = min(EC, m2 - e0);
  const int j2lo = j2c * J2C, j2n = min(J2C, L2 - j2lo);
  const int ncol = J2C * EC;
  const int tid = threadIdx.x;
  const bool isH = blockIdx.y == 0;
  const int nterm = isH ? L.T : 1;
  const int tch = sep_term_chunk(B1, J2C, L1, L.T);   // the S pass fits the H chunk
  // LDS: the stage (synchronous: [Qs | G1s | padding]; asynchronous, which the
  // plan chooses only when every lattice allows it: two chunk buffers) or T2,
  // then tw1
  const int stage_bytes = ASYNC ? sep_lds_stage(m2, B1, J2C, L1, L.T) : sep_stage_bytes(B1, J2C, L1, L.T);
  C* T2 = reinterpret_cast<C*>(lds_raw);
  C* Qs = reinterpret_cast<C*>(lds_raw);                       // [tch][ncol]
  double* G1s = reinterpret_cast<double*>(Qs + tch * ncol);    // [tch][B1][EC]
  C* tw1 = reinterpret_cast<C*>(lds_raw + stage_bytes);
  for (int q = tid; q < L1; q += 256) tw1[q] = tw[D0.tw_off + q];
  const int nsp = 256 / ncol;
  const int col = tid % ncol, sp = tid / ncol;
  const int jj = col / EC, ec = col % EC;
  const bool mine = sp < nsp && jj < j2n && ec < ecn;
  constexpr int NA = (BM + 1) / 2;   // slots per thread (nsp >= 2)
  // slots sp + nsp u, u < nu, of the column (the last may lie past the band:
  // it reads the next term's Grams or the padding into a sum that is never used)
  const int nu = __builtin_amdgcn_readfirstlane(min(NA, (B1 + nsp - 1) / nsp));
  const int ustride = nsp * EC;
  double ar[NA], ai[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) ar[u] = ai[u] = 0.0;
  const double2* g2 = gh + D1.gh_off;   // [t][L2][m2]
  const double2* g3 = gh + D2.gh_off;   // [t][L3][m2]
  const int64_t st2 = (int64_t)L2 * m2, st3 = (int64_t)L3 * m2;
  // T2 contributions of staged term tt with product qv (G1 rows from gp)
  auto accum = [&](const double* gp, int tt, C qv) {
    double g[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      g[u] = 0.0;
      if (u < nu) g[u] = gp[tt * B1 * EC + u * ustride];
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      ar[u] += g[u] * qv.x;
      ai[u] += g[u] * qv.y;
    }
  };
  if constexpr (ASYNC) {
    const int tcap = sep_async_chunk(B1, J2C, L1, L.T), bufb = sep_async_buf_bytes(B1, J2C, L1, L.T);
    const int64_t rowstep = (int64_t)(B1 == 1 ? D0.nshift : 1) * m2;   // staged row r: Gram block t0 nshift + r rs
    const double* g1b = grams + D0.gram_off + e0;
    const double2* f2b = g2 + (int64_t)j2lo * m2 + e0;
    const double2* f3b = g3 + (int64_t)j3 * m2 + e0;
    const int nch = (nterm + tcap - 1) / tcap;
    auto issue = [&](int k) {
      const int t0 = k * tcap, tc = min(tcap, nterm - t0);
      sep_async_issue(lds_raw + (k % kSepBufs) * bufb, tc, tcap, B1, J2C, j2n, g1b + (int64_t)t0 * D0.nshift * m2, rowstep,
                      f2b + t0 * st2, st2, m2, f3b + t0 * st3, st3);
    };
    issue(0);
    __builtin_amdgcn_s_waitcnt(0);   // this thread's copies have landed
    __syncthreads();                 // and everyone's
    for (int k = 0; k < nch; ++k) {
      // with two buffers the next chunk goes to the other one, whose last
      // reader passed the barrier below
      if (kSepBufs == 2 && k + 1 < nch) issue(k + 1);
      const int t0 = k * tcap, tc = min(tcap, nterm - t0);
      if (mine) {
        const char* buf = lds_raw + (k % kSepBufs) * bufb;
        const double* gp = reinterpret_cast<const double*>(buf) + sp * EC + ec;
        const C* F2 = reinterpret_cast<const C*>(buf + tcap * B1 * EC * 8) + jj * EC + ec;   // [tt][J2C][EC]
        const C* F3 = reinterpret_cast<const C*>(buf + tcap * B1 * EC * 8 + tcap * J2C * EC * 16) + ec;   // [tt][EC]
        int tt0 = 0;
        if (t0 == 0) {
          // terms 0 and 1 from S^2, S^3 (t = 0) and K^2, K^3 (t = 1)
          const C S2 = F2[0], S3 = F3[0];
          const C pss = make_double2(S2.x * S3.x - S2.y * S3.y, S2.x * S3.y + S2.y * S3.x);
          if (isH) {
            const C K2 = F2[J2C * EC], K3 = F3[EC];
            accum(gp, 0, make_double2(0.5 * ((K2.x * S3.x - K2.y * S3.y) + (S2.x * K3.x - S2.y * K3.y)),
                                      0.5 * ((K2.x * S3.y + K2.y * S3.x) + (S2.x * K3.y + S2.y * K3.x))));
            accum(gp, 1, make_double2(0.5 * pss.x, 0.5 * pss.y));
            tt0 = 2;
          } else {
            accum(gp, 0, pss);
            tt0 = 1;
          }
        }
#pragma unroll 1
        for (int tt = tt0; tt < tc; ++tt) {
          const C a = F2[tt * J2C * EC], b = F3[tt * EC];
          accum(gp, tt, make_double2(-(a.x * b.x - a.y * b.y), -(a.x * b.y + a.y * b.x)));
        }
      }
      if (kSepBufs == 1 && k + 1 < nch) {
        __syncthreads();   // this chunk is read
        issue(k + 1);
      }
      __builtin_amdgcn_s_waitcnt(0);   // the next chunk's copies have landed
      __syncthreads();                 // everyone's, and this chunk is read
    }
  }
  for (int t0 = 0; !ASYNC && t0 < nterm; t0 += tch) {
    const int tc = min(tch, nterm - t0);
    if (t0 > 0) __syncthreads();   // the previous chunk is consumed
    // the thread's first item, opaque so that no item's index is kept across chunks
    int qb = tid;
    asm volatile("" : "+v"(qb));
    // Q_t[col]: item q = qb + 256 u is (term t0 + q / ncol, column q mod ncol);
    // G1_t[s1][ec]: element q = qb + 256 u is (row r = q / EC, entry q mod EC),
    // row r = (term t0 + r / B1, slot r mod B1); B1 is nshift or 1, so the
    // row's Gram block is t0 nshift + r rs with rs = 1 or nshift.  Each round
    // has its Gram and product loads in flight together.
    const int nq = tc * ncol, ng = tc * B1 * EC, qe1 = qb % EC;
    const int rs = B1 == 1 ? D0.nshift : 1;
    const double* gb = grams + D0.gram_off + ((int64_t)t0 * D0.nshift + (qb / EC) * rs) * m2 + e0 + qe1;
    const int64_t ustep = (int64_t)(256 / EC) * rs * m2;   // 256 / EC rows further
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      if (qb + 256 * kSepQR * r >= nq && qb + 256 * kSepGR * r >= ng) break;
      double v[kSepGR];
#pragma unroll
      for (int u = 0; u < kSepGR; ++u) {
        const int q = qb + 256 * (kSepGR * r + u);
        v[u] = 0.0;
        if (q < ng && qe1 < ecn) v[u] = gb[(kSepGR * r + u) * ustep];
      }
      C a2[kSepQR], a3[kSepQR], k2 = make_double2(0.0, 0.0), k3 = k2;
      bool live[kSepQR];
      int tq[kSepQR];
#pragma unroll
      for (int u = 0; u < kSepQR; ++u) {
        const int q = qb + 256 * (kSepQR * r + u);
        const int tt = q / ncol, c2 = q - tt * ncol, qj = c2 / EC, qe = c2 % EC;
        const int t = t0 + tt;
        live[u] = q < nq && qj < j2n && qe < ecn;
        tq[u] = t;
        a2[u] = a3[u] = make_double2(0.0, 0.0);
        if (live[u]) {
          const int64_t o2 = (int64_t)(j2lo + qj) * m2 + e0 + qe, o3 = (int64_t)j3 * m2 + e0 + qe;
          const int tA = t < 2 ? 0 : t;   // terms 0 and 1 are formed from S^2 and S^3
          a2[u] = g2[tA * st2 + o2];
          a3[u] = g3[tA * st3 + o3];
          if (r == 0 && u == 0 && isH && t == 0) {   // only the first item can be term 0
            k2 = g2[st2 + o2];
            k3 = g3[st3 + o3];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kSepGR; ++u) {
        const int q = qb + 256 * (kSepGR * r + u);
        if (q < ng) G1s[q] = v[u];
      }
#pragma unroll
      for (int u = 0; u < kSepQR; ++u) {
        const int q = qb + 256 * (kSepQR * r + u);
        if (q < nq) {
          // branch-free: a divergent switch over t here was lowered with the
          // negation of the t >= 2 case missing
          const int t = tq[u];
          const C x = a2[u], y = a3[u];
          // P_t (t >= 2) or P_ss (t < 2) times 1 (S), 1/2 (H, t = 1) or -1 (H, t >= 2)
          const double h = !isH ? 1.0 : (t == 1 ? 0.5 : -1.0);
          double vx = h * (x.x * y.x - x.y * y.y), vy = h * (x.x * y.y + x.y * y.x);
          const bool ks = isH && t == 0;   // H, t = 0: P_ks / 2
          const double kx = 0.5 * ((k2.x * y.x - k2.y * y.y) + (x.x * k3.x - x.y * k3.y));
          const double ky = 0.5 * ((k2.x * y.y + k2.y * y.x) + (x.x * k3.y + x.y * k3.x));
          vx = ks ? kx : vx;
          vy = ks ? ky : vy;
          Qs[q] = make_double2(live[u] ? vx : 0.0, live[u] ? vy : 0.0);
        }
      }
    }
    __syncthreads();
    if (mine) {
      const C* qp = Qs + col;
      const double* gp = G1s + sp * EC + ec;
#pragma unroll 2
      for (int tt = 0; tt < tc; ++tt) {
        const C qv = qp[tt * ncol];
        double g[NA];
#pragma unroll
        for (int u = 0; u < NA; ++u) {
          g[u] = 0.0;
          if (u < nu) g[u] = gp[tt * B1 * EC + u * ustride];
        }
#pragma unroll
        for (int u = 0; u < NA; ++u) {
          ar[u] += g[u] * qv.x;
          ai[u] += g[u] * qv.y;
        }
      }
    }
  }
  __syncthreads();   // every stage read is done before T2 overwrites it
  if (mine) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int s1 = sp + nsp * u;
      if (s1 < B1) T2[(s1 * J2C + jj) * EC + ec] = make_double2(ar[u], ai[u]);
    }
  }
  __syncthreads();
  fused_last_stage<double, BM>(L, J2C, j2lo, j2n, j3, e0, ecn, T2, tw1, isH, barH, barS, nullptr, nullptr, half != 0);
}

constexpr int kChainEC = 8;    // block entries per chain workgroup
constexpr int kChainJC = 32;   // outputs j1 per chain workgroup
constexpr int kChainTC = 32;   // Gram terms per step
constexpr int kChainB = 32;    // widest band of a chain (as for the fused kernels)

// Separable formation of a chain (L2 = L3 = 1).  Dimensions 2 and 3 are one
// cell wide, their Grams single blocks, so per block entry e the products
//   Q_0 = (K2 S3 + S2 K3) / 2,  Q_1 = S2 S3 / 2,  Q_t = -M2_t M3_t (t >= 2),
// are plain numbers, the generator entries of slot s are
//   A^H_s = sum_t G1_t[s] Q_t  (G1_0 = S1, G1_1 = K1),   A^S_s = S1[s] S2 S3,
// and Hbar_j = sum_s w1^(j k_s) A_s.  Workgroup (lattice, kChainEC entries,
// kChainJC outputs j), thread (slot, entry) while forming A, then (j, entry):
// per step of kChainTC terms every thread issues its slot's Gram loads, the
// workgroup stages the step's Q_t in LDS meanwhile, and the thread
// accumulates; then the chunk's twiddles and one output of each operator per
// thread.  No generator stack is formed.
__global__ void __launch_bounds__(256) sep_chain_kernel(const LatDev* __restrict__ lats,
                                                        const FusedTask* __restrict__ tasks, int ntasks,
                                                        const double2* __restrict__ tw,
                                                        const double* __restrict__ grams,
                                                        double2* __restrict__ barH, double2* __restrict__ barS,
                                                        int half) {
  constexpr int EC = kChainEC, JC = kChainJC, TC = kChainTC, BC = kChainB;
  static_assert(BC * EC == 256 && JC * EC == 256, "one (slot, entry) and one (j, entry) pair per thread");
  __shared__ double Qs[TC][EC];
  __shared__ double As[2][BC][EC];
  __shared__ double2 Ws[JC][BC];
  const int64_t wg = blockIdx.x;
  const FusedTask T = tasks[find_fused(tasks, ntasks, wg)];
  const LatDev& L = lats[T.li];
  const DimDev& D0 = L.dim[0];
  const DimDev& D1 = L.dim[1];
  const DimDev& D2 = L.dim[2];
  const int L1 = L.L[0], B1 = nslot(D0), E = L.m0 * L.m0;
  const int64_t loc = wg - T.wg_base;
  const int eci = (int)(loc % T.nec), jci = (int)(loc / T.nec);
  const int e0 = eci * EC, ecn = min(EC, E - e0);
  const int j0 = jci * JC, jn = min(JC, L1 - j0);
  const int tid = threadIdx.x;
  const double* g0 = grams + D0.gram_off;   // [t][nshift][E]
  const double* g1 = grams + D1.gram_off;   // [t][E] (one slot)
  const double* g2 = grams + D2.gram_off;
  const int sl = tid / EC, ec = tid % EC;
  const bool mine = sl < B1 && ec < ecn;
  const int64_t tstride = (int64_t)D0.nshift * E;
  const double* src = g0 + (int64_t)sl * E + e0 + ec;
  double acc = 0.0, s1 = 0.0;
  for (int t0 = 0; t0 < L.T; t0 += TC) {
    const int tc = min(TC, L.T - t0);
    double x[TC];
#pragma unroll
    for (int v = 0; v < TC; ++v) x[v] = mine && v < tc ? src[(int64_t)(t0 + v) * tstride] : 0.0;
    // Q_t of the step, one (term, entry) pair per thread
    {
      const int tt = tid / EC, qe = tid % EC;
      const int t = t0 + tt;
      double q = 0.0;
      if (tt < tc && qe < ecn) {
        const int e = e0 + qe;
        if (t >= 2) q = -g1[(int64_t)t * E + e] * g2[(int64_t)t * E + e];
        else if (t == 1) q = 0.5 * g1[e] * g2[e];
        else q = 0.5 * (g1[E + e] * g2[e] + g1[e] * g2[E + e]);
      }
      Qs[tt][qe] = q;
    }
    __syncthreads();
    if (t0 == 0) s1 = x[0];
#pragma unroll
    for (int v = 0; v < TC; ++v) acc += x[v] * Qs[v][ec];
    __syncthreads();
  }
  // S2 S3 = 2 Q_1 (exact), and the twiddles w1^(j k_s) of the chunk
  const int e = e0 + ec;
  const double s23 = ec < ecn ? g1[e] * g2[e] : 0.0;
  As[0][sl][ec] = mine ? acc : 0.0;
  As[1][sl][ec] = mine ? s1 * s23 : 0.0;
  for (int q = tid; q < JC * B1; q += 256) {
    const int jj = q / B1, ss = q - jj * B1;
    const int64_t m = (int64_t)(j0 + jj) * slot_cell(D0, ss) % L1;
    Ws[jj][ss] = jj < jn ? tw[D0.tw_off + (int)m] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int jj = tid / EC;
  if (jj < jn && ec < ecn) {
    double hr = 0.0, hi = 0.0, sr = 0.0, si = 0.0;
#pragma unroll 4
    for (int ss = 0; ss < B1; ++ss) {
      const double2 w = Ws[jj][ss];
      const double ah = As[0][ss][ec], as = As[1][ss][ec];
      hr += w.x * ah;
      hi += w.y * ah;
      sr += w.x * as;
      si += w.y * as;
    }
    const int64_t o = (half ? L.half_off : L.gen_off) + (int64_t)(j0 + jj) * E + e;   // L3 = 1: both layouts agree
    barH[o] = make_double2(hr, hi);
    barS[o] = make_double2(sr, si);
  }
}

}  // namespace

// LDS bytes (complex128) of the fused kernel for a lattice, 0 when the
// lattice does not qualify (one transformed dimension, a band wider than 32
// slots, an axis longer than 4096, or more than 64 KiB).
// Workgroup ranges of a grouped Fourier launch, longest first (LPT): a
// workgroup of lattice L does about B1 (J + T) complex multiply-adds per
// column (J outputs along dimension 1, T Gram terms), and workgroups start in
// index order, so the costly lattices go first and the cheap ones fill the
// tail.  wg_base follows the new order; the kernels find their task by it.
static void order_fused_tasks(const std::vector<LatDev>& lats, std::vector<FusedTask>& tasks, bool chain) {
  auto cost = [&](const FusedTask& t) {
    const LatDev& L = lats[t.li];
    return (int64_t)nslot(L.dim[0]) * ((chain ? t.J2C : L.L[0]) + L.T);
  };
  auto nwg = [&](const FusedTask& t) {
    return chain ? (int64_t)t.nec * t.nj2c : (int64_t)lats[t.li].L[2] * t.nj2c * t.nec;
  };
  std::stable_sort(tasks.begin(), tasks.end(), [&](const FusedTask& a, const FusedTask& b) { return cost(a) > cost(b); });
  int64_t base = 0;
  for (FusedTask& t : tasks) {
    t.wg_base = base;
    base += nwg(t);
  }
}

static int64_t fused_lds_bytes(const LatDev& L) {
  int nd = 0;
  for (int d = 0; d < 3; ++d) nd += L.L[d] > 1;
  if (nd < 2 || L.L[0] > 4096) return 0;
  const int B1 = nslot(L.dim[0]), B2 = nslot(L.dim[1]), B3 = nslot(L.dim[2]);
  if (B1 > 32 || B2 > 32 || B3 > 32) return 0;
  const int J2C = std::min(L.L[1], kFusedJ2);
  const int64_t n = (int64_t)B1 * B2 * kFusedEC + (int64_t)B1 * J2C * kFusedEC + L.L[0] + (int64_t)J2C * B2 + B3;
  return n * 16 > 65536 ? 0 : n * 16;
}

void plan_block_dft(const std::vector<LatDev>& lats, int64_t target_threads, std::vector<DftTask>& tasks,
                    std::vector<DftLaunch>& launches, int64_t& tmp_elems, std::vector<FusedTask>& fused,
                    int64_t& fused_wgs, int32_t& fused_bmax, int32_t& fused_lds) {
  tasks.clear();
  launches.clear();
  fused.clear();
  fused_wgs = 0;
  fused_bmax = 0;
  fused_lds = 0;
  const int nlat = (int)lats.size();
  // lattices with two or three transformed dimensions take the fused kernel
  std::vector<bool> is_fused(nlat, false);
  for (int li = 0; li < nlat; ++li) {
    const LatDev& L = lats[li];
    const int64_t lb = fused_lds_bytes(L);
    if (lb == 0) continue;
    is_fused[li] = true;
    FusedTask t{};
    t.li = li;
    t.EC = kFusedEC;
    t.nec = (L.m0 * L.m0 + kFusedEC - 1) / kFusedEC;
    t.J2C = std::min(L.L[1], kFusedJ2);
    t.nj2c = (L.L[1] + t.J2C - 1) / t.J2C;
    t.wg_base = fused_wgs;
    fused_wgs += (int64_t)L.L[2] * t.nj2c * t.nec;
    fused.push_back(t);
    for (int d = 0; d < 3; ++d) fused_bmax = std::max(fused_bmax, nslot(L.dim[d]));
    fused_lds = std::max<int32_t>(fused_lds, (int32_t)lb);
  }
  order_fused_tasks(lats, fused, false);
  // per lattice: the transformed dimensions, last non-trivial first (a
  // one-cell lattice is a single pass over dimension 3 that copies)
  std::vector<std::vector<int>> dims(nlat);
  for (int li = 0; li < nlat; ++li) {
    if (is_fused[li]) continue;
    for (int d = 2; d >= 0; --d)
      if (lats[li].L[d] > 1) dims[li].push_back(d);
    if (dims[li].empty()) dims[li].push_back(2);
  }
  // intermediate regions: outputs of pass 0 (lattices with >= 2 passes), then
  // outputs of pass 1 (lattices with 3 passes); H then S in each
  std::vector<int64_t> out0(nlat, -1), out1(nlat, -1), sz0(nlat, 0), sz1(nlat, 0);
  int64_t off = 0;
  auto inter_size = [&](const LatDev& L, int d) {
    int64_t sz = (int64_t)L.m0 * L.m0;
    for (int q = 0; q < 3; ++q) sz *= (q < d) ? nslot(L.dim[q]) : L.L[q];
    return sz;
  };
  for (int li = 0; li < nlat; ++li)
    if (dims[li].size() >= 2) { sz0[li] = inter_size(lats[li], dims[li][0]); out0[li] = off; off += 2 * sz0[li]; }
  for (int li = 0; li < nlat; ++li)
    if (dims[li].size() >= 3) { sz1[li] = inter_size(lats[li], dims[li][1]); out1[li] = off; off += 2 * sz1[li]; }
  tmp_elems = off;
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<DftTask> cls_tasks[5];
    int64_t outputs[5] = {0, 0, 0, 0, 0};
    for (int li = 0; li < nlat; ++li) {
      const LatDev& L = lats[li];
      if ((int)dims[li].size() <= pass) continue;
      const int d = dims[li][pass];
      DftTask t{};
      t.li = li;
      t.d = d;
      int64_t O = 1;
      for (int q = 0; q < d; ++q) O *= nslot(L.dim[q]);
      int64_t I = (int64_t)L.m0 * L.m0;
      for (int q = d + 1; q < 3; ++q) I *= L.L[q];
      t.O = (int32_t)O;
      t.I = (int32_t)I;
      t.B = nslot(L.dim[d]);
      t.out_final = pass + 1 == (int)dims[li].size();
      if (pass == 1) { t.in_off = out0[li]; t.in_half = sz0[li]; }
      if (pass == 2) { t.in_off = out1[li]; t.in_half = sz1[li]; }
      if (!t.out_final) {
        t.out_off = pass == 0 ? out0[li] : out1[li];
        t.out_half = pass == 0 ? sz0[li] : sz1[li];
      }
      const int c = band_class(t.B);
      outputs[c] += O * L.L[d] * I;
      cls_tasks[c].push_back(t);
    }
    for (int c = 0; c < 5; ++c) {
      if (cls_tasks[c].empty()) continue;
      DftLaunch l{};
      l.pass = pass;
      l.cls = c;
      l.t0 = (int32_t)tasks.size();
      l.nt = (int32_t)cls_tasks[c].size();
      // outputs per thread chosen so that the launch runs ~target_threads
      const int64_t jc = std::max<int64_t>(1, outputs[c] / std::max<int64_t>(1, target_threads));
      int64_t tb = 0;
      for (DftTask& t : cls_tasks[c]) {
        const int Ld = lats[t.li].L[t.d];
        t.JC = c == 4 ? 1 : (int32_t)std::min<int64_t>(Ld, jc);
        t.njc = (Ld + t.JC - 1) / t.JC;
        t.tbase = tb;
        tb += ((int64_t)t.O * t.njc * t.I + 255) / 256 * 256;
        if (c < 4 && Ld <= kLdsTwiddles) l.lds_tw = std::max(l.lds_tw, Ld);
        tasks.push_back(t);
      }
      l.threads = tb;
      launches.push_back(l);
    }
  }
}

// Separable formation: one task per chain for sep_chain_kernel, and for every
// other lattice one task (workgroups as in the fused kernel) and the
// transforms of its Grams along dimensions 2 and 3.  ok = false when a
// lattice has a first-dimension band wider than 32 slots or needs more than
// 64 KiB of LDS.
void plan_separable(const std::vector<LatDev>& lats, std::vector<FusedTask>& tasks, std::vector<GhItem>& items,
                    int64_t& wgs, int32_t& bmax, int32_t& lds, int64_t& gh_threads, std::vector<FusedTask>& chain,
                    int64_t& chain_wgs, bool& ok, bool& async) {
  tasks.clear();
  items.clear();
  chain.clear();
  chain_wgs = 0;
  wgs = 0;
  bmax = 0;
  lds = 0;
  gh_threads = 0;
  ok = !lats.empty();
  async = true;
  int32_t lds_sync = 0, lds_async = 0;
  for (int li = 0; li < (int)lats.size(); ++li) {
    const LatDev& L = lats[li];
    const int B1 = nslot(L.dim[0]);
    if (L.L[1] == 1 && L.L[2] == 1) {
      // a chain: sep_chain_kernel, which needs no transformed Grams
      if (B1 > kChainB) ok = false;
      FusedTask c{};
      c.li = li;
      c.EC = kChainEC;
      c.nec = (L.m0 * L.m0 + kChainEC - 1) / kChainEC;
      c.J2C = kChainJC;
      c.nj2c = (L.L[0] + kChainJC - 1) / kChainJC;
      c.wg_base = chain_wgs;
      chain_wgs += (int64_t)c.nec * c.nj2c;
      chain.push_back(c);
      continue;
    }
    FusedTask t{};
    t.li = li;
    t.EC = kFusedEC;
    t.nec = (L.m0 * L.m0 + kFusedEC - 1) / kFusedEC;
    t.J2C = std::min(L.L[1], kFusedJ2);
    t.nj2c = (L.L[1] + t.J2C - 1) / t.J2C;
    // the stage of either staging or T2, whichever is larger, then the
    // dimension-1 twiddles; the asynchronous copies need every lattice to
    // allow them, with 16-byte aligned Gram rows
    const int m2 = L.m0 * L.m0;
    const int64_t bsync = (int64_t)sep_stage_bytes(B1, t.J2C, L.L[0], L.T) + (int64_t)L.L[0] * 16;
    const int64_t basync = (int64_t)sep_lds_stage(m2, B1, t.J2C, L.L[0], L.T) + (int64_t)L.L[0] * 16;
    if (B1 > 32 || bsync > 65536) ok = false;
    if (!sep_async_ok(m2, B1, t.J2C, L.L[0], L.T) || (L.dim[0].gram_off & 1) != 0 || basync > 65536) async = false;
    t.wg_base = wgs;
    wgs += (int64_t)L.L[2] * t.nj2c * t.nec;
    tasks.push_back(t);
    bmax = std::max(bmax, B1);
    lds_sync = std::max<int32_t>(lds_sync, (int32_t)bsync);
    lds_async = std::max<int32_t>(lds_async, (int32_t)basync);
    for (int d = 1; d < 3; ++d) {
      items.push_back(GhItem{li, d, gh_threads});
      gh_threads += ((int64_t)L.T * L.L[d] * L.m0 * L.m0 + 255) / 256 * 256;
    }
  }
  if (tasks.empty()) async = false;
  lds = async ? lds_async : lds_sync;
  order_fused_tasks(lats, tasks, false);
  order_fused_tasks(lats, chain, true);
}

hipError_t launch_fourier_sep(const lhf_plan_s* p, const double* g64, double2* gh, double2* bar_h, double2* bar_s,
                              hipStream_t s, bool half) {
  const int hf = half ? 1 : 0;
  if (!p->sep_ok || (p->n_sep > 0 && !gh)) return hipErrorInvalidValue;
  if (p->n_sep_chain > 0)
    hipLaunchKernelGGL(sep_chain_kernel, dim3((unsigned)p->sep_chain_wgs), dim3(256), 0, s, p->d_lat,
                       p->d_sep_chain, p->n_sep_chain, p->d_tw64, g64, bar_h, bar_s, hf);
  if (p->n_sep == 0) return hipGetLastError();
  hipLaunchKernelGGL(gram_dft_kernel, dim3((unsigned)(p->gh_threads / 256)), dim3(256), 0, s, p->d_lat,
                     p->d_gh_items, p->n_gh_items, g64, p->d_tw64, gh);
  const dim3 grid((unsigned)p->sep_wgs, 2);
  const size_t shb = (size_t)p->sep_lds;
#define LHF_SEP(BM)                                                                                          \
  if (p->sep_async)                                                                                          \
    hipLaunchKernelGGL((sep_fused_kernel<BM, true>), grid, dim3(256), shb, s, p->d_lat, p->d_sep, p->n_sep,  \
                       p->d_tw64, g64, gh, bar_h, bar_s, hf);                                                \
  else                                                                                                       \
    hipLaunchKernelGGL((sep_fused_kernel<BM, false>), grid, dim3(256), shb, s, p->d_lat, p->d_sep, p->n_sep, \
                       p->d_tw64, g64, gh, bar_h, bar_s, hf);
  if (p->sep_bmax <= 8) {
    LHF_SEP(8)
  } else if (p->sep_bmax <= 16) {
    LHF_SEP(16)
  } else {
    LHF_SEP(32)
  }
#undef LHF_SEP
  return hipGetLastError();
}

hipError_t launch_block_dft(const lhf_plan_s* p, int prec, const void* gen_h, const void* gen_s, void* bar_h,
                            void* bar_s, void* tmp, float2* b32_h, float2* b32_s, hipStream_t s, bool half) {
  if (half && b32_h) return hipErrorInvalidValue;   // no complex64 copy of the half layout
  if (prec == LHF_PREC_FP64)
    return dft_launch_all<double>(p, (const double*)gen_h, (const double*)gen_s, (double2*)bar_h, (double2*)bar_s,
                                  (double2*)tmp, p->d_tw64, b32_h, b32_s, half, s);
  return dft_launch_all<float>(p, (const float*)gen_h, (const float*)gen_s, (float2*)bar_h, (float2*)bar_s,
                               (float2*)tmp, p->d_tw32, nullptr, nullptr, half, s);
}

}  // namespace lhf
