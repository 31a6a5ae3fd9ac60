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
#include <algorithm>

#include "plan.h"

namespace lhf {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { typedef double2 T; };
template <> struct Cx<float> { typedef float2 T; };

constexpr int kLdsTwiddles = 2048;   // longest axis whose twiddles are staged in LDS

__device__ __forceinline__ int slot_cell(const DimDev& D, int s) {
  if (D.full) return s;
  int k = s - D.L0;
  return k < 0 ? k + D.L : k;
}

__device__ __forceinline__ int nslot(const DimDev& D) { return D.L == 1 ? 1 : D.nshift; }

// One pass of the pruned DFT along dimension d.  Thread t owns one input
// column (o, i) and a chunk of JC outputs j along the transformed axis: it
// loads the column's B band inputs once into registers and writes
//   Y[o][j][i] = sum_b w^(j k_b) X[o][b][i],  k_b the lattice offset of slot b
// for its JC values of j (twiddle indices advance by k_b per j, 32-bit).
// FIRST: X is the real generator stack, band-gathered over the outer dims
// (o enumerates their slots) with inner index i = block entry.
template <typename R, int BMAX, bool FIRST>
__global__ void __launch_bounds__(256) dft_pass_kernel(const LatDev* __restrict__ lats, int li, int d, int O,
                                                       int I, int JC, const typename Cx<R>::T* __restrict__ tw,
                                                       const void* __restrict__ inH, const void* __restrict__ inS,
                                                       typename Cx<R>::T* __restrict__ outH,
                                                       typename Cx<R>::T* __restrict__ outS) {
  typedef typename Cx<R>::T C;
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int Ld = D.L;
  const int B = nslot(D);
  const int njc = (Ld + JC - 1) / JC;
  const int tid = blockIdx.x * 256 + threadIdx.x;
  // twiddle table staged in LDS when the launch gives room for it
  extern __shared__ char lds_raw[];
  C* sT = reinterpret_cast<C*>(lds_raw);
  const bool lds_tw = Ld <= kLdsTwiddles;
  if (lds_tw) {
    for (int q = threadIdx.x; q < Ld; q += 256) sT[q] = tw[D.tw_off + q];
    __syncthreads();
  }
  if (tid >= O * njc * I) return;
  const int i = tid % I;
  const int jc = (tid / I) % njc;
  const int o = tid / (I * njc);
  const bool isH = blockIdx.y == 0;
  C* Y = isH ? outH : outS;
  R xr[BMAX], xi[BMAX];
  int kb[BMAX];
  if constexpr (FIRST) {
    const R* X = (const R*)(isH ? inH : inS) + L.gen_off;
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
    const C* X = (const C*)(isH ? inH : inS) + (int64_t)o * B * I + i;
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
  const C* T = lds_tw ? sT : tw + D.tw_off;
  C* dst = Y + (int64_t)o * Ld * I + i;
  for (int j = j0; j < j1; ++j) {
    R re = 0, im = 0;
#pragma unroll
    for (int b = 0; b < BMAX; ++b) {
      if (b < B) {
        const C w = T[idx[b]];
        re += w.x * xr[b] - w.y * xi[b];
        im += w.x * xi[b] + w.y * xr[b];
        idx[b] += kb[b];
        if (idx[b] >= Ld) idx[b] -= Ld;
      }
    }
    C r;
    r.x = re;
    r.y = im;
    dst[(int64_t)j * I] = r;
  }
}

// Fallback for bands wider than 32 slots: one thread per output.
template <typename R, bool FIRST>
__global__ void __launch_bounds__(256) dft_wide_kernel(const LatDev* __restrict__ lats, int li, int d, int O,
                                                       int I, const typename Cx<R>::T* __restrict__ tw,
                                                       const void* __restrict__ inH, const void* __restrict__ inS,
                                                       typename Cx<R>::T* __restrict__ outH,
                                                       typename Cx<R>::T* __restrict__ outS) {
  typedef typename Cx<R>::T C;
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int Ld = D.L;
  const int B = nslot(D);
  const int64_t tot = (int64_t)O * Ld * I;
  const int64_t tid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (tid >= tot) return;
  const int i = (int)(tid % I);
  const int j = (int)((tid / I) % Ld);
  const int o = (int)(tid / ((int64_t)I * Ld));
  const bool isH = blockIdx.y == 0;
  C* Y = isH ? outH : outS;
  const C* T = tw + D.tw_off;
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
  for (int b = 0; b < B; ++b) {
    const int k = slot_cell(D, b);
    const C w = T[(int)(((int64_t)j * k) % Ld)];
    R xr, xi;
    if (FIRST) {
      kk[d] = k;
      const int cell = (kk[0] * L.L[1] + kk[1]) * L.L[2] + kk[2];
      xr = ((const R*)(isH ? inH : inS))[L.gen_off + (int64_t)cell * L.m0 * L.m0 + i];
      xi = R(0);
    } else {
      const C x = ((const C*)(isH ? inH : inS))[((int64_t)o * B + b) * I + i];
      xr = x.x;
      xi = x.y;
    }
    re += w.x * xr - w.y * xi;
    im += w.x * xi + w.y * xr;
  }
  C r;
  r.x = re;
  r.y = im;
  Y[tid] = r;
}

// A one-cell lattice: the single block is its own transform.
template <typename R>
__global__ void __launch_bounds__(256) dft_copy_kernel(const LatDev* __restrict__ lats, int li,
                                                       const R* __restrict__ genH, const R* __restrict__ genS,
                                                       typename Cx<R>::T* __restrict__ outH,
                                                       typename Cx<R>::T* __restrict__ outS) {
  const LatDev& L = lats[li];
  const int E = L.m0 * L.m0;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= E) return;
  const R* X = (blockIdx.y == 0 ? genH : genS) + L.gen_off;
  typename Cx<R>::T* Y = blockIdx.y == 0 ? outH : outS;
  Y[e].x = X[e];
  Y[e].y = 0;
}

}  // namespace

int64_t block_dft_tmp_elems(const LatDev& L) {
  // largest intermediate (non-final) pass output, for H and S together
  int dims[3], nd = 0;
  for (int d = 2; d >= 0; --d)
    if (L.L[d] > 1) dims[nd++] = d;
  int64_t best = 0;
  const int64_t E = (int64_t)L.m0 * L.m0;
  for (int pi = 0; pi + 1 < nd; ++pi) {
    const int d = dims[pi];
    int64_t sz = E;
    for (int q = 0; q < 3; ++q) {
      const DimDev& D = L.dim[q];
      const int64_t ns = D.L == 1 ? 1 : D.nshift;
      sz *= (q < d) ? ns : D.L;
    }
    best = std::max(best, sz);
  }
  return 2 * best;
}

template <typename R>
static hipError_t dft_lattice(const lhf_plan_s* p, int li, const R* gH, const R* gS,
                              typename Cx<R>::T* bH, typename Cx<R>::T* bS, typename Cx<R>::T* ta,
                              typename Cx<R>::T* tb, const typename Cx<R>::T* tw, hipStream_t s) {
  typedef typename Cx<R>::T C;
  const LatDev& L = p->lat[li];
  const int64_t E = (int64_t)L.m0 * L.m0;
  int dims[3], nd = 0;
  for (int d = 2; d >= 0; --d)
    if (L.L[d] > 1) dims[nd++] = d;
  C* outH = bH ? bH + L.gen_off : nullptr;
  C* outS = bS ? bS + L.gen_off : nullptr;
  const unsigned ny = 2;
  if (nd == 0) {
    hipLaunchKernelGGL(dft_copy_kernel<R>, dim3((unsigned)((E + 255) / 256), ny), dim3(256), 0, s,
                       p->d_lat, li, gH, gS, outH, outS);
    return hipGetLastError();
  }
  auto nsl = [&](int d) -> int64_t { return L.L[d] == 1 ? 1 : L.dim[d].nshift; };
  // sizes of intermediates
  auto inter_size = [&](int d) -> int64_t {
    int64_t sz = E;
    for (int q = 0; q < 3; ++q) sz *= (q < d) ? nsl(q) : L.L[q];
    return sz;
  };
  const void* cur_h = gH;
  const void* cur_s = gS;
  for (int pi = 0; pi < nd; ++pi) {
    const int d = dims[pi];
    const bool last = pi + 1 == nd;
    const int64_t sz = inter_size(d);
    C* dst = (pi % 2 == 0) ? ta : tb;
    C* oh = last ? outH : dst;
    C* os = last ? outS : dst + sz;
    int64_t O = 1;
    for (int q = 0; q < d; ++q) O *= nsl(q);
    const int Ld = L.L[d];
    const int64_t I = pi == 0 ? E : sz / (O * Ld);
    const int B = (int)nsl(d);
    if (B <= 32) {
      // chunk the transformed axis so that at least ~128k threads run
      int64_t cols = O * I;
      int JC = (int)std::max<int64_t>(1, std::min<int64_t>(Ld, cols * Ld / 131072));
      const int njc = (Ld + JC - 1) / JC;
      const dim3 grid((unsigned)((cols * njc + 255) / 256), ny);
      const size_t shb = Ld <= kLdsTwiddles ? sizeof(C) * Ld : 0;
#define LHF_PASS(BM)                                                                                     \
  if (pi == 0)                                                                                           \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, true>), grid, dim3(256), shb, s, p->d_lat, li, d, (int)O, \
                       (int)I, JC, tw, cur_h, cur_s, oh, os);                                            \
  else                                                                                                   \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, false>), grid, dim3(256), shb, s, p->d_lat, li, d, (int)O,\
                       (int)I, JC, tw, cur_h, cur_s, oh, os);
      if (B <= 4) { LHF_PASS(4) }
      else if (B <= 8) { LHF_PASS(8) }
      else if (B <= 16) { LHF_PASS(16) }
      else { LHF_PASS(32) }
#undef LHF_PASS
    } else {
      const dim3 grid((unsigned)((O * Ld * I + 255) / 256), ny);
      if (pi == 0)
        hipLaunchKernelGGL((dft_wide_kernel<R, true>), grid, dim3(256), 0, s, p->d_lat, li, d, (int)O, (int)I, tw,
                           cur_h, cur_s, oh, os);
      else
        hipLaunchKernelGGL((dft_wide_kernel<R, false>), grid, dim3(256), 0, s, p->d_lat, li, d, (int)O, (int)I, tw,
                           cur_h, cur_s, oh, os);
    }
    cur_h = dst;
    cur_s = dst + sz;
  }
  return hipGetLastError();
}

hipError_t launch_block_dft(const lhf_plan_s* p, int li, int prec, const void* gen_h, const void* gen_s,
                            void* bar_h, void* bar_s, void* tmp_a, void* tmp_b, hipStream_t s) {
  if (prec == LHF_PREC_FP64)
    return dft_lattice<double>(p, li, (const double*)gen_h, (const double*)gen_s, (double2*)bar_h,
                               (double2*)bar_s, (double2*)tmp_a, (double2*)tmp_b, p->d_tw64, s);
  return dft_lattice<float>(p, li, (const float*)gen_h, (const float*)gen_s, (float2*)bar_h,
                            (float2*)bar_s, (float2*)tmp_a, (float2*)tmp_b, p->d_tw32, s);
}

}  // namespace lhf
