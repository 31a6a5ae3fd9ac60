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

__device__ __forceinline__ int slot_cell(const DimDev& D, int s) {
  if (D.full) return s;
  int k = s - D.L0;
  return k < 0 ? k + D.L : k;
}

__device__ __forceinline__ int nslot(const DimDev& D) { return D.L == 1 ? 1 : D.nshift; }

// First pass: real generator stack -> complex, transforming dimension df.
template <typename R>
__global__ void __launch_bounds__(256) dft_first_kernel(const LatDev* __restrict__ lats, int li, int df,
                                                        const typename Cx<R>::T* __restrict__ tw,
                                                        const R* __restrict__ genH, const R* __restrict__ genS,
                                                        typename Cx<R>::T* __restrict__ outH,
                                                        typename Cx<R>::T* __restrict__ outS) {
  typedef typename Cx<R>::T C;
  const LatDev& L = lats[li];
  const int E = L.m0 * L.m0;
  const DimDev& D = L.dim[df];
  int O = 1;
  for (int d = 0; d < df; ++d) O *= nslot(L.dim[d]);
  const int64_t tot = (int64_t)O * D.L * E;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= tot) return;
  const R* X = (blockIdx.y == 0 ? genH : genS) + L.gen_off;
  C* Y = blockIdx.y == 0 ? outH : outS;
  const int e = (int)(idx % E);
  const int j = (int)((idx / E) % D.L);
  int o = (int)(idx / ((int64_t)E * D.L));
  // cells of the outer (not yet transformed) dimensions from their band slots
  int kk[3] = {0, 0, 0};
  for (int d = df - 1; d >= 0; --d) {
    const int ns = nslot(L.dim[d]);
    kk[d] = slot_cell(L.dim[d], o % ns);
    o /= ns;
  }
  const C* T = tw + D.tw_off;
  R re = 0, im = 0;
  const int B = nslot(D);
  for (int b = 0; b < B; ++b) {
    kk[df] = slot_cell(D, b);
    const int64_t cell = ((int64_t)kk[0] * L.L[1] + kk[1]) * L.L[2] + kk[2];
    const R x = X[cell * E + e];
    const C w = T[(int)(((int64_t)j * kk[df]) % D.L)];
    re += w.x * x;
    im += w.y * x;
  }
  C r;
  r.x = re;
  r.y = im;
  Y[idx] = r;
}

// Later passes: [O][B][I] (slots of dimension d) -> [O][L_d][I].
template <typename R>
__global__ void __launch_bounds__(256) dft_next_kernel(const LatDev* __restrict__ lats, int li, int d, int O,
                                                       int64_t I, const typename Cx<R>::T* __restrict__ tw,
                                                       const typename Cx<R>::T* __restrict__ inH,
                                                       const typename Cx<R>::T* __restrict__ inS,
                                                       typename Cx<R>::T* __restrict__ outH,
                                                       typename Cx<R>::T* __restrict__ outS) {
  typedef typename Cx<R>::T C;
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int B = nslot(D);
  const int64_t tot = (int64_t)O * D.L * I;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= tot) return;
  const C* X = blockIdx.y == 0 ? inH : inS;
  C* Y = blockIdx.y == 0 ? outH : outS;
  const int64_t i = idx % I;
  const int j = (int)((idx / I) % D.L);
  const int64_t o = idx / (I * D.L);
  const C* T = tw + D.tw_off;
  const C* src = X + o * B * I + i;
  R re = 0, im = 0;
  for (int b = 0; b < B; ++b) {
    const int k = slot_cell(D, b);
    const C w = T[(int)(((int64_t)j * k) % D.L)];
    const C x = src[(int64_t)b * I];
    re += w.x * x.x - w.y * x.y;
    im += w.x * x.y + w.y * x.x;
  }
  C r;
  r.x = re;
  r.y = im;
  Y[idx] = r;
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
  C* cur_h = nullptr;
  C* cur_s = nullptr;
  for (int pi = 0; pi < nd; ++pi) {
    const int d = dims[pi];
    const bool last = pi + 1 == nd;
    const int64_t sz = inter_size(d);
    C* dst = (pi % 2 == 0) ? ta : tb;
    C* oh = last ? outH : dst;
    C* os = last ? outS : dst + sz;
    int64_t O = 1;
    for (int q = 0; q < d; ++q) O *= nsl(q);
    const int64_t tot = O * L.L[d] * (pi == 0 ? E : sz / (O * L.L[d]));
    const dim3 grid((unsigned)((tot + 255) / 256), ny);
    if (pi == 0) {
      hipLaunchKernelGGL(dft_first_kernel<R>, grid, dim3(256), 0, s, p->d_lat, li, d, tw, gH, gS,
                         oh ? oh : dst, os ? os : dst + sz);
    } else {
      const int64_t I = sz / (O * L.L[d]);
      hipLaunchKernelGGL(dft_next_kernel<R>, grid, dim3(256), 0, s, p->d_lat, li, d, (int)O, I, tw,
                         cur_h, cur_s, oh ? oh : dst, os ? os : dst + sz);
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
