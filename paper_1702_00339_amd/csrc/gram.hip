// 1D Gram contractions on MFMA (Prop. 2.2; proof of Lemma 2.1; Lemma 3.4).
//
// For one lattice and one dimension, with G the node-major nodal factors of
// cell 0 ([n][m0]), every generator slot s (lattice offset k_s) and term t:
//   Gram_t[s](mu, nu) = sum_i G[(i - k_s nc) mod n][mu] * (Op_t G)[i][nu]
// Op_0 = S = (h/6) tridiag(1, 4, 1), Op_1 = A = (1/h) tridiag(-1, 2, -1)
// (cyclic on periodic dims, truncated on box dims), Op_(2+r) = diag(P_r).
// This is one GEMM C = A B with rows (t, nu), columns (s, mu) and the grid as
// the contraction index; the operands are formed in registers from the
// L2-resident factors (the shifted right operand is a cyclic window of G, so
// it is never materialised).  Each wave owns a 32 x 32 output tile (2 x 2
// MFMA tiles); the contraction is split over waves and the partial tiles are
// summed by a second kernel that also scatters to the Gram layout
// [t][s][mu][nu].
//
// Variants: FP64 (v_mfma_f64_16x16x4f64), FP32 operands
// (v_mfma_f32_16x16x4f32), and bf16 hi+lo split products
// hi*hi + hi*lo + lo*hi (v_mfma_f32_16x16x32_bf16), both with FP32 accumulation.
#include "plan.h"

namespace lhf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 2, TN = 2;   // 16 x 16 MFMA tiles per wave along rows / columns

struct RowInfo { int t, nu; bool ok; };
struct ColInfo { int mu, sn; bool ok; };

__device__ __forceinline__ double gval(const double* G, const DimDev& D, int m0, int j, int f) {
  if (D.periodic) {
    if (j < 0) j += D.n; else if (j >= D.n) j -= D.n;
  } else if (j < 0 || j >= D.n) {
    return 0.0;
  }
  return G[(int64_t)j * m0 + f];
}

// Left operand (Op_t G)[i][nu].
__device__ __forceinline__ double aval(const double* G, const double* P, const DimDev& D, int m0,
                                       const RowInfo& r, int i) {
  if (!r.ok || i >= D.n) return 0.0;
  double g0 = gval(G, D, m0, i, r.nu);
  if (r.t >= 2) {
    int pi = D.replicate ? i % D.nc : i;
    return P[(int64_t)(r.t - 2) * D.npot + pi] * g0;
  }
  double gm = gval(G, D, m0, i - 1, r.nu), gp = gval(G, D, m0, i + 1, r.nu);
  if (r.t == 0) return (D.h / 6.0) * (gm + 4.0 * g0 + gp);
  return (2.0 * g0 - gm - gp) / D.h;
}

// Right operand G[(i - k_s nc) mod n][mu].
__device__ __forceinline__ double bval(const double* G, const DimDev& D, int m0, const ColInfo& c,
                                       int i) {
  if (!c.ok || i >= D.n) return 0.0;
  int j = i - c.sn;
  if (j < 0) j += D.n;
  return G[(int64_t)j * m0 + c.mu];
}

__device__ __forceinline__ void lane_info(const LatDev& L, const DimDev& D, int tm, int tn, int lr,
                                          RowInfo* ri, ColInfo* ci) {
  const int M = L.T * L.m0, N = D.nshift * L.m0;
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    int r = (tm * TM + a) * 16 + lr;
    ri[a].ok = r < M;
    ri[a].t = r / L.m0;
    ri[a].nu = r % L.m0;
  }
#pragma unroll
  for (int b = 0; b < TN; ++b) {
    int c = (tn * TN + b) * 16 + lr;
    ci[b].ok = c < N;
    int slot = c / L.m0;
    ci[b].mu = c % L.m0;
    int k = D.full ? slot : slot - D.L0;
    int sn = 0;
    if (D.periodic) {
      sn = (int)(((int64_t)k * D.nc) % D.n);
      if (sn < 0) sn += D.n;
    }
    ci[b].sn = sn;
  }
}

__global__ void __launch_bounds__(64) gram_f64_kernel(const LatDev* __restrict__ lats, int li, int d,
                                                      const double* __restrict__ fac,
                                                      double* __restrict__ part) {
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int tiles_n = (N + 16 * TN - 1) / (16 * TN);
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int ks = blockIdx.y;
  const int lane = threadIdx.x, lr = lane & 15, lk = lane >> 4;
  const double* G = fac + D.g_off;
  const double* P = fac + D.p_off;
  RowInfo ri[TM];
  ColInfo ci[TN];
  lane_info(L, D, tm, tn, lr, ri, ci);
  d4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int k_beg = ks * D.kchunk;
  const int k_end = min(D.n, k_beg + D.kchunk);
  for (int k0 = k_beg; k0 < k_end; k0 += 4) {
    const int i = k0 + lk;
    double av[TM], bv[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) av[a] = aval(G, P, D, L.m0, ri[a], i);
#pragma unroll
    for (int b = 0; b < TN; ++b) bv[b] = bval(G, D, L.m0, ci[b], i);
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
  // v_mfma_f64_16x16x4f64 result layout: row lk + 4 v, column lr
  double* out = part + D.part_off + (int64_t)ks * M * N;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int c = (tn * TN + b) * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (tm * TM + a) * 16 + lk + 4 * v;
        if (r < M && c < N) out[(int64_t)r * N + c] = acc[a][b][v];
      }
    }
}

// Split-precision variants; MODE 1 = FP32 operands, MODE 2 = bf16 hi + lo.
template <int MODE>
__global__ void __launch_bounds__(64) gram_split_kernel(const LatDev* __restrict__ lats, int li,
                                                        int d, const double* __restrict__ fac,
                                                        float* __restrict__ part) {
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int tiles_n = (N + 16 * TN - 1) / (16 * TN);
  const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int ks = blockIdx.y;
  const int lane = threadIdx.x, lr = lane & 15, lk = lane >> 4;
  const double* G = fac + D.g_off;
  const double* P = fac + D.p_off;
  RowInfo ri[TM];
  ColInfo ci[TN];
  lane_info(L, D, tm, tn, lr, ri, ci);
  f4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const int k_beg = ks * D.kchunk;
  const int k_end = min(D.n, k_beg + D.kchunk);
  if constexpr (MODE == 1) {
    for (int k0 = k_beg; k0 < k_end; k0 += 4) {
      const int i = k0 + lk;
      float av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = (float)aval(G, P, D, L.m0, ri[a], i);
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = (float)bval(G, D, L.m0, ci[b], i);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  } else {
    for (int k0 = k_beg; k0 < k_end; k0 += 32) {
      bf8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = k0 + 8 * lk + e;
#pragma unroll
        for (int a = 0; a < TM; ++a) {
          float x = (float)aval(G, P, D, L.m0, ri[a], i);
          __bf16 hi = (__bf16)x;
          ah[a][e] = hi;
          al[a][e] = (__bf16)(x - (float)hi);
        }
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          float x = (float)bval(G, D, L.m0, ci[b], i);
          __bf16 hi = (__bf16)x;
          bh[b][e] = hi;
          bl[b][e] = (__bf16)(x - (float)hi);
        }
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
  }
  // f32 / bf16 MFMA result layout: row 4 lk + v, column lr
  float* out = part + D.part_off + (int64_t)ks * M * N;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int c = (tn * TN + b) * 16 + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (tm * TM + a) * 16 + 4 * lk + v;
        if (r < M && c < N) out[(int64_t)r * N + c] = acc[a][b][v];
      }
    }
}

// Sum the split-K partials and scatter C[(t, nu)][(s, mu)] to Gram[t][s][mu][nu].
template <typename T>
__global__ void __launch_bounds__(256) gram_reduce_kernel(const LatDev* __restrict__ lats, int li, int d,
                                                          const T* __restrict__ part,
                                                          T* __restrict__ grams) {
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  const int r = (int)(idx / N), c = (int)(idx % N);
  const T* src = part + D.part_off + idx;
  T acc = 0;
  for (int ks = 0; ks < D.ksplit; ++ks) acc += src[(int64_t)ks * M * N];
  const int t = r / L.m0, nu = r % L.m0, slot = c / L.m0, mu = c % L.m0;
  grams[D.gram_off + (((int64_t)t * D.nshift + slot) * L.m0 + mu) * L.m0 + nu] = acc;
}

}  // namespace

hipError_t launch_gram_f64(const lhf_plan_s* p, int li, int d, const double* fac, double* part,
                           double* grams, hipStream_t s) {
  const LatDev& L = p->lat[li];
  const DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int tiles = ((M + 16 * TM - 1) / (16 * TM)) * ((N + 16 * TN - 1) / (16 * TN));
  hipLaunchKernelGGL(gram_f64_kernel, dim3(tiles, D.ksplit), dim3(64), 0, s, p->d_lat, li, d, fac, part);
  const int64_t tot = (int64_t)M * N;
  hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     p->d_lat, li, d, part, grams);
  return hipGetLastError();
}

hipError_t launch_gram_split(const lhf_plan_s* p, int li, int d, int mode, const double* fac,
                             float* part, float* grams, hipStream_t s) {
  const LatDev& L = p->lat[li];
  const DimDev& D = L.dim[d];
  const int M = L.T * L.m0, N = D.nshift * L.m0;
  const int tiles = ((M + 16 * TM - 1) / (16 * TM)) * ((N + 16 * TN - 1) / (16 * TN));
  if (mode == LHF_GRAM_FP32)
    hipLaunchKernelGGL(gram_split_kernel<1>, dim3(tiles, D.ksplit), dim3(64), 0, s, p->d_lat, li, d, fac, part);
  else
    hipLaunchKernelGGL(gram_split_kernel<2>, dim3(tiles, D.ksplit), dim3(64), 0, s, p->d_lat, li, d, fac, part);
  const int64_t tot = (int64_t)M * N;
  hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     p->d_lat, li, d, part, grams);
  return hipGetLastError();
}

}  // namespace lhf
