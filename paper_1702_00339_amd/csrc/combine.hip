// Hadamard combination of the 1D Grams into the generator stacks (Lemma 3.4,
// eqs. BC-Core, BC-mass, BC-Laplace; Prop. 2.2 eqs. Mass_Gal_fact and
// Lapl_Gal_fact):
//   S_k = S1[k1] o S2[k2] o S3[k3]
//   H_k = 1/2 (K1 o S2 o S3 + S1 o K2 o S3 + S1 o S2 o K3) - sum_r M1_r o M2_r o M3_r
// for every cell k of the lattice, written as the dense first block column
// [k1][k2][k3][mu][nu]; cells whose offset lies outside the band in any
// dimension are written as zero.  One thread per (cell, mu, nu); the Grams
// are small and stay in L2.  Arithmetic in FP64 (FP64 Grams) or FP32 (the
// split-precision Grams of the mixed pipeline).
//
// Grouped launch: every lattice's thread range starts at a multiple of 256
// (table elem_start), so a workgroup serves one lattice, found by binary
// search over the table.
#include "plan.h"

namespace lhf {
namespace {

__device__ __forceinline__ int slot_of(const DimDev& D, int k) {
  if (D.full) return k;
  int s = k <= D.L / 2 ? k : k - D.L;   // signed offset
  if (s < -D.L0 || s > D.L0) return -1;
  return s + D.L0;
}

template <typename G, typename O>
__global__ void __launch_bounds__(256) combine_kernel(const LatDev* __restrict__ lats,
                                                      const int64_t* __restrict__ elem_start, int nlat,
                                                      const G* __restrict__ grams,
                                                      O* __restrict__ H, O* __restrict__ S) {
  const int64_t wg0 = (int64_t)blockIdx.x * 256;
  int lo = 0, hi = nlat - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (elem_start[mid] <= wg0) lo = mid; else hi = mid - 1;
  }
  const LatDev& L = lats[lo];
  const int m2 = L.m0 * L.m0;
  const int idx = (int)(wg0 - elem_start[lo]) + threadIdx.x;   // the planner keeps nblk m0^2 < 2^31
  if (idx >= L.nblk * m2) return;
  const int cell = idx / m2;
  const int e = idx - cell * m2;
  const int k3 = cell % L.L[2];
  const int k2 = (cell / L.L[2]) % L.L[1];
  const int k1 = cell / (L.L[2] * L.L[1]);
  const int s1 = slot_of(L.dim[0], k1), s2 = slot_of(L.dim[1], k2), s3 = slot_of(L.dim[2], k3);
  const int64_t out = L.gen_off + idx;
  if (s1 < 0 || s2 < 0 || s3 < 0) {
    H[out] = O(0);
    S[out] = O(0);
    return;
  }
  const DimDev& D1 = L.dim[0];
  const DimDev& D2 = L.dim[1];
  const DimDev& D3 = L.dim[2];
  // Gram[t][s][e] with e = mu m0 + nu
  auto at = [&](const DimDev& D, int t, int s) -> G {
    return grams[D.gram_off + ((int64_t)t * D.nshift + s) * m2 + e];
  };
  G a1 = at(D1, 0, s1), a2 = at(D2, 0, s2), a3 = at(D3, 0, s3);
  G b1 = at(D1, 1, s1), b2 = at(D2, 1, s2), b3 = at(D3, 1, s3);
  G sv = a1 * a2 * a3;
  G tv = G(0.5) * (b1 * a2 * a3 + a1 * b2 * a3 + a1 * a2 * b3);
  // potential terms eight at a time: 24 independent loads in flight, four
  // partial sums (a fixed order, so the result is deterministic)
  G vv[4] = {G(0), G(0), G(0), G(0)};
  int t = 2;
  for (; t + 8 <= L.T; t += 8) {
    G x1[8], x2[8], x3[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x1[u] = at(D1, t + u, s1);
      x2[u] = at(D2, t + u, s2);
      x3[u] = at(D3, t + u, s3);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the 24 loads ahead of their uses
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u & 3] += x1[u] * x2[u] * x3[u];
  }
  for (; t < L.T; ++t) vv[0] += at(D1, t, s1) * at(D2, t, s2) * at(D3, t, s3);
  H[out] = O(tv - ((vv[0] + vv[1]) + (vv[2] + vv[3])));
  S[out] = O(sv);
}

}  // namespace

hipError_t launch_combine(const lhf_plan_s* p, const double* g64, const float* g32, double* H64,
                          double* S64, float* H32, float* S32, hipStream_t s) {
  const dim3 grid((unsigned)(p->combine_threads / 256));
  const int64_t* es = p->d_elem_start;
  if (H64) hipLaunchKernelGGL((combine_kernel<double, double>), grid, dim3(256), 0, s, p->d_lat, es, p->nlat, g64, H64, S64);
  if (H32) {
    if (g32)
      hipLaunchKernelGGL((combine_kernel<float, float>), grid, dim3(256), 0, s, p->d_lat, es, p->nlat, g32, H32, S32);
    else
      hipLaunchKernelGGL((combine_kernel<double, float>), grid, dim3(256), 0, s, p->d_lat, es, p->nlat, g64, H32, S32);
  }
  return hipGetLastError();
}

}  // namespace lhf
