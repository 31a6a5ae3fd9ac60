// 1D Gram contractions on MFMA (Prop. 2.2; proof of Lemma 2.1; Lemma 3.4).
//
// For one lattice and one dimension, with G the node-major nodal factors of
// cell 0 ([n][m0]), every generator slot s (lattice offset k_s) and term t:
//   Gram_t[s](mu, nu) = sum_i G[(i - k_s nc) mod n][mu] * (Op_t G)[i][nu]
// Op_0 = S = (h/6) tridiag(1, 4, 1), Op_1 = A = (1/h) tridiag(-1, 2, -1)
// (cyclic on periodic dims, truncated on box dims), Op_(2+r) = diag(P_r).
// This is one GEMM C = A B with rows (t, nu), columns (s, mu) and the grid as
// the contraction index, restricted to the window of nodes where the cell-0
// factor in every summand is not negligible (all nodes on one-cell dims).
//
// Grouped launch: one work list covers every lattice, dimension, 64 x 64
// output tile and split of the window.  A workgroup (4 waves) stages 32-node
// chunks of both operands in LDS (the next chunk's global loads, held in
// registers, overlap the current chunk's MFMAs) -- the left operand formed from the factors
// (stencil or potential product), the right one a cyclic window of G, so the
// shifted copies are never materialised -- and each wave accumulates a
// 32 x 32 sub-tile with MFMA.  Partial tiles of the splits are summed by a
// grouped reduction that also scatters to the Gram layout [t][s][mu][nu].
//
// Arithmetic: FP64 (v_mfma_f64_16x16x4f64), FP32 operands
// (v_mfma_f32_16x16x4f32), or hi+lo split products hi*hi + hi*lo + lo*hi in
// bf16 (v_mfma_f32_16x16x32_bf16) or FP16 (v_mfma_f32_16x16x32_f16), the last
// three with FP32 accumulation.  FP16 has five exponent bits, so each work
// item first scales every operand row and column by a power of two that puts
// its largest value over the item's nodes in [2^13, 2^14); the FP16 hi and lo
// then carry 22 bits of each value, and the scales come off exactly when the
// item's partial tile is written.
#include <algorithm>
#include <type_traits>

#include "plan.h"

namespace lhf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int KC = 32;   // window nodes per LDS chunk

__device__ __forceinline__ double gval(const double* G, const DimDev& D, int m0, int j, int f) {
  if (D.periodic) {
    if (j < 0) j += D.n; else if (j >= D.n) j -= D.n;
  } else if (j < 0 || j >= D.n) {
    return 0.0;
  }
  return G[(int64_t)j * m0 + f];
}

// TL: workgroup output tile (rows and columns), 64 or 32; the four wavefronts
// each own a TL/2 x TL/2 quarter (2 x 2 or 1 x 1 MFMA tiles).  The 32 tile
// gives launches with fewer work items than CUs four times the items.
template <int MODE, int TL>
__global__ void __launch_bounds__(256) gram_kernel(const LatDev* __restrict__ lats,
                                                   const GramItem* __restrict__ items, int nitems,
                                                   const double* __restrict__ fac, void* __restrict__ part_) {
  // one chunk buffer; the global loads of chunk c+1 go to registers and are
  // in flight while the MFMAs of chunk c run
  __shared__ double As[KC][TL + 1];
  __shared__ double Bs[KC][TL + 1];
  __shared__ int scA[MODE == 3 ? TL : 1], scB[MODE == 3 ? TL : 1];   // FP16 scale exponents
  typedef typename std::conditional<MODE == 0, d4, f4>::type Acc;
  constexpr int NQ = 256 / TL;      // node groups of the staging threads
  constexpr int NV = KC / NQ;       // nodes staged per thread and chunk
  constexpr int WS = TL / 2, NA = WS / 16;   // wave quarter and its MFMA tiles per side
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const GramItem item = items[it];
    const LatDev& L = lats[item.li];
    const DimDev& D = L.dim[item.d];
    const int m0 = L.m0, M = L.T * m0, N = D.nshift * m0;
    const double* G = fac + D.g_off;
    const double* P = fac + D.p_off;
    const int row0 = item.tm * TL, col0 = item.tn * TL;
    const int wr = (wave >> 1) * WS, wc = (wave & 1) * WS;   // wave quarter within the tile
    Acc acc[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NA; ++b) acc[a][b] = Acc{0, 0, 0, 0};
    const int k_beg = item.ks * D.kchunk;
    const int k_end = min(D.kwin, k_beg + D.kchunk);
    // this thread stages column `col` of both operand tiles, nodes kq + NQ v
    const int col = tid & (TL - 1), kq = tid / TL;
    const int r = row0 + col, c = col0 + col;
    const bool rok = r < M, cok = c < N;
    const int t = r / m0, nu = r - t * m0;
    const int slot = c / m0, mu = c - slot * m0;
    int sn = 0;
    if (D.periodic) {
      const int k = D.full ? slot : slot - D.L0;
      sn = (k * D.nc) % D.n;
      if (sn < 0) sn += D.n;
    }
    const double* Pt = P + (int64_t)(t >= 2 ? t - 2 : 0) * D.npot;
    const double h6 = D.h / 6.0, hinv = 1.0 / D.h;
    // raw operand values of one chunk: g0, (g-, g+) or (P, -), and the right operand
    double x0[NV], x1[NV], x2[NV], y[NV];
    auto load_chunk = [&](int kc0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int k = kc0 + kq + NQ * v;
        x0[v] = 0.0; x1[v] = 0.0; x2[v] = 0.0; y[v] = 0.0;
        if (k < k_end) {
          int i = D.kstart + k;
          if (i >= D.n) i -= D.n;
          if (rok) {
            x0[v] = G[(int64_t)i * m0 + nu];
            if (t >= 2) {
              x1[v] = Pt[D.replicate ? i % D.nc : i];
            } else {
              x1[v] = gval(G, D, m0, i - 1, nu);
              x2[v] = gval(G, D, m0, i + 1, nu);
            }
          }
          if (cok) {
            int j = i - sn;
            if (j < 0) j += D.n;
            y[v] = G[(int64_t)j * m0 + mu];
          }
        }
      }
    };
    auto store_chunk = [&]() {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int kk = kq + NQ * v;
        As[kk][col] = t >= 2 ? x1[v] * x0[v]
                          : t == 0 ? h6 * (x1[v] + 4.0 * x0[v] + x2[v]) : hinv * (2.0 * x0[v] - x1[v] - x2[v]);
        Bs[kk][col] = y[v];
      }
    };
    auto aval = [&](int v) {
      return t >= 2 ? x1[v] * x0[v] : t == 0 ? h6 * (x1[v] + 4.0 * x0[v] + x2[v]) : hinv * (2.0 * x0[v] - x1[v] - x2[v]);
    };
    double fa[NA], fb[NA];   // FP16: this lane's row and column scales
    if constexpr (MODE == 3) {
      // largest |value| of every A row and B column over the item's nodes
      double ma = 0.0, mb = 0.0;
      for (int kc0 = k_beg; kc0 < k_end; kc0 += KC) {
        load_chunk(kc0);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          ma = fmax(ma, fabs(aval(v)));
          mb = fmax(mb, fabs(y[v]));
        }
      }
      As[kq][col] = ma;
      Bs[kq][col] = mb;
      __syncthreads();
      if (tid < TL) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < NQ; ++q) {
          a = fmax(a, As[q][tid]);
          b = fmax(b, Bs[q][tid]);
        }
        int ea = 0, eb = 0;
        (void)frexp(a, &ea);
        (void)frexp(b, &eb);
        // capped so that 2^sc stays finite: a row or column whose largest
        // value is below 2^-886 (a far tail of a Gaussian in this item's
        // nodes) then underflows to zero in FP16, below any FP32 output
        scA[tid] = a > 0.0 ? min(14 - ea, 900) : 0;
        scB[tid] = b > 0.0 ? min(14 - eb, 900) : 0;
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        fa[a] = ldexp(1.0, scA[wr + a * 16 + lr]);
        fb[a] = ldexp(1.0, scB[wc + a * 16 + lr]);
      }
    }
    if (k_beg < k_end) {
      load_chunk(k_beg);
      store_chunk();
    }
    __syncthreads();
    for (int kc0 = k_beg; kc0 < k_end; kc0 += KC) {
      const bool more = kc0 + KC < k_end;
      if (more) load_chunk(kc0 + KC);
      if constexpr (MODE == 3) {
        h8 ah[NA], al[NA], bh[NA], bl[NA];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const float x = (float)(As[8 * lk + e][wr + a * 16 + lr] * fa[a]);
            const _Float16 hi = (_Float16)x;
            ah[a][e] = hi;
            al[a][e] = (_Float16)(x - (float)hi);
          }
#pragma unroll
          for (int b = 0; b < NA; ++b) {
            const float x = (float)(Bs[8 * lk + e][wc + b * 16 + lr] * fb[b]);
            const _Float16 hi = (_Float16)x;
            bh[b][e] = hi;
            bl[b][e] = (_Float16)(x - (float)hi);
          }
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NA; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
      } else if constexpr (MODE == 2) {
        bf8 ah[NA], al[NA], bh[NA], bl[NA];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const float x = (float)As[8 * lk + e][wr + a * 16 + lr];
            const __bf16 hi = (__bf16)x;
            ah[a][e] = hi;
            al[a][e] = (__bf16)(x - (float)hi);
          }
#pragma unroll
          for (int b = 0; b < NA; ++b) {
            const float x = (float)Bs[8 * lk + e][wc + b * 16 + lr];
            const __bf16 hi = (__bf16)x;
            bh[b][e] = hi;
            bl[b][e] = (__bf16)(x - (float)hi);
          }
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NA; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NA; ++b) {
              const double x = As[kk + lk][wr + a * 16 + lr];
              const double yy = Bs[kk + lk][wc + b * 16 + lr];
              if constexpr (MODE == 0)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, yy, acc[a][b], 0, 0, 0);
              else
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)x, (float)yy, acc[a][b], 0, 0, 0);
            }
        }
      }
      __syncthreads();
      if (more) {
        store_chunk();
        __syncthreads();
      }
    }
    // result layout: f64 MFMA row lk + 4 v; f32 / bf16 MFMA row 4 lk + v; column lr
    typedef typename std::conditional<MODE == 0, double, float>::type T;
    T* out = reinterpret_cast<T*>(part_) + D.part_off + (int64_t)item.ks * M * N;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NA; ++b) {
        const int c = col0 + wc + b * 16 + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rl = wr + a * 16 + (MODE == 0 ? lk + 4 * v : 4 * lk + v), r = row0 + rl;
          if (r < M && c < N) {
            if constexpr (MODE == 3)
              out[(int64_t)r * N + c] = ldexpf(acc[a][b][v], -(scA[rl] + scB[wc + b * 16 + lr]));
            else
              out[(int64_t)r * N + c] = (T)acc[a][b][v];
          }
        }
      }
  }
}

// Sum the split partials and scatter C[(t, nu)][(s, mu)] to Gram[t][s][mu][nu];
// blockIdx.y enumerates (lattice, dimension).  Each workgroup step takes nb
// whole m0 x m0 blocks (t, s) and transposes them through LDS: the partials
// are read along mu (contiguous in C) and the Grams written along nu
// (contiguous in the Gram layout).
template <typename T>
__global__ void __launch_bounds__(256) gram_reduce_kernel(const LatDev* __restrict__ lats,
                                                          const T* __restrict__ part, T* __restrict__ grams) {
  __shared__ T tile[512];   // nb blocks of m0 x (m0 + 1) (m0^2 <= 256), or m0 x (256 / m0 + 1)
  const int li = blockIdx.y / 3, d = blockIdx.y % 3;
  const LatDev& L = lats[li];
  const DimDev& D = L.dim[d];
  const int m0 = L.m0, m2 = m0 * m0;
  const int N = D.nshift * m0;
  const int64_t MN = (int64_t)L.T * m0 * N;
  const int nblocks = L.T * D.nshift;
  const T* src0 = part + D.part_off;
  if (m2 <= 256) {
    const int nb = 256 / m2, tid = threadIdx.x;
    const int bl = tid / m2, e = tid - bl * m2;
    for (int b0 = blockIdx.x * nb; b0 < nblocks; b0 += gridDim.x * nb) {
      const int b = b0 + bl;
      const bool ok = bl < nb && b < nblocks;
      if (ok) {
        const int t = b / D.nshift, slot = b - t * D.nshift;
        const int nu = e / m0, mu = e - nu * m0;
        const T* src = src0 + (int64_t)(t * m0 + nu) * N + slot * m0 + mu;
        T acc = 0;
        for (int ks = 0; ks < D.ksplit; ++ks) acc += src[(int64_t)ks * MN];
        tile[bl * (m2 + m0) + nu * (m0 + 1) + mu] = acc;
      }
      __syncthreads();
      if (ok) {
        const int mu = e / m0, nu = e - mu * m0;
        grams[D.gram_off + (int64_t)b * m2 + e] = tile[bl * (m2 + m0) + nu * (m0 + 1) + mu];
      }
      __syncthreads();
    }
  } else {
    // m0 > 16: one block per step, in row groups of 256 / m0 rows nu
    const int rows = 256 / m0, tid = threadIdx.x;
    const int rr = tid / m0, mu = tid - rr * m0;
    for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
      const int t = b / D.nshift, slot = b - t * D.nshift;
      for (int nu0 = 0; nu0 < m0; nu0 += rows) {
        const int nu = nu0 + rr;
        const bool ok = rr < rows && nu < m0;
        if (ok) {
          const T* src = src0 + (int64_t)(t * m0 + nu) * N + slot * m0 + mu;
          T acc = 0;
          for (int ks = 0; ks < D.ksplit; ++ks) acc += src[(int64_t)ks * MN];
          tile[mu * (rows + 1) + rr] = acc;
        }
        __syncthreads();
        // write rows mu, columns nu0 .. nu0 + rows - 1 (runs of `rows` doubles)
        const int wmu = tid / rows, wr = tid - wmu * rows;
        if (wmu < m0 && nu0 + wr < m0)
          grams[D.gram_off + (int64_t)b * m2 + (int64_t)wmu * m0 + nu0 + wr] = tile[wmu * (rows + 1) + wr];
        __syncthreads();
      }
    }
  }
}

}  // namespace

hipError_t launch_grams(const lhf_plan_s* p, int mode, const double* fac, void* part, void* grams,
                        hipStream_t s) {
  const int grid = std::min(p->n_gram_items, p->gram_grid);
  const bool t32 = p->gram_tile == 32;
  if (mode == LHF_GRAM_FP64) {
    if (t32) hipLaunchKernelGGL((gram_kernel<0, 32>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
    else hipLaunchKernelGGL((gram_kernel<0, 64>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
  } else if (mode == LHF_GRAM_FP32) {
    if (t32) hipLaunchKernelGGL((gram_kernel<1, 32>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
    else hipLaunchKernelGGL((gram_kernel<1, 64>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
  } else if (mode == LHF_GRAM_BF16X3) {
    if (t32) hipLaunchKernelGGL((gram_kernel<2, 32>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
    else hipLaunchKernelGGL((gram_kernel<2, 64>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
  } else {
    if (t32) hipLaunchKernelGGL((gram_kernel<3, 32>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
    else hipLaunchKernelGGL((gram_kernel<3, 64>), dim3(grid), dim3(256), 0, s, p->d_lat, p->d_gram_items, p->n_gram_items, fac, part);
  }
  int64_t maxmn = 0;
  for (const LatDev& L : p->lat)
    for (int d = 0; d < 3; ++d) maxmn = std::max<int64_t>(maxmn, (int64_t)L.T * L.m0 * L.dim[d].nshift * L.m0);
  // about one output element per thread (256 per workgroup step)
  const dim3 rgrid((unsigned)std::max<int64_t>(1, std::min<int64_t>((maxmn + 255) / 256, 1024)), (unsigned)(3 * p->nlat));
  if (mode == LHF_GRAM_FP64)
    hipLaunchKernelGGL(gram_reduce_kernel<double>, rgrid, dim3(256), 0, s, p->d_lat, (const double*)part, (double*)grams);
  else
    hipLaunchKernelGGL(gram_reduce_kernel<float>, rgrid, dim3(256), 0, s, p->d_lat, (const float*)part, (float*)grams);
  return hipGetLastError();
}

}  // namespace lhf
