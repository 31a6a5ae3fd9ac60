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
                                                       typename Cx<R>::T* __restrict__ barS) {
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
  C* Y = T.out_final ? (isH ? barH : barS) + L.gen_off : tmp + T.out_off + (isH ? 0 : T.out_half);
  C* dst = Y + (int64_t)o * Ld * I + i;
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
    dst[(int64_t)j * I] = r;
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
                                                       typename Cx<R>::T* __restrict__ barS) {
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
  C* Y = T.out_final ? (isH ? barH : barS) + L.gen_off : tmp + T.out_off + (isH ? 0 : T.out_half);
  C r;
  r.x = re;
  r.y = im;
  Y[tid] = r;
}

int band_class(int B) { return B <= 4 ? 0 : B <= 8 ? 1 : B <= 16 ? 2 : B <= 32 ? 3 : 4; }

template <typename R>
hipError_t dft_launch_all(const lhf_plan_s* p, const R* gH, const R* gS, typename Cx<R>::T* bH,
                          typename Cx<R>::T* bS, typename Cx<R>::T* tmp, const typename Cx<R>::T* tw,
                          hipStream_t s) {
  typedef typename Cx<R>::T C;
  for (const DftLaunch& l : p->dft_launches) {
    const dim3 grid((unsigned)(l.threads / 256), 2);
    const DftTask* tk = p->d_dft_tasks + l.t0;
    const size_t shb = sizeof(C) * (size_t)l.lds_tw;
    const bool first = l.pass == 0;
#define LHF_PASS(BM)                                                                                      \
  if (first)                                                                                              \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, true>), grid, dim3(256), shb, s, p->d_lat, tk, l.nt, tw,   \
                       gH, gS, tmp, bH, bS);                                                              \
  else                                                                                                    \
    hipLaunchKernelGGL((dft_pass_kernel<R, BM, false>), grid, dim3(256), shb, s, p->d_lat, tk, l.nt, tw,  \
                       gH, gS, tmp, bH, bS);
    switch (l.cls) {
      case 0: LHF_PASS(4) break;
      case 1: LHF_PASS(8) break;
      case 2: LHF_PASS(16) break;
      case 3: LHF_PASS(32) break;
      default:
        if (first)
          hipLaunchKernelGGL((dft_wide_kernel<R, true>), grid, dim3(256), 0, s, p->d_lat, tk, l.nt, tw, gH, gS,
                             tmp, bH, bS);
        else
          hipLaunchKernelGGL((dft_wide_kernel<R, false>), grid, dim3(256), 0, s, p->d_lat, tk, l.nt, tw, gH, gS,
                             tmp, bH, bS);
    }
#undef LHF_PASS
  }
  return hipGetLastError();
}

}  // namespace

void plan_block_dft(const std::vector<LatDev>& lats, int64_t target_threads, std::vector<DftTask>& tasks,
                    std::vector<DftLaunch>& launches, int64_t& tmp_elems) {
  tasks.clear();
  launches.clear();
  const int nlat = (int)lats.size();
  // per lattice: the transformed dimensions, last non-trivial first (a
  // one-cell lattice is a single pass over dimension 3 that copies)
  std::vector<std::vector<int>> dims(nlat);
  for (int li = 0; li < nlat; ++li) {
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

hipError_t launch_block_dft(const lhf_plan_s* p, int prec, const void* gen_h, const void* gen_s, void* bar_h,
                            void* bar_s, void* tmp, hipStream_t s) {
  if (prec == LHF_PREC_FP64)
    return dft_launch_all<double>(p, (const double*)gen_h, (const double*)gen_s, (double2*)bar_h, (double2*)bar_s,
                                  (double2*)tmp, p->d_tw64, s);
  return dft_launch_all<float>(p, (const float*)gen_h, (const float*)gen_s, (float2*)bar_h, (float2*)bar_s,
                               (float2*)tmp, p->d_tw32, s);
}

}  // namespace lhf
