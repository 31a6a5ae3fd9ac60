// One-dimensional factors of one lattice, in FP64:
//  * nodal values of every basis function of cell 0 (Sec. 2.4 interpolant),
//    periodised over supercell translates on periodic dimensions;
//  * the collocated, lattice-summed potential factor of every (nucleus, sinc
//    term) pair (eqs. galten, sinc_general, EwaldTensorGl, EwaldSumP): on a
//    replicated dimension the sum over the L-image window centred on a cell is
//    stored for one cell's nodes; on a one-cell dimension the cell's own
//    nucleus is evaluated on every node.  Z_nu w_q is folded into dimension 1.
#include <algorithm>

#include "gauss.h"
#include "plan.h"

namespace lhf {
namespace {

// Grouped factor launch: one workgroup of FT threads per work item, for
// every lattice.
//  * item.row < 0: the nodal values of every basis function on nodes
//    [chunk FT/m0, (chunk + 1) FT/m0) of dimension item.d; thread t takes
//    function t % m0 of node t / m0, so the node-major store [i][m0] is
//    contiguous across the workgroup;
//  * item.row >= 0, item.chunk >= 0: FT nodes of the potential term item.row of
//    a one-cell dimension, on the cell's own nodes;
//  * item.chunk < 0: the lattice-window potential factor (eq. EwaldSumP) of
//    term item.row of a replicated dimension, for the central cell's nodes
//    j0 .. j0 + nn - 1 (node group g = -1 - item.chunk of size nn, so that
//    every thread sums about one image).  Thread t sums the images
//    k = klo + c, c = t / nn (mod FT / nn), for node j0 + t % nn; the image
//    partial sums are folded in two fixed-order levels, so the result is
//    deterministic.
constexpr int FT = 1024;
constexpr int kFold = 32;   // first-level fold width of the window partials

// Nodes per group of a window item: groups enough that the FT threads of a
// workgroup cover every (node, image) pair about once, at most one per node.
// The item count is ceil(nc / nn), every group non-empty.
__host__ __device__ inline int window_nodes(int nc, int L) {
  int ng = (nc * L + FT - 1) / FT;
  ng = ng < 1 ? 1 : (ng > nc ? nc : ng);
  return (nc + ng - 1) / ng;
}

__global__ void __launch_bounds__(FT) factors_kernel(const LatDev* __restrict__ lats,
                                                     const FacItem* __restrict__ items, int nitems,
                                                     double* __restrict__ fac) {
  __shared__ double part[FT];
  __shared__ double part2[FT];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const FacItem item = items[it];
    const LatDev& L = lats[item.li];
    const DimDev& D = L.dim[item.d];
    const int d = item.d;
    const int tid = threadIdx.x;
    if (item.row < 0) {
      const int m0 = L.m0, per = FT / m0;
      const int mu = tid % m0, i = item.chunk * per + tid / m0;
      if (tid < per * m0 && i < D.n) {
        const double al = L.alpha[mu];
        const double c = D.X0 + L.cen[mu][d];
        const double x = D.x0 + i * D.h;
        const int pw = L.lpow[mu][d];
        double acc = 0.0;
        for (int s = -D.nimg; s <= D.nimg; ++s) {
          const double u = x - c - s * D.period;
          const double g = exp(-al * u * u);
          acc += pw ? g * u : g;
        }
        fac[D.g_off + (int64_t)i * m0 + mu] = L.norm[mu][d] * acc;
      }
      continue;
    }
    if (item.chunk >= 0) {
      const int i = item.chunk * FT + tid;
      if (i < D.npot) {
        const int r = item.row;   // potential term nu R + q
        const int nu = r / L.R, q = r % L.R;
        double v = cell_gauss(D.x0 + i * D.h, D.h, L.tq[q], D.X0 + L.nuc[nu][d]);
        if (d == 0) v *= L.Z[nu] * L.wq[q];
        fac[D.p_off + (int64_t)r * D.npot + i] = v;
      }
      continue;
    }
    const int r = item.row;
    const int nu = r / L.R, q = r % L.R;
    const double t = L.tq[q], A = L.nuc[nu][d];
    const int nn = window_nodes(D.nc, D.L), j0 = (-1 - item.chunk) * nn;
    const int nc = min(nn, D.nc - j0);   // nodes of this group (>= 1)
    const int chunks = FT / nc;
    const int j = tid % nc, c = tid / nc;
    int klo, khi;
    if (D.L & 1) { klo = -(D.L - 1) / 2; khi = (D.L - 1) / 2; }
    else { klo = -D.L / 2; khi = D.L / 2; }
    double acc = 0.0;
    if (c < chunks) {
      const double y = D.y0 + (j0 + j) * D.h;
      for (int k = klo + c; k <= khi; k += chunks) {
        const double wk = ((D.L & 1) == 0 && (k == klo || k == khi)) ? 0.5 : 1.0;
        acc += wk * cell_gauss(y, D.h, t, A + k * D.a);
      }
    }
    part[tid] = acc;
    __syncthreads();
    // level 1: partial g of node j sums chunks g, g + G1, g + 2 G1, ...
    const int G1 = chunks < kFold ? chunks : kFold;
    if (c < G1) {
      double v = 0.0;
      for (int cc = c; cc < chunks; cc += G1) v += part[cc * nc + j];
      part2[c * nc + j] = v;
    }
    __syncthreads();
    if (tid < nc) {
      double v = 0.0;
      for (int g = 0; g < G1; ++g) v += part2[g * nc + tid];
      if (d == 0) v *= L.Z[nu] * L.wq[q];
      fac[D.p_off + (int64_t)r * D.npot + j0 + tid] = v;
    }
    __syncthreads();   // part[] and part2[] are reused by the next item
  }
}

}  // namespace

void plan_factors(const std::vector<LatDev>& lats, std::vector<FacItem>& items) {
  items.clear();
  for (int li = 0; li < (int)lats.size(); ++li) {
    const LatDev& L = lats[li];
    // window items first: they are the long ones
    for (int d = 0; d < 3; ++d)
      if (L.dim[d].replicate) {
        const int nn = window_nodes(L.dim[d].nc, L.dim[d].L), ng = (L.dim[d].nc + nn - 1) / nn;
        for (int r = 0; r < L.M0 * L.R; ++r)
          for (int g = 0; g < ng; ++g) items.push_back(FacItem{li, d, r, -1 - g});
      }
    for (int d = 0; d < 3; ++d) {
      const DimDev& D = L.dim[d];
      const int per = FT / L.m0;   // nodes per basis chunk
      for (int ch = 0; ch < (D.n + per - 1) / per; ++ch) items.push_back(FacItem{li, d, -1, ch});
      if (!D.replicate)
        for (int r = 0; r < L.M0 * L.R; ++r)
          for (int ch = 0; ch < (D.npot + FT - 1) / FT; ++ch) items.push_back(FacItem{li, d, r, ch});
    }
  }
  // longest first over the whole plan (LPT): a window item sums its node
  // group over the L + 1 images, the others evaluate one chunk of FT values
  auto cost = [&](const FacItem& it) -> int64_t {
    if (it.chunk >= 0) return FT;
    const DimDev& D = lats[it.li].dim[it.d];
    return (int64_t)window_nodes(D.nc, D.L) * (D.L + 1);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const FacItem& a, const FacItem& b) { return cost(a) > cost(b); });
}

hipError_t launch_factors(const lhf_plan_s* p, double* fac, hipStream_t s) {
  const int grid = std::min(p->n_fac_items, 8192);
  hipLaunchKernelGGL(factors_kernel, dim3(grid), dim3(FT), 0, s, p->d_lat, p->d_fac_items, p->n_fac_items, fac);
  return hipGetLastError();
}

}  // namespace lhf
