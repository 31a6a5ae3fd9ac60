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

// Grouped factor launch: one workgroup per work item, for every lattice.
//  * item.chunk >= 0: 256 nodes of one row of dimension item.d -- a basis
//    function (row < m0, every dimension) or a potential term (row - m0) of a
//    one-cell dimension, evaluated on the cell's own nodes;
//  * item.chunk < 0: the lattice-window potential factor (eq. EwaldSumP) of
//    term item.row of a replicated dimension.  Thread t sums the images
//    k = klo + c, c = t / nc (mod 256 / nc), for node t % nc of the central
//    cell; the chunk sums are added in a fixed order, so the result is
//    deterministic.
__global__ void __launch_bounds__(256) factors_kernel(const LatDev* __restrict__ lats,
                                                      const FacItem* __restrict__ items, int nitems,
                                                      double* __restrict__ fac) {
  __shared__ double part[256];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const FacItem item = items[it];
    const LatDev& L = lats[item.li];
    const DimDev& D = L.dim[item.d];
    const int d = item.d;
    if (item.chunk >= 0) {
      const int i = item.chunk * 256 + threadIdx.x;
      const int row = item.row;
      if (row < L.m0) {
        if (i < D.n) {
          const int mu = row;
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
          fac[D.g_off + (int64_t)i * L.m0 + mu] = L.norm[mu][d] * acc;
        }
      } else if (i < D.npot) {
        const int r = row - L.m0;   // potential term nu R + q
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
    const int nc = D.nc;
    const int chunks = 256 / nc;
    const int tid = threadIdx.x;
    const int j = tid % nc, c = tid / nc;
    int klo, khi;
    if (D.L & 1) { klo = -(D.L - 1) / 2; khi = (D.L - 1) / 2; }
    else { klo = -D.L / 2; khi = D.L / 2; }
    double acc = 0.0;
    if (c < chunks) {
      const double y = D.y0 + j * D.h;
      for (int k = klo + c; k <= khi; k += chunks) {
        const double wk = ((D.L & 1) == 0 && (k == klo || k == khi)) ? 0.5 : 1.0;
        acc += wk * cell_gauss(y, D.h, t, A + k * D.a);
      }
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < nc) {
      double v = 0.0;
      for (int cc = 0; cc < chunks; ++cc) v += part[cc * nc + tid];
      if (d == 0) v *= L.Z[nu] * L.wq[q];
      fac[D.p_off + (int64_t)r * D.npot + tid] = v;
    }
    __syncthreads();   // part[] is reused by the next item
  }
}

}  // namespace

void plan_factors(const std::vector<LatDev>& lats, std::vector<FacItem>& items) {
  items.clear();
  for (int li = 0; li < (int)lats.size(); ++li) {
    const LatDev& L = lats[li];
    // window items first: they are the long ones
    for (int d = 0; d < 3; ++d)
      if (L.dim[d].replicate)
        for (int r = 0; r < L.M0 * L.R; ++r) items.push_back(FacItem{li, d, r, -1});
    for (int d = 0; d < 3; ++d) {
      const DimDev& D = L.dim[d];
      for (int row = 0; row < L.m0; ++row)
        for (int ch = 0; ch < (D.n + 255) / 256; ++ch) items.push_back(FacItem{li, d, row, ch});
      if (!D.replicate)
        for (int r = 0; r < L.M0 * L.R; ++r)
          for (int ch = 0; ch < (D.npot + 255) / 256; ++ch) items.push_back(FacItem{li, d, L.m0 + r, ch});
    }
  }
}

hipError_t launch_factors(const lhf_plan_s* p, double* fac, hipStream_t s) {
  const int grid = std::min(p->n_fac_items, 8192);
  hipLaunchKernelGGL(factors_kernel, dim3(grid), dim3(256), 0, s, p->d_lat, p->d_fac_items, p->n_fac_items, fac);
  return hipGetLastError();
}

}  // namespace lhf
