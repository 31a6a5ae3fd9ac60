// Eigenvectors of the full lattice problem from the Fourier-block
// eigenvectors (Prop. 5.1, eq. eigvecA): U = (F^* x I_m0) bdiag(Ubar_j) with
// F = F_L1 x F_L2 x F_L3, (F_L)_(j,k) = w^(j k) / sqrt(L), w = exp(-2 pi i / L).
// Column c of Ubar_j becomes the vector whose block on cell k is
//   U(k, mu) = L^(-1/2) conj(w1^(j1 k1) w2^(j2 k2) w3^(j3 k3)) Ubar_j(mu, c).
// One thread per output entry (selection, cell, mu), mu fastest, so the
// stores of a wavefront are contiguous; the phase comes from the plan's
// twiddle table exp(-2 pi i m / L_l), conjugated.  The work is one complex
// write per entry: HBM-write bound.
#include <cmath>
#include <string>

#include "plan.h"

namespace lhf {
namespace {

__global__ void __launch_bounds__(256) eigvec_kernel(const LatDev* __restrict__ lat, const double2* __restrict__ tw,
                                                     const double2* __restrict__ V, int64_t nout,
                                                     const int32_t* __restrict__ sel, double2* __restrict__ U) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= nout) return;
  const LatDev& L = *lat;
  const int m0 = L.m0, nblk = L.nblk, L1 = L.L[0], L2 = L.L[1], L3 = L.L[2];
  const int mu = (int)(idx % m0);
  const int64_t q = idx / m0;
  const int k = (int)(q % nblk);
  const int64_t s = q / nblk;
  const int j = sel[2 * s], c = sel[2 * s + 1];
  if (j < 0 || j >= nblk || c < 0 || c >= m0) {
    U[idx] = make_double2(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  const int j1 = j / (L2 * L3), j2 = (j / L3) % L2, j3 = j % L3;
  const int k1 = k / (L2 * L3), k2 = (k / L3) % L2, k3 = k % L3;
  const double2 t1 = tw[L.dim[0].tw_off + (j1 * k1) % L1];
  const double2 t2 = tw[L.dim[1].tw_off + (j2 * k2) % L2];
  const double2 t3 = tw[L.dim[2].tw_off + (j3 * k3) % L3];
  // conj(t1 t2 t3) / sqrt(L)
  const double ax = t1.x * t2.x - t1.y * t2.y, ay = t1.x * t2.y + t1.y * t2.x;
  const double sc = 1.0 / sqrt((double)nblk);
  const double px = (ax * t3.x - ay * t3.y) * sc, py = -(ax * t3.y + ay * t3.x) * sc;
  const double2 v = V[L.gen_off + ((int64_t)j * m0 + mu) * m0 + c];
  U[idx] = make_double2(px * v.x - py * v.y, px * v.y + py * v.x);
}

}  // namespace

hipError_t launch_eigvecs(const lhf_plan_s* p, int li, const double2* V, int nsel, const int32_t* sel, double2* U,
                          hipStream_t s) {
  const LatDev& L = p->lat[li];
  const int64_t nout = (int64_t)nsel * L.nblk * L.m0;
  const int64_t blocks = (nout + 255) / 256;
  hipLaunchKernelGGL(eigvec_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p->d_lat + li, p->d_tw64, V, nout, sel,
                     U);
  return hipGetLastError();
}

}  // namespace lhf

extern "C" int32_t lhf_eigvecs_lattice(lhf_plan_t p, int32_t lattice, const void* V, int32_t nsel,
                                       const int32_t* sel, void* U, lhf_stream_t stream) {
  if (!p) { lhf::set_error("NULL plan"); return LHF_ERR_INVALID; }
  if (lattice < 0 || lattice >= p->nlat) {
    lhf::set_error("lattice index " + std::to_string(lattice) + " out of range");
    return LHF_ERR_INVALID;
  }
  if (nsel < 0) { lhf::set_error("nsel < 0"); return LHF_ERR_INVALID; }
  if (nsel == 0) return LHF_OK;
  if (!V || !sel || !U) { lhf::set_error("V, sel and U are required"); return LHF_ERR_INVALID; }
  const lhf::LatDev& L = p->lat[lattice];
  const int64_t nout = (int64_t)nsel * L.nblk * L.m0;
  if ((nout + 255) / 256 > 0x7fffffffLL) {
    lhf::set_error("too many output entries for one launch");
    return LHF_ERR_UNSUPPORTED;
  }
  const hipError_t e = lhf::launch_eigvecs(p, lattice, static_cast<const double2*>(V), nsel, sel,
                                           static_cast<double2*>(U), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    lhf::set_error(std::string("eigenvector back-transform: ") + hipGetErrorString(e));
    return LHF_ERR_HIP;
  }
  return LHF_OK;
}
