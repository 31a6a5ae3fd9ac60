// Device helper shared by the kernels that collocate the rank-R potential:
// the integral of one Gaussian term over the piecewise-constant cell of a node
// (eq. galten, one dimension).
#pragma once

#include <hip/hip_runtime.h>

namespace lhf {

// Integral of exp(-t^2 (y - A)^2) over [x - h/2, x + h/2].  With u = t h and
// v = t (x - A): when the cell is much narrower than the Gaussian
// (u <= 0.1 and u |v| <= 0.1) the erf difference would cancel, so the
// midpoint expansion h exp(-v^2) sum_k u^2k H_2k(v) / (4^k (2k+1)!), k <= 4,
// is used (H_n: physicists' Hermite polynomials); otherwise the difference
// of erf, or of erfc on the far side of A.
__device__ inline double cell_gauss(double x, double h, double t, double A) {
  const double u = t * h, v = t * (x - A);
  if (u <= 0.1 && u * fabs(v) <= 0.1) {
    const double v2 = v * v, u2 = u * u;
    const double H2 = 4.0 * v2 - 2.0;
    const double H4 = (16.0 * v2 - 48.0) * v2 + 12.0;
    const double H6 = ((64.0 * v2 - 480.0) * v2 + 720.0) * v2 - 120.0;
    const double H8 = (((256.0 * v2 - 3584.0) * v2 + 13440.0) * v2 - 13440.0) * v2 + 1680.0;
    const double s = 1.0 + u2 * (H2 / 24.0 + u2 * (H4 / 1920.0 + u2 * (H6 / 322560.0 + u2 * H8 / 92897280.0)));
    return h * exp(-v2) * s;
  }
  const double lo = t * (x - 0.5 * h - A);
  const double hi = t * (x + 0.5 * h - A);
  if (lo > 27.5 || hi < -27.5) return 0.0;   // erfc below the smallest double
  double d;
  if (lo > 0.0) d = erfc(lo) - erfc(hi);
  else if (hi < 0.0) d = erfc(-hi) - erfc(-lo);
  else d = erf(hi) - erf(lo);
  return d * (0.886226925452758014 / t);  // sqrt(pi) / 2
}

}  // namespace lhf
