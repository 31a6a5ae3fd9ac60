// One row of a Sturm count of a real symmetric tridiagonal matrix T (diagonal
// d_j, squared subdiagonal e2_j = e_(j-1)^2) at a shift x.
//
// The count of eigenvalues of T below x is the number of sign changes of the
// leading principal minors p_j of T - x I, which obey
//   p_j = (d_j - x) p_(j-1) - e_(j-1)^2 p_(j-2),  p_(-1) = 1, p_(-2) = 0,
// with a zero minor taken as positive: with e != 0 a zero p_(j-1) makes
// p_j = -e^2 p_(j-2), of the opposite sign of p_(j-2), so the zero still
// counts once, as in the ratio form with zero pivots made negative.
//
// A zero coupling e_(j-1) = 0 splits T into independent blocks whose
// characteristic polynomials multiply, and the count is the sum of the
// blocks' counts.  The product form cannot carry that through a zero: once
// p_(j-1) = 0 exactly (x an eigenvalue of the leading block), every later
// minor is zero and the sign changes of the trailing block are lost.  So the
// recurrence restarts at a split, p_(j-1) = 1 and p_(j-2) = 0, which gives the
// trailing block's own minors; with p_(j-1) != 0 the restart only rescales
// them, so the count is the same either way.
//
// The row function is shared by the bisection kernel and the host tests.
#pragma once

#include <hip/hip_runtime.h>

namespace lhf {

// p1 = p_(j-1), p2 = p_(j-2), neg = (p_(j-1) < 0), cnt = sign changes so far;
// all four are advanced to row j.
template <typename R>
__host__ __device__ inline void sturm_row(R d, R e2, R x, R& p1, R& p2, bool& neg, int& cnt) {
  const bool split = e2 == R(0);
  const R q1 = split ? R(1) : p1;
  const R q2 = split ? R(0) : p2;
  const bool n1 = split ? false : neg;
  const R p = fma(d - x, q1, -e2 * q2);
  const bool m = p < R(0);
  cnt += m != n1 ? 1 : 0;
  neg = m;
  p2 = q1;
  p1 = p;
}

// Count of eigenvalues of the n x n tridiagonal (d, e2) below x, rescaling
// the minors by 2^-+256 every eighth row (exact and sign-preserving); T is
// expected scaled to norm below one, so the minors grow at most 3x per row.
template <typename R>
__host__ __device__ inline int sturm_count(const R* d, const R* e2, int n, R x) {
  const R kBig = R(1.157920892373162e77), kSmall = R(8.636168555094445e-78);   // 2^256, 2^-256
  R p1 = d[0] - x, p2 = R(1);
  bool neg = p1 < R(0);
  int cnt = neg ? 1 : 0;
  for (int j = 1; j < n; ++j) {
    sturm_row(d[j], e2[j], x, p1, p2, neg, cnt);
    if ((j & 7) == 7) {
      const R s = fabs(p1) > kBig ? kSmall : (fabs(p1) < kSmall ? kBig : R(1));
      p1 *= s;
      p2 *= s;
    }
  }
  return cnt;
}

}  // namespace lhf
