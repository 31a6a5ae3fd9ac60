// Sturm counts of a real symmetric tridiagonal matrix T (diagonal d_j,
// squared subdiagonal e2_j = e_(j-1)^2), scaled to norm below one.
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
// minor is zero and the sign changes of the trailing block are lost.  So at a
// split the recurrence restarts, p_(j-1) = 1 and p_(j-2) = 0, which gives the
// trailing block's own minors; with p_(j-1) != 0 the restart only rescales
// them, so the count is the same either way (sturm_row with SPLIT).  Matrices
// without a zero coupling take the plain row (SPLIT false), which computes the
// same counts with fewer operations.
//
// A sign change is read from the sign bits of consecutive minors (integer
// operations only).  A zero minor then counts by the sign of its zero, which
// does not change the total: a zero p_(j-1) is isolated, p_j = -e^2 p_(j-2)
// and p_(j-2) have opposite signs, so exactly one of the two changes around
// it is counted whatever sign the zero carries; after a restart the zero is
// +0.
//
// Shared by the bisection kernel and the host tests.
#pragma once

#include <hip/hip_runtime.h>

namespace lhf {

// The sign bit of x: 1 or 0.
__host__ __device__ inline int sign_bit(double x) {
  return (int)(__builtin_bit_cast(unsigned long long, x) >> 63);
}
__host__ __device__ inline int sign_bit(float x) { return (int)(__builtin_bit_cast(unsigned int, x) >> 31); }

// One row: p1 = p_(j-1), p2 = p_(j-2), neg = sign bit of p_(j-1), cnt = sign
// changes so far; all four are advanced to row j.
template <bool SPLIT, typename R>
__host__ __device__ inline void sturm_row(R d, R e2, R x, R& p1, R& p2, int& neg, int& cnt) {
  R q1 = p1, q2 = p2;
  int n1 = neg;
  if constexpr (SPLIT) {
    const bool split = e2 == R(0);
    q1 = split ? R(1) : p1;
    q2 = split ? R(0) : p2;
    n1 = split ? 0 : neg;
  }
  const R p = fma(d - x, q1, -e2 * q2);
  const int m = sign_bit(p);
  cnt += m ^ n1;
  neg = m;
  p2 = q1;
  p1 = p;
}

// Count of eigenvalues of the n x n tridiagonal (d, e2) below x (e2[0]
// unused), rescaling the minors by 2^-+256 every eighth row (exact and
// sign-preserving; T below unit norm, so the minors grow at most 3x per row),
// as the bisection kernel computes it.
template <bool SPLIT, typename R>
__host__ __device__ inline int sturm_count(const R* d, const R* e2, int n, R x) {
  const R kBig = R(1.157920892373162e77), kSmall = R(8.636168555094445e-78);   // 2^256, 2^-256
  R p1 = d[0] - x, p2 = R(1);
  int neg = sign_bit(p1);
  int cnt = neg;
  for (int j = 1; j < n; ++j) {
    sturm_row<SPLIT>(d[j], e2[j], x, p1, p2, neg, cnt);
    if ((j & 7) == 7) {
      const R s = fabs(p1) > kBig ? kSmall : (fabs(p1) < kSmall ? kBig : R(1));
      p1 *= s;
      p2 *= s;
    }
  }
  return cnt;
}

}  // namespace lhf
