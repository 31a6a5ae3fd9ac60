// Dense FP64 kernels of the block LOBPCG driver: Gram products of tall
// blocks, block combinations, residuals, Cholesky-QR orthonormalisation and a one-workgroup
// symmetric eigensolver for the Rayleigh-Ritz problems (size <= 112).
//
// Blocks of vectors are row-major [N][ld] (column j = vector j).  Reductions
// over N are split into fixed chunks whose partial results are added in chunk
// order, so every result is deterministic.
#include <algorithm>

#include "toeplitz.h"

namespace lhf {
namespace {

constexpr int kGT = 32;      // Gram output tile
constexpr int kGRows = 64;   // rows staged per step

// part[c][i][j] = sum over rows n of chunk c of A[n][i] B[n][j]
__global__ void __launch_bounds__(256) gram_part_kernel(int N, int k1, int k2, int chunk, const double* __restrict__ A,
                                                        int lda, const double* __restrict__ B, int ldb,
                                                        double* __restrict__ part) {
  __shared__ double As[kGRows][kGT + 1];
  __shared__ double Bs[kGRows][kGT + 1];
  const int c = blockIdx.x, i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  const int ti = threadIdx.x % kGT, tj = threadIdx.x / kGT;   // outputs (ti, tj + 8 u)
  double acc[4] = {0, 0, 0, 0};
  const int n0 = c * chunk, n1 = min(N, n0 + chunk);
  for (int nb = n0; nb < n1; nb += kGRows) {
    for (int e = threadIdx.x; e < kGRows * kGT; e += 256) {
      const int r = e / kGT, q = e % kGT, n = nb + r;
      As[r][q] = (n < n1 && i0 + q < k1) ? A[(int64_t)n * lda + i0 + q] : 0.0;
      Bs[r][q] = (n < n1 && j0 + q < k2) ? B[(int64_t)n * ldb + j0 + q] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < kGRows; ++r) {
      const double a = As[r][ti];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += a * Bs[r][tj + 8 * u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ti, j = j0 + tj + 8 * u;
    if (i < k1 && j < k2) part[((int64_t)c * k1 + i) * k2 + j] = acc[u];
  }
}

__global__ void __launch_bounds__(256) gram_reduce_kernel(int k1, int k2, int nchunk, const double* __restrict__ part,
                                                          double* __restrict__ G, int ldg) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= k1 * k2) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * k1 * k2 + e];
  G[(e / k2) * ldg + e % k2] = s;
}

constexpr int kCRows = 16;   // rows per combine workgroup

// Y = beta Z + A T
__global__ void __launch_bounds__(256) combine_kernel(int N, int k1, int k2, const double* __restrict__ A, int lda,
                                                      const double* __restrict__ T, int ldt, double beta,
                                                      const double* Z, int ldz, double* Y, int ldy) {
  __shared__ double As[kCRows][kMaxSmall];
  const int r0 = blockIdx.x * kCRows;
  for (int e = threadIdx.x; e < kCRows * k1; e += 256) {
    const int r = e / k1, i = e % k1;
    As[r][i] = r0 + r < N ? A[(int64_t)(r0 + r) * lda + i] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kCRows * k2; e += 256) {
    const int r = e / k2, j = e % k2, n = r0 + r;
    if (n >= N) continue;
    double s = 0.0;
    for (int i = 0; i < k1; ++i) s += As[r][i] * T[(int64_t)i * ldt + j];
    if (beta != 0.0) s += beta * Z[(int64_t)n * ldz + j];
    Y[(int64_t)n * ldy + j] = s;
  }
}

// R = HX - SX diag(theta); part[c][j] = sum over chunk rows of R^2
__global__ void __launch_bounds__(256) residual_kernel(int N, int k, int chunk, const double* __restrict__ HX,
                                                       const double* __restrict__ SX, int ld,
                                                       const double* __restrict__ theta, double* __restrict__ R,
                                                       int ldr, double* __restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int n0 = c * chunk, n1 = min(N, n0 + chunk);
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int n = n0 + threadIdx.x; n < n1; n += 256) {
      const double r = HX[(int64_t)n * ld + j] - SX[(int64_t)n * ld + j] * theta[j];
      R[(int64_t)n * ldr + j] = r;
      s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)c * k + j] = red[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) norms_kernel(int k, int nchunk, const double* __restrict__ part,
                                                    double* __restrict__ norms) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * k + j];
  norms[j] = sqrt(s);
}

// SplitMix64 (Steele, Lea and Flood, 2014): a counter-based stream; values
// uniform in [-1, 1).
__global__ void __launch_bounds__(256) random_kernel(int N, int k, uint64_t seed, double* __restrict__ X, int ld) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)N * k) return;
  uint64_t z = seed + (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[(e / k) * ld + e % k] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void __launch_bounds__(256) copy_cols_kernel(int N, int k, const double* __restrict__ A, int lda,
                                                        double* __restrict__ B, int ldb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)N * k) return;
  B[(e / k) * ldb + e % k] = A[(e / k) * lda + e % k];
}

__global__ void __launch_bounds__(256) scale_sym_kernel(int m, const double* __restrict__ G, int ldg,
                                                        double* __restrict__ Gs, int lds, double* __restrict__ d) {
  __shared__ double dv[kMaxSmall];
  for (int i = threadIdx.x; i < m; i += 256) {
    const double g = G[i * ldg + i];
    dv[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
    d[i] = dv[i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const int i = e / m, j = e % m;
    Gs[i * lds + j] = 0.5 * (G[i * ldg + j] + G[j * ldg + i]) * dv[i] * dv[j];
  }
}

constexpr int kCholThreads = 1024;   // 8 row groups x 128 columns
constexpr int kCholCols = 128;
static_assert(kMaxSmall <= kCholCols, "one column per lane of a row group");

// S-orthonormalisation by Cholesky-QR with deflation, one workgroup.  Gs is
// the scaled Gram matrix D G D (unit diagonal) of the basis columns in the
// order [X W P].  Gaussian elimination of [Gs | I] by rows yields the unit
// lower triangular L^-1 =: E and the pivots p_j (Schur complements: the
// squared S-distance of scaled column j from the span of the kept columns
// before it), with E Gs E^T = diag(p).  A column whose pivot is at most
// `drop` is not used to eliminate and gets no output column, so the kept
// set K satisfies E_KK Gs_KK E_KK^T = diag(p_K).  Output: the kk kept columns
// of T = D E^T diag(p)^-1/2 (m x kk, upper triangular in the kept indices;
// T^T G T = I), and kk in *kk_out (as a double).
//
// E and the eliminated Gs share one m x m array in LDS: before step j, row
// i > j holds E[i][c] in slots c < j and the partially eliminated Gs in
// slots c >= j.  Step j reads row j and a snapshot of column j (written by
// the previous step into a double-buffered vector), so one barrier per step.
__global__ void __launch_bounds__(kCholThreads) cholqr_t_kernel(int m, const double* __restrict__ Gs, int ldg,
                                                                const double* __restrict__ d, double drop,
                                                                double* __restrict__ T, int ldt,
                                                                double* __restrict__ kk_out) {
  extern __shared__ double a[];   // m x m, row stride m
  __shared__ double colv[2][kMaxSmall], rs[kMaxSmall];
  __shared__ int src[kMaxSmall];
  __shared__ int nkeep;
  const int tid = threadIdx.x, c = tid % kCholCols, rg = tid / kCholCols;
  constexpr int kRG = kCholThreads / kCholCols;
  for (int e = tid; e < m * m; e += kCholThreads) {
    const int i = e / m, k = e - i * m;
    a[e] = Gs[i * ldg + k];
    if (k == 0) colv[0][i] = a[e];
  }
  __syncthreads();
  for (int j = 0; j + 1 < m; ++j) {
    const double* cj = colv[j & 1];
    double* cn = colv[(j + 1) & 1];
    const double p = cj[j];
    const double rp = p > drop ? 1.0 / p : 0.0;   // dropped: f = 0 leaves the rows as they are
    if (c < m) {
      const double rj = a[j * m + c];
      for (int i = j + 1 + rg; i < m; i += kRG) {
        const double f = cj[i] * rp;
        // c < j: E[i][c] -= f E[j][c]; c == j: E[i][j] = -f (E[j][j] = 1); c > j: Schur update
        const double v = c == j ? -f : a[i * m + c] - f * rj;
        a[i * m + c] = v;
        if (c == j + 1) cn[i] = v;
      }
    }
    __syncthreads();
  }
  // slot (j, j) holds p_j, slots (j, c < j) hold E[j][c]
  if (tid == 0) {
    int k = 0;
    for (int j = 0; j < m; ++j) {
      const double p = a[j * m + j];
      if (p > drop) {
        rs[k] = 1.0 / sqrt(p);
        src[k++] = j;
      }
    }
    nkeep = k;
    *kk_out = (double)k;
  }
  __syncthreads();
  const int kk = nkeep;
  for (int e = tid; e < m * kk; e += kCholThreads) {
    const int r = e / kk, k = e - r * kk, j = src[k];
    const double ejr = r < j ? a[j * m + r] : (r == j ? 1.0 : 0.0);
    T[r * ldt + k] = d[r] * ejr * rs[k];
  }
}

__global__ void __launch_bounds__(256) symmetrize_kernel(int m, double* __restrict__ G, int ldg) {
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const int i = e / m, j = e % m;
    if (i < j) {
      const double s = 0.5 * (G[i * ldg + j] + G[j * ldg + i]);
      G[i * ldg + j] = s;
      G[j * ldg + i] = s;
    }
  }
}

// Round-robin pair i of round s among Me indices (Me even; 0 <= s, i < Me - 1).
__device__ __forceinline__ void rr_pair(int i, int s, int Me, int& p, int& q) {
  const int m = Me - 1;
  if (i == 0) {
    p = 0;
    q = 1 + s;
  } else {
    int a = s + i, b = s - i + m;   // both in (0, 2m)
    if (a >= m) a -= m;
    if (b >= m) b -= m;
    p = 1 + a;
    q = 1 + b;
  }
}

constexpr int kSyevThreads = 1024;

// Real symmetric eigensolver, one workgroup: cyclic Jacobi in the parallel
// round-robin order (size padded to even Me with a decoupled zero index).
// Everything lives in LDS: A as its packed upper triangle (the rotations keep
// it symmetric, so each unordered 2 x 2 block pair is rotated once) and V
// transposed (column c of V contiguous).  Rotations are computed by one
// thread per pair; blocks (bi <= bj) of A and rows of the pairs' V columns
// are spread over the threads.  Stops when the off-diagonal Frobenius norm
// is below 4 Me eps of the norm of A.  Output: eigenvalues ascending in w,
// eigenvector j in column j of Vout.
__device__ __forceinline__ int tri_index(int r, int c, int Me) {
  if (r > c) { const int x = r; r = c; c = x; }
  return r * Me - (r * (r - 1)) / 2 + (c - r);
}

__global__ void __launch_bounds__(kSyevThreads) syev_kernel(int m, const double* __restrict__ Ain, int lda,
                                                            double* __restrict__ w, double* __restrict__ Vout,
                                                            int ldv) {
  extern __shared__ double lds[];
  __shared__ double cs[kMaxSmall / 2], sn[kMaxSmall / 2], dn[kMaxSmall], red[kSyevThreads / 64];
  __shared__ int rank[kMaxSmall];
  __shared__ int done;
  const int Me = m + (m & 1), H = Me / 2;
  double* A = lds;                         // packed upper triangle, Me (Me + 1) / 2
  double* V = lds + Me * (Me + 1) / 2;     // transposed: V[c * Me + r] is entry (r, c)
  const int tid = threadIdx.x;
  const int ntri = Me * (Me + 1) / 2, nblk = H * (H + 1) / 2;
  for (int e = tid; e < Me * Me; e += kSyevThreads) {
    const int r = e / Me, c = e % Me;
    if (r <= c) A[tri_index(r, c, Me)] = (r < m && c < m) ? 0.5 * (Ain[r * lda + c] + Ain[c * lda + r]) : 0.0;
    V[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  auto block_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kSyevThreads / 64; ++q) s += red[q];
    __syncthreads();
    return s;
  };
  // norms: diagonal once, off-diagonal twice; row r of the packed triangle
  // starts at r Me - r (r - 1) / 2
  auto row_of = [&](int e) {
    int r = (int)((2.0 * Me + 1.0 - sqrt((2.0 * Me + 1.0) * (2.0 * Me + 1.0) - 8.0 * e)) * 0.5);
    while (r > 0 && r * Me - (r * (r - 1)) / 2 > e) --r;
    while ((r + 1) * Me - ((r + 1) * r) / 2 <= e) ++r;
    return r;
  };
  double nl = 0.0;
  for (int e = tid; e < ntri; e += kSyevThreads) {
    const int r = row_of(e), c = r + (e - (r * Me - (r * (r - 1)) / 2));
    nl += (r == c ? 1.0 : 2.0) * A[e] * A[e];
  }
  const double nrm2 = block_sum(nl);
  const double tol = 4.0 * Me * 1.1102230246251565e-16;
  // this thread's blocks (bi <= bj) and eigenvector items (pair, row): fixed
  // for every round
  constexpr int kMaxBlk = (kMaxSmall / 2) * (kMaxSmall / 2 + 1) / 2 / kSyevThreads + 1;
  constexpr int kMaxItem = (kMaxSmall / 2) * kMaxSmall / kSyevThreads + 1;
  int blk_i[kMaxBlk], blk_j[kMaxBlk], item_i[kMaxItem], item_r[kMaxItem];
#pragma unroll
  for (int k = 0; k < kMaxBlk; ++k) {
    const int bb = tid + k * kSyevThreads;
    blk_i[k] = -1;
    blk_j[k] = -1;
    if (bb < nblk) {
      int bi = (int)((2.0 * H + 1.0 - sqrt((2.0 * H + 1.0) * (2.0 * H + 1.0) - 8.0 * bb)) * 0.5);
      while (bi > 0 && bi * H - (bi * (bi - 1)) / 2 > bb) --bi;
      while ((bi + 1) * H - ((bi + 1) * bi) / 2 <= bb) ++bi;
      blk_i[k] = bi;
      blk_j[k] = bi + (bb - (bi * H - (bi * (bi - 1)) / 2));
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxItem; ++k) {
    const int it = tid + k * kSyevThreads;
    item_i[k] = it < H * Me ? it / Me : -1;
    item_r[k] = it < H * Me ? it - (it / Me) * Me : 0;
  }
  for (int sw = 0; sw < 60; ++sw) {
    double ol = 0.0;
    for (int e = tid; e < ntri; e += kSyevThreads) {
      const int r = row_of(e), c = r + (e - (r * Me - (r * (r - 1)) / 2));
      if (r != c) ol += 2.0 * A[e] * A[e];
    }
    const double off = block_sum(ol);
    if (tid == 0) done = off <= tol * tol * nrm2;
    __syncthreads();
    if (done) break;
    for (int s = 0; s < Me - 1; ++s) {
      for (int i = tid; i < H; i += kSyevThreads) {
        int p, q;
        rr_pair(i, s, Me, p, q);
        const double app = A[tri_index(p, p, Me)], aqq = A[tri_index(q, q, Me)], b = A[tri_index(p, q, Me)];
        const double ab = fabs(b), d = aqq - app;
        double c = 1.0, sv = 0.0, dp = app, dq = aqq;
        if (b * b < 1e-8 * d * d) {
          // small angle: t = (b / d)(1 - x + 2 x^2), x = b^2 / d^2; one division
          const double id = 1.0 / d, x = b * b * id * id;
          const double f = 1.0 - x + 2.0 * x * x, t2 = x * f * f;
          c = 1.0 - 0.5 * t2 + 0.375 * t2 * t2;
          sv = b * id * f * c;
          dp = app - b * b * id * f;
          dq = aqq + b * b * id * f;
        } else if (ab > 0.0) {
          const double tau = (aqq - app) / (2.0 * ab);
          const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sv = (b >= 0.0 ? 1.0 : -1.0) * t * c;
          dp = app - t * ab;
          dq = aqq + t * ab;
        }
        cs[i] = c;
        sn[i] = sv;
        dn[p] = dp;
        dn[q] = dq;
      }
      __syncthreads();
      // A <- J^T A J on the blocks bi <= bj of the pairs
#pragma unroll
      for (int k = 0; k < kMaxBlk; ++k) {
        const int bi = blk_i[k], bj = blk_j[k];
        if (bi < 0) continue;
        int pi, qi, pj, qj;
        rr_pair(bi, s, Me, pi, qi);
        rr_pair(bj, s, Me, pj, qj);
        if (bi == bj) {
          A[tri_index(pi, pi, Me)] = dn[pi];
          A[tri_index(qi, qi, Me)] = dn[qi];
          A[tri_index(pi, qi, Me)] = 0.0;
        } else {
          const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
          const int i00 = tri_index(pi, pj, Me), i01 = tri_index(pi, qj, Me);
          const int i10 = tri_index(qi, pj, Me), i11 = tri_index(qi, qj, Me);
          const double b00 = A[i00], b01 = A[i01], b10 = A[i10], b11 = A[i11];
          const double t00 = b00 * cj - b01 * sj, t01 = b00 * sj + b01 * cj;
          const double t10 = b10 * cj - b11 * sj, t11 = b10 * sj + b11 * cj;
          A[i00] = ci * t00 - si * t10;
          A[i01] = ci * t01 - si * t11;
          A[i10] = si * t00 + ci * t10;
          A[i11] = si * t01 + ci * t11;
        }
      }
      // V <- V J: columns p, q of every pair, one row per thread
#pragma unroll
      for (int k = 0; k < kMaxItem; ++k) {
        const int i = item_i[k], r = item_r[k];
        if (i < 0) continue;
        int p, q;
        rr_pair(i, s, Me, p, q);
        const double c = cs[i], sv = sn[i];
        const double vp = V[p * Me + r], vq = V[q * Me + r];
        V[p * Me + r] = vp * c - vq * sv;
        V[q * Me + r] = vp * sv + vq * c;
      }
      __syncthreads();
    }
  }
  // ascending ranks among the m real indices (ties by index)
  for (int i = tid; i < m; i += kSyevThreads) {
    const double li = A[tri_index(i, i, Me)];
    int k = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = A[tri_index(j, j, Me)];
      k += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
    rank[i] = k;
  }
  __syncthreads();
  for (int i = tid; i < m; i += kSyevThreads) w[rank[i]] = A[tri_index(i, i, Me)];
  for (int e = tid; e < m * m; e += kSyevThreads) {
    const int r = e / m, c = e % m;
    Vout[r * ldv + rank[c]] = V[c * Me + r];
  }
}

}  // namespace

hipError_t dense_gram(int N, int k1, int k2, const double* A, int lda, const double* B, int ldb, double* part,
                      int nchunk, double* G, int ldg, hipStream_t s) {
  const int chunk = (N + nchunk - 1) / nchunk;
  const dim3 grid(nchunk, (k1 + kGT - 1) / kGT, (k2 + kGT - 1) / kGT);
  hipLaunchKernelGGL(gram_part_kernel, grid, dim3(256), 0, s, N, k1, k2, chunk, A, lda, B, ldb, part);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((k1 * k2 + 255) / 256), dim3(256), 0, s, k1, k2, nchunk, part, G,
                     ldg);
  return hipGetLastError();
}

hipError_t dense_combine(int N, int k1, int k2, const double* A, int lda, const double* T, int ldt, double beta,
                         const double* Z, int ldz, double* Y, int ldy, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3((N + kCRows - 1) / kCRows), dim3(256), 0, s, N, k1, k2, A, lda, T, ldt,
                     beta, Z, ldz, Y, ldy);
  return hipGetLastError();
}

hipError_t dense_syev_w(int m, const double* A, int lda, double* w, double* V, int ldv, double* work,
                        hipStream_t s) {
  (void)work;
  if (m < 1 || m > kMaxSmall) return hipErrorInvalidValue;
  const int Me = m + (m & 1);
  const size_t lds = sizeof(double) * ((size_t)Me * (Me + 1) / 2 + (size_t)Me * Me);
  (void)hipFuncSetAttribute((const void*)syev_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(syev_kernel, dim3(1), dim3(kSyevThreads), lds, s, m, A, lda, w, V, ldv);
  return hipGetLastError();
}

hipError_t dense_residual(int N, int k, const double* HX, const double* SX, int ld, const double* theta, double* R,
                          int ldr, double* part, int nchunk, double* norms, hipStream_t s) {
  const int chunk = (N + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(residual_kernel, dim3(nchunk), dim3(256), 0, s, N, k, chunk, HX, SX, ld, theta, R, ldr, part);
  hipLaunchKernelGGL(norms_kernel, dim3((k + 255) / 256), dim3(256), 0, s, k, nchunk, part, norms);
  return hipGetLastError();
}

hipError_t dense_random(int N, int k, uint64_t seed, double* X, int ld, hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  hipLaunchKernelGGL(random_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, k, seed, X, ld);
  return hipGetLastError();
}

hipError_t dense_copy_cols(int N, int k, const double* A, int lda, double* B, int ldb, hipStream_t s) {
  const int64_t n = (int64_t)N * k;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, k, A, lda, B, ldb);
  return hipGetLastError();
}

hipError_t dense_scale_sym(int m, const double* G, int ldg, double* Gs, int lds, double* dvec, hipStream_t s) {
  hipLaunchKernelGGL(scale_sym_kernel, dim3(1), dim3(256), 0, s, m, G, ldg, Gs, lds, dvec);
  return hipGetLastError();
}

hipError_t dense_cholqr_t(int m, const double* Gs, int ldg, const double* dvec, double drop, double* T, int ldt,
                          double* kk_out, hipStream_t s) {
  if (m < 1 || m > kMaxSmall) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (size_t)m * m;
  (void)hipFuncSetAttribute((const void*)cholqr_t_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(cholqr_t_kernel, dim3(1), dim3(kCholThreads), lds, s, m, Gs, ldg, dvec, drop, T, ldt, kk_out);
  return hipGetLastError();
}

hipError_t dense_symmetrize(int m, double* G, int ldg, hipStream_t s) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(1), dim3(256), 0, s, m, G, ldg);
  return hipGetLastError();
}

}  // namespace lhf
