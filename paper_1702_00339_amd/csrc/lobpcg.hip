// Dense FP64 kernels of the block LOBPCG driver: Gram products of tall
// blocks, block combinations, residuals and Cholesky-QR orthonormalisation
// (the Rayleigh-Ritz eigensolver is in rrsyev.hip).
//
// Blocks of vectors are row-major [N][ld] (column j = vector j).  Reductions
// over N are split into fixed chunks whose partial results are added in chunk
// order, so every result is deterministic.
#include <algorithm>
#include <type_traits>

#include "toeplitz.h"

namespace lhf {
namespace {

constexpr int kGT = 56;      // Gram output tile (rows and columns)
constexpr int kGM = 4;       // outputs per thread along each side
constexpr int kGL = kGT / kGM;   // 14 x 14 threads own a tile
constexpr int kGRows = 32;   // rows staged per step

// part[c][i][j] = sum over rows n of chunk c of A[n][i] B[n][j] on one output
// tile; thread (ti, tj) owns rows ti + 14 u and columns tj + 14 v of the tile
// (consecutive lanes read consecutive staged entries)
__global__ void __launch_bounds__(256) gram_part_kernel(int N, int k1, int k2, int chunk, const double* __restrict__ A,
                                                        int lda, const double* __restrict__ B, int ldb,
                                                        double* __restrict__ part) {
  __shared__ double As[kGRows][kGT];
  __shared__ double Bs[kGRows][kGT];
  const int c = blockIdx.x, i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  const int t = threadIdx.x, ti = t / kGL, tj = t % kGL;
  const bool act = t < kGL * kGL;
  double acc[kGM][kGM];
#pragma unroll
  for (int u = 0; u < kGM; ++u)
#pragma unroll
    for (int v = 0; v < kGM; ++v) acc[u][v] = 0.0;
  const int n0 = c * chunk, n1 = min(N, n0 + chunk);
  // the next rows are fetched into registers while the current ones are used
  constexpr int kS = (kGRows * kGT + 255) / 256;
  double ra[kS], rb[kS];
  auto fetch = [&](int nb) {
#pragma unroll
    for (int u = 0; u < kS; ++u) {
      const int e = t + 256 * u, r = e / kGT, q = e % kGT, n = nb + r;
      const bool in = e < kGRows * kGT && n < n1;
      ra[u] = (in && i0 + q < k1) ? A[(int64_t)n * lda + i0 + q] : 0.0;
      rb[u] = (in && j0 + q < k2) ? B[(int64_t)n * ldb + j0 + q] : 0.0;
    }
  };
  if (n0 < n1) fetch(n0);
  for (int nb = n0; nb < n1; nb += kGRows) {
#pragma unroll
    for (int u = 0; u < kS; ++u) {
      const int e = t + 256 * u;
      if (e < kGRows * kGT) {
        As[e / kGT][e % kGT] = ra[u];
        Bs[e / kGT][e % kGT] = rb[u];
      }
    }
    __syncthreads();
    if (nb + kGRows < n1) fetch(nb + kGRows);
    if (act) {
      for (int r = 0; r < kGRows; ++r) {
        double av[kGM], bv[kGM];
#pragma unroll
        for (int u = 0; u < kGM; ++u) {
          av[u] = As[r][ti + kGL * u];
          bv[u] = Bs[r][tj + kGL * u];
        }
#pragma unroll
        for (int u = 0; u < kGM; ++u)
#pragma unroll
          for (int v = 0; v < kGM; ++v) acc[u][v] += av[u] * bv[v];
      }
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int u = 0; u < kGM; ++u)
#pragma unroll
      for (int v = 0; v < kGM; ++v) {
        const int i = i0 + ti + kGL * u, j = j0 + tj + kGL * v;
        if (i < k1 && j < k2) part[((int64_t)c * k1 + i) * k2 + j] = acc[u][v];
      }
  }
}

__global__ void __launch_bounds__(256) gram_reduce_kernel(int k1, int k2, int nchunk, const double* __restrict__ part,
                                                          double* __restrict__ G, int ldg) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= k1 * k2) return;
  // chunk order kept; loads of 8 chunks in flight together
  constexpr int kU = 8;
  const int64_t st = (int64_t)k1 * k2;
  double s = 0.0;
  int c = 0;
  for (; c + kU <= nchunk; c += kU) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = part[(c + u) * st + e];
#pragma unroll
    for (int u = 0; u < kU; ++u) s += v[u];
  }
  for (; c < nchunk; ++c) s += part[c * st + e];
  G[(e / k2) * ldg + e % k2] = s;
}

constexpr int kCbR = 32;                              // rows per combine workgroup
constexpr int kCbK = 16;                              // inner-dimension chunk staged per step
constexpr int kCbC = 8;                               // columns per thread
constexpr int kCbG = (kMaxSmall + kCbC - 1) / kCbC;   // 14 column groups
static_assert(kCbC == 8, "the combine kernel's column-slot dispatch covers 1 .. 8");

// Y_a = beta Z + A_a T for a = blockIdx.y (beta only with one product).  A
// workgroup owns kCbR rows; thread (rg, cg) owns rows 2 rg, 2 rg + 1 and
// columns cg + 14 c, c < 8 (consecutive lanes read consecutive staged T).
__global__ void __launch_bounds__(256) combine_kernel(int N, int k1, int k2, const double* __restrict__ A0,
                                                      const double* __restrict__ A1, const double* __restrict__ A2,
                                                      int lda, const double* __restrict__ T, int ldt, double beta,
                                                      const double* Z, int ldz, double* Y0, double* Y1, double* Y2,
                                                      int ldy) {
  __shared__ double As[kCbR][kCbK + 1];
  __shared__ double Ts[kCbK][kCbG * kCbC];
  const double* A = blockIdx.y == 0 ? A0 : (blockIdx.y == 1 ? A1 : A2);
  double* Y = blockIdx.y == 0 ? Y0 : (blockIdx.y == 1 ? Y1 : Y2);
  const int r0 = blockIdx.x * kCbR, t = threadIdx.x;
  const int rg = t / kCbG, cg = t % kCbG;
  const bool act = rg < kCbR / 2;
  const int ncu = (k2 + kCbG - 1) / kCbG;   // column slots in use (uniform)
  double acc[2][kCbC];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int c = 0; c < kCbC; ++c) acc[u][c] = 0.0;
  // the next chunk is fetched into registers while the current one is used
  constexpr int kSA = (kCbR * kCbK + 255) / 256, kST = (kCbK * kCbG * kCbC + 255) / 256;
  double ra[kSA], rt[kST];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int u = 0; u < kSA; ++u) {
      const int e = t + 256 * u, r = e / kCbK, kk = e % kCbK;
      ra[u] = (e < kCbR * kCbK && r0 + r < N && kc + kk < k1) ? A[(int64_t)(r0 + r) * lda + kc + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kST; ++u) {
      const int e = t + 256 * u, kk = e / (kCbG * kCbC), j = e % (kCbG * kCbC);
      rt[u] = (e < kCbK * kCbG * kCbC && kc + kk < k1 && j < k2) ? T[(int64_t)(kc + kk) * ldt + j] : 0.0;
    }
  };
  fetch(0);
  for (int kc = 0; kc < k1; kc += kCbK) {
#pragma unroll
    for (int u = 0; u < kSA; ++u) {
      const int e = t + 256 * u;
      if (e < kCbR * kCbK) As[e / kCbK][e % kCbK] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < kST; ++u) {
      const int e = t + 256 * u;
      if (e < kCbK * kCbG * kCbC) Ts[e / (kCbG * kCbC)][e % (kCbG * kCbC)] = rt[u];
    }
    __syncthreads();
    if (kc + kCbK < k1) fetch(kc + kCbK);
    if (act) {
      // only the column slots c < ncu reach a column j = cg + kCbG c < k2
      // (the others would multiply staged zeros), unrolled per count
      auto sums = [&](auto ncc) {
        constexpr int NC = decltype(ncc)::value;
#pragma unroll 4
        for (int kk = 0; kk < kCbK; ++kk) {
          const double a0 = As[2 * rg][kk], a1 = As[2 * rg + 1][kk];
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double tv = Ts[kk][cg + kCbG * c];
            acc[0][c] += a0 * tv;
            acc[1][c] += a1 * tv;
          }
        }
      };
      switch (ncu) {
        case 1: sums(std::integral_constant<int, 1>{}); break;
        case 2: sums(std::integral_constant<int, 2>{}); break;
        case 3: sums(std::integral_constant<int, 3>{}); break;
        case 4: sums(std::integral_constant<int, 4>{}); break;
        case 5: sums(std::integral_constant<int, 5>{}); break;
        case 6: sums(std::integral_constant<int, 6>{}); break;
        case 7: sums(std::integral_constant<int, 7>{}); break;
        default: sums(std::integral_constant<int, kCbC>{}); break;
      }
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int n = r0 + 2 * rg + u;
      if (n >= N) continue;
#pragma unroll
      for (int c = 0; c < kCbC; ++c) {
        const int j = cg + kCbG * c;
        if (j < k2) Y[(int64_t)n * ldy + j] = beta != 0.0 ? acc[u][c] + beta * Z[(int64_t)n * ldz + j] : acc[u][c];
      }
    }
  }
}

// R = HX - SX diag(theta); part[c][j] = sum over chunk rows of R^2.  The
// blocks are row-major, so consecutive threads take consecutive columns of a
// tile of up to 256 (coalesced) and 256 / kc row lanes walk the chunk's rows;
// the lanes' sums of a column are added in lane order.
__global__ void __launch_bounds__(256) residual_kernel(int N, int k, int chunk, const double* __restrict__ HX,
                                                       const double* __restrict__ SX, int ld,
                                                       const double* __restrict__ theta, double* __restrict__ R,
                                                       int ldr, double* __restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const int n0 = c * chunk, n1 = min(N, n0 + chunk);
  for (int j0 = 0; j0 < k; j0 += 256) {
    const int kc = min(256, k - j0), nr = 256 / kc;
    const int jl = threadIdx.x % kc, rl = threadIdx.x / kc, j = j0 + jl;
    double s = 0.0;
    if (rl < nr) {
      const double th = theta[j];
      for (int n = n0 + rl; n < n1; n += nr) {
        const double r = HX[(int64_t)n * ld + j] - SX[(int64_t)n * ld + j] * th;
        R[(int64_t)n * ldr + j] = r;
        s += r * r;
      }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < kc) {
      double t = 0.0;
      for (int q = 0; q < nr; ++q) t += red[q * kc + threadIdx.x];
      part[(int64_t)c * k + j0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// norms[j] = sqrt(sum over chunks of part[c][j]): one workgroup per column,
// the chunks strided over its threads, then a tree in LDS (fixed order)
__global__ void __launch_bounds__(256) norms_kernel(int k, int nchunk, const double* __restrict__ part,
                                                    double* __restrict__ norms) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) s += part[(int64_t)c * k + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[j] = sqrt(red[0]);
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

constexpr int kCholThreads = 1024;
constexpr int kCholCols = 128;                                 // column slots (> m: the rest stay zero)
constexpr int kCholRG = kCholThreads / kCholCols;              // row groups
constexpr int kCholW = (kMaxSmall + kCholRG - 1) / kCholRG;    // rows per thread
static_assert(kCholCols >= kMaxSmall && kCholW * kCholRG >= kMaxSmall, "one slot per column and row");
static_assert(kCholW == 14, "the dispatch below names every block count");

// 1 / x for a normal x to within a few ulps: the hardware estimate refined by
// two Newton steps.
__device__ __forceinline__ double chol_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

template <int N>
using CholIC = std::integral_constant<int, N>;
// F(CholIC<J>{}) for a block count 1 <= J <= kCholW known only at run time
#define CHOL_DISPATCH(J, F)                                                                                   \
  switch (J) {                                                                                                \
    case 1: F(CholIC<1>{}); break;   case 2: F(CholIC<2>{}); break;   case 3: F(CholIC<3>{}); break;          \
    case 4: F(CholIC<4>{}); break;   case 5: F(CholIC<5>{}); break;   case 6: F(CholIC<6>{}); break;          \
    case 7: F(CholIC<7>{}); break;   case 8: F(CholIC<8>{}); break;   case 9: F(CholIC<9>{}); break;          \
    case 10: F(CholIC<10>{}); break; case 11: F(CholIC<11>{}); break; case 12: F(CholIC<12>{}); break;        \
    case 13: F(CholIC<13>{}); break; case 14: F(CholIC<14>{}); break; default: break;                         \
  }

// S-orthonormalisation by Cholesky-QR with deflation, one workgroup.  The
// Gram matrix G of the basis columns in the order [X W P] is scaled on load,
// Gs = D (G + G^T) / 2 D with D = diag(G)^-1/2 (unit diagonal).  Gaussian
// elimination of [Gs | I] by rows yields the unit lower triangular L^-1 =: E
// and the pivots p_j (Schur complements: the squared S-distance of scaled
// column j from the span of the kept columns before it), with
// E Gs E^T = diag(p).  A column whose pivot is at most `drop` is not used to
// eliminate and gets no output column, so the kept set K satisfies
// E_KK Gs_KK E_KK^T = diag(p_K).  Output: the kk kept columns of
// T = D E^T diag(p)^-1/2 (m x kk, upper triangular in the kept indices;
// T^T G T = I), and kk in *kk_out (as a double).
//
// E and the eliminated Gs share one m x m array, in registers: lane c of row
// group g holds column c at the rows of reversed index idx = m - 1 - i =
// g + kCholRG k; before step j, row i > j holds E[i][c] in columns c < j and
// the partially eliminated Gs in columns c >= j.  Step j reads row j and
// column j (zero at the rows up to j) from double-buffered LDS vectors, updates
// its rows after j (the first J = ceil((m - 1 - j) / kCholRG) of its register
// rows: the steps run in phases of equal J compiled for that J) and publishes
// row and column j + 1; one barrier per step.
__global__ void __launch_bounds__(kCholThreads) cholqr_kernel(int m, const double* __restrict__ G, int ldg,
                                                              double drop, double* __restrict__ T, int ldt,
                                                              double* __restrict__ kk_out) {
  __shared__ double rowb[2][kCholCols], colb[2][kCholCols], dsc[kCholCols], rs[kCholCols];
  __shared__ int kidx[kCholCols];
  const int tid = threadIdx.x, c = tid % kCholCols, g = tid / kCholCols;
  for (int i = tid; i < kCholCols; i += kCholThreads) {
    const double gi = i < m ? G[(int64_t)i * ldg + i] : 0.0;
    dsc[i] = gi > 0.0 ? 1.0 / sqrt(gi) : 0.0;
  }
  __syncthreads();
  double a[kCholW];
#pragma unroll
  for (int k = 0; k < kCholW; ++k) {
    const int idx = g + kCholRG * k, r = m - 1 - idx;
    a[k] = (c < m && idx < m) ? 0.5 * (G[(int64_t)r * ldg + c] + G[(int64_t)c * ldg + r]) * dsc[r] * dsc[c] : 0.0;
  }
  // row 0 (reversed index m - 1) and column 0 below the diagonal
#pragma unroll
  for (int k = 0; k < kCholW; ++k) {
    const int idx = g + kCholRG * k;
    if (idx == m - 1) rowb[0][c] = a[k];
    if (c == 0) colb[0][idx] = idx < m - 1 ? a[k] : 0.0;
  }
  __syncthreads();
  auto steps = [&](auto Jc, int jb, int je) {
    constexpr int J = decltype(Jc)::value;
#pragma unroll 1
    for (int j = jb; j < je; ++j) {
      const int bs = j & 1, na = m - 1 - j;   // rows after j: reversed indices below na
      const double p = rowb[bs][j];
      const double rp = p > drop ? chol_recip(p) : 0.0;   // dropped: zero multipliers
      const double rj = rowb[bs][c];
      double f[J];
#pragma unroll
      for (int k = 0; k < J; ++k) f[k] = colb[bs][g + kCholRG * k] * rp;
      // register row k of this lane has reversed index g + kCholRG k: it lies
      // after row j for k < ka, and after row j + 1 for k < k1; row j + 1
      // (reversed index na - 1, in the last of the J blocks) is register row
      // J - 1 of row group gr
      const int ka = (na - g + kCholRG - 1) / kCholRG, r1 = na - 1;
      const int k1 = (r1 - g + kCholRG - 1) / kCholRG, gr = r1 % kCholRG;
      // E[i][c] -= f E[j][c] (c < j) or the Schur update (c > j) ...
#pragma unroll
      for (int k = 0; k < J; ++k) a[k] = fma(-f[k], rj, a[k]);
      // ... and column j takes the multipliers, E[i][j] = -f_i / p_j (one
      // lane per row group)
      if (c == j) {
#pragma unroll
        for (int k = 0; k < J; ++k)
          if (k < ka) a[k] = -f[k];
      }
      // row j + 1 and column j + 1 below the diagonal into the other buffers
      if (g == gr) rowb[bs ^ 1][c] = a[J - 1];
      if (c == j + 1) {
#pragma unroll
        for (int k = 0; k < J; ++k) colb[bs ^ 1][g + kCholRG * k] = k < k1 ? a[k] : 0.0;
      }
      __syncthreads();
    }
  };
  for (int j0 = 0; j0 < m - 1;) {
    const int J = (m - 1 - j0 + kCholRG - 1) / kCholRG;
    const int je = min(m - 1, m - 1 - kCholRG * (J - 1));   // the first step with fewer blocks
    CHOL_DISPATCH(J, [&](auto Jc) { steps(Jc, j0, je); });
    j0 = je;
  }
  // pivots p_j on the diagonal; kept columns numbered in order (two ballots)
#pragma unroll
  for (int k = 0; k < kCholW; ++k) {
    const int idx = g + kCholRG * k, r = m - 1 - idx;
    if (idx < m && r == c) rs[c] = a[k] > drop ? 1.0 / sqrt(a[k]) : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    const bool k0 = tid < m && rs[tid] > 0.0, k1 = tid + 64 < m && rs[tid + 64] > 0.0;
    const unsigned long long b0 = __ballot(k0), b1 = __ballot(k1);
    const unsigned long long below = (1ull << tid) - 1ull;   // lanes before this one
    kidx[tid] = k0 ? __popcll(b0 & below) : -1;
    kidx[tid + 64] = k1 ? __popcll(b0) + __popcll(b1 & below) : -1;
    if (tid == 0) *kk_out = (double)(__popcll(b0) + __popcll(b1));
  }
  __syncthreads();
  // T[r][kidx[j]] = d_r E[j][r] / sqrt(p_j) for kept j: the thread of column r
  // and row j writes it (E[j][j] = 1, zero above)
  if (c < m) {
#pragma unroll
    for (int k = 0; k < kCholW; ++k) {
      const int idx = g + kCholRG * k, j = m - 1 - idx;
      if (idx < m && kidx[j] >= 0) {
        const double ejr = c < j ? a[k] : (c == j ? 1.0 : 0.0);
        T[(int64_t)c * ldt + kidx[j]] = dsc[c] * ejr * rs[j];
      }
    }
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
  if (k2 > kMaxSmall) return hipErrorInvalidValue;
  hipLaunchKernelGGL(combine_kernel, dim3((N + kCbR - 1) / kCbR, 1), dim3(256), 0, s, N, k1, k2, A, A, A, lda, T, ldt,
                     beta, Z, ldz, Y, Y, Y, ldy);
  return hipGetLastError();
}

hipError_t dense_combine3(int N, int k1, int k2, const double* A0, const double* A1, const double* A2, int lda,
                          const double* T, int ldt, double* Y0, double* Y1, double* Y2, int ldy, hipStream_t s) {
  if (k2 > kMaxSmall) return hipErrorInvalidValue;
  hipLaunchKernelGGL(combine_kernel, dim3((N + kCbR - 1) / kCbR, 3), dim3(256), 0, s, N, k1, k2, A0, A1, A2, lda, T,
                     ldt, 0.0, nullptr, 0, Y0, Y1, Y2, ldy);
  return hipGetLastError();
}

hipError_t dense_residual(int N, int k, const double* HX, const double* SX, int ld, const double* theta, double* R,
                          int ldr, double* part, int nchunk, double* norms, hipStream_t s) {
  const int chunk = (N + nchunk - 1) / nchunk;
  hipLaunchKernelGGL(residual_kernel, dim3(nchunk), dim3(256), 0, s, N, k, chunk, HX, SX, ld, theta, R, ldr, part);
  if (k > 0) hipLaunchKernelGGL(norms_kernel, dim3(k), dim3(256), 0, s, k, nchunk, part, norms);
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

hipError_t dense_cholqr(int m, const double* G, int ldg, double drop, double* T, int ldt, double* kk_out,
                        hipStream_t s) {
  if (m < 1 || m > kMaxSmall) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cholqr_kernel, dim3(1), dim3(kCholThreads), 0, s, m, G, ldg, drop, T, ldt, kk_out);
  return hipGetLastError();
}

}  // namespace lhf
