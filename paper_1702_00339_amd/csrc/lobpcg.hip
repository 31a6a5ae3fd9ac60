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
#pragma unroll 4
      for (int kk = 0; kk < kCbK; ++kk) {
        const double a0 = As[2 * rg][kk], a1 = As[2 * rg + 1][kk];
#pragma unroll
        for (int c = 0; c < kCbC; ++c) {
          const double tv = Ts[kk][cg + kCbG * c];
          acc[0][c] += a0 * tv;
          acc[1][c] += a1 * tv;
        }
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
constexpr int kCholB = 4;           // rows per batch of a thread
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
      // rows in batches of kCholB (loads of a batch in flight together)
      for (int i0 = j + 1 + rg; i0 < m; i0 += kCholB * kRG) {
        // unconditional loads (rows clamped into range) so that they issue together
        double f[kCholB], v[kCholB];
#pragma unroll
        for (int u = 0; u < kCholB; ++u) {
          const int i = min(i0 + u * kRG, m - 1);
          f[u] = cj[i];
          v[u] = a[i * m + c];
        }
#pragma unroll
        for (int u = 0; u < kCholB; ++u) {
          const int i = i0 + u * kRG;
          if (i < m) {
            // c < j: E[i][c] -= f E[j][c]; c == j: E[i][j] = -f (E[j][j] = 1); c > j: Schur update
            const double fu = f[u] * rp;
            const double nv = c == j ? -fu : v[u] - fu * rj;
            a[i * m + c] = nv;
            if (c == j + 1) cn[i] = nv;
          }
        }
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

// Real symmetric eigensolver: cyclic Jacobi in the parallel round-robin
// order (size padded to even Me with a decoupled zero index).
//
// The matrix lives in the LDS of one workgroup in "slot space": the Me
// indices occupy Me storage slots, and the pairs of every round are the
// same slot pairs, (0, 1) and (1 + i, Me - i) for i = 1 .. Me/2 - 1.  After
// each round the contents of slots 2 .. Me-1 move down one slot, slot 1
// moves to slot Me-1 and slot 0 stays (the circle method of the round-robin
// tournament), so after the Me - 1 rounds of a sweep every slot holds its
// own index again.  Storage follows the pairs: the diagonal 2 x 2 block of
// pair i as three arrays (first-first, second-second, first-second), and the
// blocks of pairs bi < bj as four arrays (entry first/second of bi times
// first/second of bj) indexed by the block's rank in the strict upper
// triangle.  A thread owns fixed blocks and reads and writes fixed
// addresses every round: consecutive threads own consecutive blocks of a
// block row, so loads and stores are contiguous, and the loop has no index
// arithmetic.  A round is two phases: the first wave computes the rotations
// of the pairs from their diagonal blocks while the other threads load
// their blocks; after a barrier the rotated blocks are written to the
// shifted slots.  Stops at a sweep boundary once the off-diagonal Frobenius
// norm is below 4 Me eps of the norm of A.
//
// Eigenvectors: the rotations of every round are recorded in global memory,
// and a second kernel replays them on the rows of V = I, one wavefront per
// row (the rows are independent): lane i holds the row's entries in the
// two slots of pair i and the slot shift is a one-lane DPP move.  Output:
// eigenvalues ascending in w, eigenvector j in column j of Vout.
__device__ __forceinline__ int slot_first(int i) { return i == 0 ? 0 : 1 + i; }
__device__ __forceinline__ int slot_second(int i, int Me) { return i == 0 ? 1 : Me - i; }
__device__ __forceinline__ int slot_shift(int x, int Me) { return x == 0 ? 0 : (x == 1 ? Me - 1 : x - 1); }
// pair holding slot x; first = whether x is the pair's first slot
__device__ __forceinline__ int slot_pair(int x, int Me, bool& first) {
  if (x <= 1) {
    first = x == 0;
    return 0;
  }
  first = x <= Me / 2;
  return first ? x - 1 : Me - x;
}
// rank of the block of pairs bi < bj in the strict upper triangle (row-major)
__device__ __forceinline__ int offblk(int bi, int bj, int H) { return bi * H - (bi * (bi + 1)) / 2 + (bj - bi - 1); }
// storage offset of the entry of slots (x, y) (symmetric)
__device__ __forceinline__ int jstore(int x, int y, int Me) {
  const int H = Me / 2, nob = H * (H - 1) / 2;
  bool fx, fy;
  int px = slot_pair(x, Me, fx), py = slot_pair(y, Me, fy);
  if (px == py) return x == y ? (fx ? px : H + px) : 2 * H + px;
  if (px > py) {
    const int t = px; px = py; py = t;
    const bool u = fx; fx = fy; fy = u;
  }
  return 3 * H + ((fx ? 0 : 2) + (fy ? 0 : 1)) * nob + offblk(px, py, H);
}

// Rotation annihilating b = A(p, q): with d = aqq - app, r = sqrt(d^2 + 4 b^2)
// and u = |d| + r, the classical t = sign(d) 2|b| / u gives c = u rho and
// s = sign(d) 2 b rho with rho = (2 r u)^-1/2, and t |b| = 2 b^2 / u =
// 4 b^2 r rho^2 (no division; no cancellation for small or large angles).
// dp, dq: the rotated diagonal entries.
__device__ __forceinline__ void jacobi_rot(double app, double aqq, double b, double& c, double& s, double& dp,
                                           double& dq) {
  c = 1.0;
  s = 0.0;
  dp = app;
  dq = aqq;
  if (b != 0.0) {
    const double d = aqq - app, sd = d >= 0.0 ? 1.0 : -1.0;
    const double r = sqrt(d * d + 4.0 * b * b), u = fabs(d) + r, rho = rsqrt(2.0 * r * u);
    c = u * rho;
    s = sd * 2.0 * b * rho;
    const double del = 4.0 * b * b * r * rho * rho;
    dp = app - sd * del;
    dq = aqq + sd * del;
  }
}

constexpr int kSyevThreads = 1024;

__global__ void __launch_bounds__(kSyevThreads) syev_kernel(int m, const double* __restrict__ Ain, int lda,
                                                            double* __restrict__ w, double2* __restrict__ rec,
                                                            int* __restrict__ hdr) {
  extern __shared__ double lds[];
  __shared__ double rc[kMaxSmall / 2], rs[kMaxSmall / 2];   // this round's rotations
  __shared__ double red[kSyevThreads / 64];
  __shared__ int rank[kMaxSmall];
  __shared__ int done;
  const int Me = m + (m & 1), H = Me / 2, Mc = Me - 1, nob = H * (H - 1) / 2;
  double* A = lds;   // pair-block storage over slots, Me (Me + 1) / 2
  const int tid = threadIdx.x;
  for (int e = tid; e < Me * Me; e += kSyevThreads) {
    const int r = e / Me, c = e % Me;
    if (r <= c) A[jstore(r, c, Me)] = (r < m && c < m) ? 0.5 * (Ain[r * lda + c] + Ain[c * lda + r]) : 0.0;
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
  // the pair this thread rotates (first wave) and its diagonal block's
  // shifted write addresses (first-first, second-second, first-second)
  const bool rotor = tid < H;
  int dw[3] = {0, 0, 0};
  if (rotor) {
    const int f = slot_shift(slot_first(tid), Me), sc = slot_shift(slot_second(tid, Me), Me);
    dw[0] = jstore(f, f, Me);
    dw[1] = jstore(sc, sc, Me);
    dw[2] = jstore(f, sc, Me);
  }
  // this thread's off-diagonal blocks (bi < bj, fixed): entry q = first/second
  // of bi (q >> 1) times first/second of bj (q & 1) at 3H + q nob + rank,
  // written to the storage of the shifted slots
  constexpr int kMaxBlk = (kMaxSmall / 2) * (kMaxSmall / 2 - 1) / 2 / kSyevThreads + 1;
  int bpi[kMaxBlk], bpj[kMaxBlk], rda[kMaxBlk], wra[kMaxBlk][4];
#pragma unroll
  for (int k = 0; k < kMaxBlk; ++k) {
    const int ob = tid + k * kSyevThreads;
    bpi[k] = -1;
    bpj[k] = -1;
    rda[k] = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) wra[k][q] = 0;
    if (ob < nob) {
      const double hb = H - 0.5;
      int bi = (int)(hb - sqrt(hb * hb - 2.0 * ob));
      if (bi < 0) bi = 0;
      while (bi > 0 && offblk(bi, bi + 1, H) > ob) --bi;
      while (bi + 1 < H && offblk(bi + 1, bi + 2, H) <= ob) ++bi;
      const int bj = ob - offblk(bi, bi + 1, H) + bi + 1;
      bpi[k] = bi;
      bpj[k] = bj;
      rda[k] = 3 * H + ob;
      const int xs[2] = {slot_shift(slot_first(bi), Me), slot_shift(slot_second(bi, Me), Me)};
      const int ys[2] = {slot_shift(slot_first(bj), Me), slot_shift(slot_second(bj, Me), Me)};
#pragma unroll
      for (int q = 0; q < 4; ++q) wra[k][q] = jstore(xs[q >> 1], ys[q & 1], Me);
    }
  }
  // squared norms over this thread's blocks: diagonal once, off-diagonal twice
  auto block_norms = [&](double& dg, double& od) {
    dg = 0.0;
    od = 0.0;
    if (rotor) {
      const double a0 = A[tid], a1 = A[H + tid], a2 = A[2 * H + tid];
      dg = a0 * a0 + a1 * a1;
      od = 2.0 * a2 * a2;
    }
#pragma unroll
    for (int k = 0; k < kMaxBlk; ++k) {
      if (bpi[k] < 0) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) od += 2.0 * A[rda[k] + q * nob] * A[rda[k] + q * nob];
    }
  };
  double dg0, od0;
  block_norms(dg0, od0);
  const double nrm2 = block_sum(dg0 + od0);
  const double tol = 4.0 * Me * 1.1102230246251565e-16;
  int sw = 0;
  for (; sw < kSyevMaxSweeps; ++sw) {
    double dg, od;
    block_norms(dg, od);
    const double off = block_sum(od);
    if (tid == 0) done = off <= tol * tol * nrm2;
    __syncthreads();
    if (done) break;
    for (int s = 0; s < Mc; ++s) {
      // rotations of this round's pairs; blocks into registers
      double dp = 0.0, dq = 0.0;
      if (rotor) {
        double c, sv;
        jacobi_rot(A[tid], A[H + tid], A[2 * H + tid], c, sv, dp, dq);
        rc[tid] = c;
        rs[tid] = sv;
        if (rec) rec[(sw * Mc + s) * H + tid] = make_double2(c, sv);
      }
      double a[kMaxBlk][4];
#pragma unroll
      for (int k = 0; k < kMaxBlk; ++k) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a[k][q] = A[rda[k] + q * nob];   // in range for unused blocks too (rda 0)
      }
      __syncthreads();
      // A <- J^T A J, written to the shifted slots
      if (rotor) {
        A[dw[0]] = dp;
        A[dw[1]] = dq;
        A[dw[2]] = 0.0;
      }
#pragma unroll
      for (int k = 0; k < kMaxBlk; ++k) {
        const int bi = bpi[k], bj = bpj[k];
        if (bi < 0) continue;
        const double ci = rc[bi], si = rs[bi], cj = rc[bj], sj = rs[bj];
        const double t00 = a[k][0] * cj - a[k][1] * sj, t01 = a[k][0] * sj + a[k][1] * cj;
        const double t10 = a[k][2] * cj - a[k][3] * sj, t11 = a[k][2] * sj + a[k][3] * cj;
        A[wra[k][0]] = ci * t00 - si * t10;
        A[wra[k][1]] = ci * t01 - si * t11;
        A[wra[k][2]] = si * t00 + ci * t10;
        A[wra[k][3]] = si * t01 + ci * t11;
      }
      __syncthreads();
    }
  }
  // ascending ranks among the m real indices (ties by index); slot = index here
  for (int i = tid; i < m; i += kSyevThreads) {
    const double li = A[jstore(i, i, Me)];
    int k = 0;
    for (int j = 0; j < m; ++j) {
      const double lj = A[jstore(j, j, Me)];
      k += (lj < li || (lj == li && j < i)) ? 1 : 0;
    }
    rank[i] = k;
  }
  __syncthreads();
  for (int i = tid; i < m; i += kSyevThreads) {
    w[rank[i]] = A[jstore(i, i, Me)];
    if (hdr) hdr[1 + i] = rank[i];
  }
  if (hdr && tid == 0) hdr[0] = sw * Mc;   // rounds recorded (whole sweeps)
}

constexpr int kReplayBatch = 8;   // recorded rounds loaded ahead

// Wavefront-wide one-lane shifts of a double (DPP wave_shl:1 / wave_shr:1 on
// both halves): lane i receives lane i + 1's value, resp. lane i - 1's; the
// lane without a source receives 0.
__device__ __forceinline__ double from_next_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_prev_lane(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// V = I J_1 J_2 ... (the recorded rotations), row r of V per workgroup of one
// wavefront; lane i holds the row's entries in the slots of pair i (first
// slot in F, second in S).  The shift after each round: F takes lane i+1's
// F (lane 0 keeps slot 0, lane H-1 takes its own S), S takes lane i-1's S
// (lane 0 takes lane 1's F).  Entry (r, c) is written to column perm[c].
__global__ void __launch_bounds__(64) syev_vectors_kernel(int m, const double2* __restrict__ rec,
                                                          const int* __restrict__ hdr, double* __restrict__ Vout,
                                                          int ldv) {
  const int r = blockIdx.x, i = threadIdx.x;
  const int Me = m + (m & 1), H = Me / 2, R = hdr[0];
  const int f = slot_first(i), sc = slot_second(i, Me);
  const bool act = i < H;
  double F = (act && f == r) ? 1.0 : 0.0, S = (act && sc == r) ? 1.0 : 0.0;
  double2 cur[kReplayBatch], nxt[kReplayBatch];
  auto load = [&](int k0, double2* b) {
#pragma unroll
    for (int j = 0; j < kReplayBatch; ++j) b[j] = (act && k0 + j < R) ? rec[(k0 + j) * H + i] : make_double2(1.0, 0.0);
  };
  load(0, cur);
  for (int k0 = 0; k0 < R; k0 += kReplayBatch) {
    load(k0 + kReplayBatch, nxt);
#pragma unroll
    for (int j = 0; j < kReplayBatch; ++j) {
      if (k0 + j >= R) break;
      const double nF = F * cur[j].x - S * cur[j].y, nS = F * cur[j].y + S * cur[j].x;
      const double Fd = from_next_lane(nF), Su = from_prev_lane(nS);
      F = i == 0 ? nF : (i == H - 1 ? nS : Fd);
      S = i == 0 ? (H > 1 ? Fd : nS) : Su;
    }
#pragma unroll
    for (int j = 0; j < kReplayBatch; ++j) cur[j] = nxt[j];
  }
  if (act && r < m) {
    const int* perm = hdr + 1;
    if (f < m) Vout[r * ldv + perm[f]] = F;
    if (sc < m) Vout[r * ldv + perm[sc]] = S;
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

hipError_t dense_syev_w(int m, const double* A, int lda, double* w, double* V, int ldv, double* work,
                        hipStream_t s) {
  if (m < 1 || m > kMaxSmall || (V && !work)) return hipErrorInvalidValue;
  const int Me = m + (m & 1);
  const size_t lds = sizeof(double) * ((size_t)Me * (Me + 1) / 2);
  int* hdr = V ? reinterpret_cast<int*>(work) : nullptr;
  double2* rec = V ? reinterpret_cast<double2*>(work + kSyevHeaderDoubles) : nullptr;
  (void)hipFuncSetAttribute((const void*)syev_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(syev_kernel, dim3(1), dim3(kSyevThreads), lds, s, m, A, lda, w, rec, hdr);
  if (V) hipLaunchKernelGGL(syev_vectors_kernel, dim3(m), dim3(64), 0, s, m, rec, hdr, V, ldv);
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
