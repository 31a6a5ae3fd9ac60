// Internal device-visible descriptors shared by the host planner and the HIP
// kernels of the lattice core-Hamiltonian library.  Plain-old-data only: the
// planner fills them on the host and copies them to device memory once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lhf {

constexpr int kMaxM0 = 32;     // basis functions per cell
constexpr int kMaxNuc = 4;     // nuclei per cell
constexpr int kMaxR = 64;      // sinc terms
constexpr int kMaxTerms = 2 + 96;  // S, K and at most 96 potential terms (M0 * R)

// One dimension of one lattice.
struct DimDev {
  int32_t L;          // cells along this dimension
  int32_t n;          // grid nodes
  int32_t nc;         // nodes per cell (replicated potential dims), else 0
  int32_t periodic;   // cyclic FEM operators and periodised basis
  int32_t replicate;  // potential stored for one cell and replicated (L >= 2)
  int32_t npot;       // stored potential nodes per term (nc or n)
  int32_t nimg;       // periodic images each side for the basis factors
  int32_t nshift;     // generator shifts computed for the Grams (slots)
  int32_t full;       // 1: slots are shifts 0..L-1; 0: slots are -L0..L0
  int32_t L0;         // band half-width (banded dims)
  int32_t kstart;     // first node of the Gram contraction window
  int32_t kwin;       // nodes in the window (cyclic from kstart); n when the
                      // basis factors are non-negligible everywhere
  int32_t ksplit;     // split-K factor of the Gram contraction
  int32_t kchunk;     // window nodes per split (multiple of 32)
  double h;           // node spacing
  double x0;          // coordinate of node 0
  double y0;          // replicated dims: offset of a cell's first node from its centre
  double a;           // lattice step
  double X0;          // centre of cell 0
  double period;      // supercell length on periodic dims
  int64_t g_off;      // doubles: nodal factors [n][m0] (node-major)
  int64_t p_off;      // doubles: potential factors [terms][npot]
  int64_t gram_off;   // elements: Grams [T][nshift][m0][m0]
  int64_t part_off;   // elements: split-K partials [ksplit][T m0][nshift m0]
  int64_t tw_off;     // complex elements: twiddles exp(-2 pi i m / L), m < L
  int64_t gh_off;     // complex elements: 1D-transformed Grams [T][L][m0][m0] (dimensions 2, 3)
};

struct LatDev {
  int32_t m0, M0, R, T;       // T = 2 + M0 R Gram terms
  int32_t L[3];
  int32_t nblk;               // L1 L2 L3
  int64_t gen_off;            // elements of this lattice's generator / Fourier stack
  int64_t w_off;              // eigenvalue offset (nblk m0)
  int64_t blk_off;            // first global block index
  int64_t half_off;           // elements of this lattice's stack in the half layout [L1][L2][L3/2+1][m0][m0]
  DimDev dim[3];
  int32_t lpow[kMaxM0][3];    // angular power per function and dimension
  double alpha[kMaxM0];
  double cen[kMaxM0][3];      // centre relative to the cell centre
  double norm[kMaxM0][3];     // 1D normalisation per dimension
  double Z[kMaxNuc];
  double nuc[kMaxNuc][3];
  double tq[kMaxR];
  double wq[kMaxR];
};

// One workgroup's share of the grouped Gram contraction: a 64 x 64 output
// tile (rows (t, nu), columns (slot, mu)) of one lattice and dimension, over
// split ks of the contraction window.
struct GramItem {
  int32_t li, d, tm, tn, ks, pad;
};

// Grouped factor work of one lattice dimension: row < 0, every basis function
// on one chunk of nodes; row >= 0 with chunk >= 0, one chunk of nodes of the
// potential term `row` of a one-cell dimension; chunk < 0, the lattice-window
// potential factor of term `row` of a replicated dimension.
struct FacItem {
  int32_t li, d, row, chunk;
};

// One lattice's share of one pass of the grouped block DFT: transform
// dimension d of X[O][B][I] (B band slots) into Y[O][L_d][I], JC outputs along
// the axis per thread (njc = ceil(L_d / JC) chunks), over the pass threads
// [tbase, tbase + O njc I); tbase is a multiple of 256 so that a workgroup
// serves one task.  The first pass reads the real generator stack of the
// lattice; later passes read an intermediate; the last writes the Fourier
// blocks.
struct DftTask {
  int32_t li, d, O, I, JC, njc, B, out_final;
  int64_t in_off, in_half;     // intermediate input: H part at in_off, S part in_half later
  int64_t out_off, out_half;   // intermediate output (when not final)
  int64_t tbase;
};

// One lattice of the fused multi-dimensional pass: workgroup w of the lattice
// (w in [wg_base, wg_base + nwg)) transforms all three dimensions for one j3,
// a chunk of J2C values of j2 and a chunk of EC block entries, writing the
// Fourier blocks once.
struct FusedTask {
  int32_t li, J2C, nj2c, EC, nec, pad;
  int64_t wg_base;
};

// One (lattice, dimension) of the 1D transform of the Grams along dimensions
// 2 and 3: outputs [T][L][m0^2] from thread `start` on (a multiple of 256).
struct GhItem {
  int32_t li, d;
  int64_t start;
};

// Host-side record of one grouped DFT launch: tasks [t0, t0 + nt) of one pass
// and one band-width class, `threads` threads (a multiple of 256), twiddles of
// axes up to `lds_tw` entries staged in LDS.
struct DftLaunch {
  int32_t pass, cls, t0, nt;
  int64_t threads;
  int32_t lds_tw;
};

}  // namespace lhf
