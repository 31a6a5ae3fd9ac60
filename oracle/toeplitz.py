"""Dirichlet chain with defect cells: the perturbed block-Toeplitz model.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Paper passages followed:
  * Sec. 3 (finite lattices in a box; the defect discussion around Fig. 3.2):
    the box-case Galerkin matrix is block Toeplitz once the potential of the
    central cell is replicated to every cell; defects and the cells near the
    walls break this only in a few block rows and columns ("perturbed"
    block-Toeplitz, a low-rank correction).
  * Remark 3.2: a block-Toeplitz matrix is embedded in a block-circulant
    matrix of about twice the size, whose action is two FFTs over the block
    index and one small product per frequency.
  * Sec. 2.1-2.4: the Galerkin pair (H, S), 1D FEM Grams and the collocated
    rank-R potential, as in ``model``.

Readings where the paper is silent (all of them choices of this model):
  T1 the chain runs along dimension 1 with L cells; every dimension is a box
     dimension (reading R2).  The chain's nodes are aligned with its cells:
     n1 = nc L and pad1 = h / 2 with h = a / nc, so every cell holds the same
     nc node offsets.
  T2 pristine blocks A_s = <g_(0,mu), H_rep g_(s,nu)>, s = 0..L0, are taken on
     the chain grid extended without walls (untruncated stencils; the sums run
     over every node where the factors do not underflow).  H_rep has the
     potential V_rep: the lattice-window potential of the central cell
     (reading R4 with the window of L cells) replicated to every cell with
     period a.  T(k, m) = A_(m-k) for m >= k, A_(k-m)^T otherwise, zero when
     |k - m| > L0.  The same for S without potential.
  T3 the band half-width L0 = ceil((2 max|c_mu| + sqrt(101.4 / alpha_min)) / a)
     with alpha_min over the pristine and the scaled defect exponents (overlap
     decay below 1e-22), capped at L - 1.
  T4 X = defect cells and the cells within L0 of a wall (k < L0 or
     k > L - 1 - L0).  H_model(k, m) = T(k, m) unless k or m is in X (and
     |k - m| <= L0); then it is the block of the actual basis (exponents times
     the defect's scale factor on defect cells) on the box grid with its walls,
     with potential V_rep + sum over defect cells c in {k, m} of
     (Z_def,c - Z_nu) V_(c,nu), V_(c,nu) the collocated rank-R potential of
     nucleus nu of cell c alone.  S_model the same without potential.
     Dropped by the model: the defect charge acting on blocks that do not
     touch its cell, and the difference between V_rep and the true finite
     chain potential.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .model import Grid1D, angular_power, cell_integral_gauss, fem_1d, grids, gto_1d, sinc_rule, window


# ----------------------------------------------------------------------------- set-up

def chain_grids(inst):
    """Box grids of the chain (T1); returns (grids, nodes per cell)."""
    if inst.bc != "dirichlet" or inst.L[1] != 1 or inst.L[2] != 1:
        raise ValueError("the Toeplitz model is a Dirichlet L x 1 x 1 chain")
    L, n, a = inst.L[0], inst.n[0], inst.a
    if n % L:
        raise ValueError("n1 must be a multiple of L")
    nc = n // L
    gs = grids(inst)
    if abs(gs[0].h - a / nc) > 1e-12 * a or abs(inst.pad[0] - 0.5 * a / nc) > 1e-12 * a:
        raise ValueError("chain nodes must be cell aligned: pad1 = a / (2 nc)")
    return gs, nc


def defect_scale(inst, k: int) -> float:
    hit = np.nonzero(inst.def_cells == k)[0]
    return float(inst.def_scale[hit[0]]) if len(hit) else 1.0


def defect_charge(inst, k: int):
    hit = np.nonzero(inst.def_cells == k)[0]
    return float(inst.def_Z[hit[0]]) if len(hit) else None


def band(inst) -> int:
    """L0 of reading T3."""
    amin = float(inst.alpha.min())
    if len(inst.def_scale):
        amin = min(amin, amin * float(inst.def_scale.min()))
    jmax = float(np.abs(inst.centre).max())
    L0 = int(math.ceil((2.0 * jmax + math.sqrt(101.4 / amin)) / inst.a))
    return min(L0, inst.L[0] - 1)


def cross_cells(inst, L0: int) -> np.ndarray:
    """X of reading T4, ascending."""
    L = inst.L[0]
    walls = [k for k in range(L) if k < L0 or k > L - 1 - L0]
    return np.unique(np.concatenate([np.asarray(walls, np.int64), inst.def_cells.astype(np.int64)]))


# ----------------------------------------------------------------------------- 1D pieces

def _factors(inst, x, centre, ell, scale):
    """[len(x), m0] nodal values of the dimension-ell factors of a cell's
    functions centred at `centre` (cell centre), exponents times `scale`."""
    out = np.empty((len(x), inst.m0))
    for mu in range(inst.m0):
        l = angular_power(int(inst.ang[mu]), ell)
        out[:, mu] = gto_1d(x, float(inst.alpha[mu]) * scale, l, centre + inst.centre[mu, ell])
    return out


def _fem(x, h, L, a):
    """Truncated tridiagonal stiffness and mass on the consecutive node set x."""
    g = Grid1D(False, L, len(x), a, h, x, np.zeros(1), 0.0)
    return fem_1d(g)


def _rep_potential_cell(inst, g):
    """[M0 R, nc] V_rep factors on the nc node offsets of a cell (T2), Z_nu w_q
    folded in; node i of the chain (1-based, any integer on the extended grid)
    carries column (i - 1) mod nc."""
    L, a = inst.L[0], inst.a
    nc = inst.n[0] // L
    off = -0.5 * a + (np.arange(nc) + 0.5) * g.h     # node offsets from the cell centre
    t, w = sinc_rule(inst)
    ks, wk = window(L)
    out = np.zeros((inst.M0 * inst.R, nc))
    for nu in range(inst.M0):
        A = float(inst.nuc[nu, 0])
        for q in range(inst.R):
            acc = np.zeros(nc)
            for k, wt in zip(ks, wk):
                acc += wt * cell_integral_gauss(off, g.h, t[q], A + k * a)
            out[nu * inst.R + q] = inst.Z[nu] * w[q] * acc
    return out


def _nucleus_potential(inst, x, h, ell, centre, nu):
    """[R, len(x)] collocated potential factors of one nucleus (no window)."""
    t, _ = sinc_rule(inst)
    A = centre + float(inst.nuc[nu, ell])
    return np.stack([cell_integral_gauss(x, h, t[q], A) for q in range(inst.R)])


def _grams(Gk, Gm, A, S, P):
    """S-, A- and potential Grams between the factor sets (rows mu of cell k,
    columns nu of cell m)."""
    s = Gk.T @ (S @ Gm)
    k = Gk.T @ (A @ Gm)
    v = np.einsum("im,ti,in->tmn", Gk, P, Gm) if P is not None else None
    return s, k, v


# ----------------------------------------------------------------------------- blocks

class ChainModel:
    """Pieces of the model for one instance: the transverse Grams per pair of
    exponent scales, the pristine generators A_s (H and S) and exact blocks."""

    def __init__(self, inst):
        self.inst = inst
        self.gs, self.nc = chain_grids(inst)
        self.L0 = band(inst)
        self.X = cross_cells(inst, self.L0)
        t, w = sinc_rule(inst)
        self.w = w
        amin = float(inst.alpha.min()) * min([1.0] + list(inst.def_scale))
        jmax = float(np.abs(inst.centre).max())
        # cells of margin beyond which every factor underflows (exp < 1e-35)
        self.margin = int(math.ceil((math.sqrt(80.6 / amin) + jmax) / inst.a)) + 1
        self._trans = {}
        self.vrep = _rep_potential_cell(inst, self.gs[0])

    def rep_potential(self, i):
        """V_rep factors [M0 R, len(i)] at chain node indices i (1-based)."""
        return self.vrep[:, (np.asarray(i) - 1) % self.nc]

    def centre(self, k):
        return -0.5 * self.inst.L[0] * self.inst.a + (k + 0.5) * self.inst.a

    def transverse(self, sk, sm):
        """Dimension-2 and -3 Grams (S, A, potential [M0 R]) for exponent
        scales sk (row cell) and sm (column cell)."""
        key = (sk, sm)
        if key not in self._trans:
            inst = self.inst
            out = []
            for ell in (1, 2):
                g = self.gs[ell]
                A, S = fem_1d(g)
                Gk = _factors(inst, g.x, g.centres[0], ell, sk)
                Gm = _factors(inst, g.x, g.centres[0], ell, sm)
                P = np.concatenate([_nucleus_potential(inst, g.x, g.h, ell, g.centres[0], nu)
                                    for nu in range(inst.M0)])
                out.append(_grams(Gk, Gm, A, S, P))
            self._trans[key] = out
        return self._trans[key]

    def _combine(self, gx, ty, tz, extra=()):
        """H and S of a block from the three dimensions' Grams (Prop. 2.2)."""
        sx, kx, vx = gx
        sy, ky, vy = ty
        sz, kz, vz = tz
        S = sx * sy * sz
        H = 0.5 * (kx * sy * sz + sx * ky * sz + sx * sy * kz) - np.einsum("tmn,tmn,tmn->mn", vx, vy, vz)
        for vxe in extra:
            H = H - np.einsum("tmn,tmn,tmn->mn", vxe, vy, vz)
        return H, S

    def generator(self, s):
        """Pristine A_s (H and S), reading T2: cells 0 and s on the wall-free
        extended grid."""
        inst, g = self.inst, self.gs[0]
        E = self.margin
        i = np.arange(1 - E * self.nc, (s + 1 + E) * self.nc + 1)
        x = -0.5 * (inst.L[0] * inst.a + 2.0 * inst.pad[0]) + i * g.h
        A, S = _fem(x, g.h, inst.L[0], inst.a)
        Gk = _factors(inst, x, self.centre(0), 0, 1.0)
        Gm = _factors(inst, x, self.centre(s), 0, 1.0)
        gx = _grams(Gk, Gm, A, S, self.rep_potential(i))
        ty, tz = self.transverse(1.0, 1.0)
        return self._combine(gx, ty, tz)

    def exact_block(self, k, m):
        """H_model(k, m) and S_model(k, m) of a cross block (reading T4)."""
        inst, g = self.inst, self.gs[0]
        x = g.x
        A, S = fem_1d(g)
        sk, sm = defect_scale(inst, k), defect_scale(inst, m)
        Gk = _factors(inst, x, self.centre(k), 0, sk)
        Gm = _factors(inst, x, self.centre(m), 0, sm)
        gx = _grams(Gk, Gm, A, S, self.rep_potential(np.arange(1, g.n + 1)))
        extra = []
        for c in sorted({k, m}):
            zc = defect_charge(inst, c)
            if zc is None:
                continue
            P = []
            for nu in range(inst.M0):
                dz = zc - float(inst.Z[nu])
                P.append((dz * self.w)[:, None] * _nucleus_potential(inst, x, g.h, 0, self.centre(c), nu))
            P = np.concatenate(P)
            extra.append(np.einsum("im,ti,in->tmn", Gk, P, Gm))
        ty, tz = self.transverse(sk, sm)
        return self._combine(gx, ty, tz, extra)

    def generators(self):
        """[L0 + 1, m0, m0] stacks A_s of H and S."""
        HS = [self.generator(s) for s in range(self.L0 + 1)]
        return np.stack([h for h, _ in HS]), np.stack([s for _, s in HS])

    def cross_blocks(self):
        """{(k, m): (H, S)} for every cross block with k <= m."""
        out = {}
        L = self.inst.L[0]
        for c in self.X:
            for m in range(max(0, c - self.L0), min(L, c + self.L0 + 1)):
                k0, m0 = min(c, m), max(c, m)
                if (k0, m0) not in out:
                    out[(k0, m0)] = self.exact_block(k0, m0)
        return out


def toeplitz_dense(gen, L):
    """Dense block-Toeplitz T with T(k, m) = A_(m-k), A_(-s) = A_s^T (T2)."""
    L0 = gen.shape[0] - 1
    m0 = gen.shape[1]
    T = np.zeros((L * m0, L * m0))
    for k in range(L):
        for m in range(max(0, k - L0), min(L, k + L0 + 1)):
            blk = gen[m - k] if m >= k else gen[k - m].T
            T[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0] = blk
    return T


def model_dense(model: ChainModel, gens=None, crosses=None):
    """Dense H_model and S_model (N x N, N = m0 L)."""
    inst = model.inst
    L, m0 = inst.L[0], inst.m0
    gH, gS = gens if gens is not None else model.generators()
    H = toeplitz_dense(gH, L)
    S = toeplitz_dense(gS, L)
    cr = crosses if crosses is not None else model.cross_blocks()
    for (k, m), (bh, bs) in cr.items():
        H[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0] = bh
        S[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0] = bs
        H[m * m0:(m + 1) * m0, k * m0:(k + 1) * m0] = bh.T
        S[m * m0:(m + 1) * m0, k * m0:(k + 1) * m0] = bs.T
    return H, S


# ----------------------------------------------------------------------------- embedding

def embedding_size(L: int, L0: int) -> int:
    """Smallest power of two P >= L + L0 (Remark 3.2 asks for about 2 L)."""
    P = 1
    while P < L + L0:
        P *= 2
    return P


def embed_matvec(gen, L, x, P=None):
    """T x through the block-circulant embedding (Remark 3.2), FFT routine of
    numpy: x is [L, m0, nvec]; returns [L, m0, nvec]."""
    L0, m0 = gen.shape[0] - 1, gen.shape[1]
    P = P or embedding_size(L, L0)
    c = np.zeros((P, m0, m0))
    # y_k = sum_d B_d x_(k-d), B_d = T(k, k-d): B_d = A_d^T (d >= 0), B_(-d) = A_d
    for d in range(L0 + 1):
        c[d] = gen[d].T
        if d:
            c[P - d] = gen[d]
    xp = np.zeros((P,) + x.shape[1:])
    xp[:L] = x
    yh = np.einsum("fmn,fnv->fmv", np.fft.fft(c, axis=0), np.fft.fft(xp, axis=0))
    return np.fft.ifft(yh, axis=0)[:L].real


def lowest_eigenpairs(H, S, nev):
    """The nev lowest generalized eigenpairs (LAPACK)."""
    return scipy.linalg.eigh(H, S, subset_by_index=[0, nev - 1])
