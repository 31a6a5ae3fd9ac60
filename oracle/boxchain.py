"""The exact box case (B) of a Dirichlet chain: finite-lattice potential,
every block computed.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Paper passages followed:
  * Sec. 2.3 (case (B), eq. EwaldSumE): the potential of a lattice system in
    a box is the sum over every unit cell k of the finite lattice of the
    potentials of its nuclei; in the canonical form of eq. EwaldTensorGl each
    rank term is a product of 1D factors, each the sum over the cells of the
    shifted 1D collocation vectors.
  * Sec. 2.3 (eq. nuc_MatrSparsP, Lemma 2.1): the block (k, m) of the
    Galerkin matrix is the contraction of the basis of cells k and m with that
    potential, banded: blocks with |k - m| beyond the overlap constant vanish.
  * Sec. 2.3, items (A) and (B) after Fig. 2.4: the box matrix differs from
    the block-Toeplitz (replicated central cell) one by the asymmetry of the
    finite lattice sum (A, non-local) and by the boundary layer within L0 of
    the walls (B, local).
  * Sec. 2.4: FEM Grams and nodal basis on the box grid with its walls.

Readings (shared with the perturbed block-Toeplitz model where they overlap):
  T1 chain along dimension 1, cell-aligned nodes (n1 = nc L, pad1 = a/(2 nc)),
     every dimension a box dimension (reading R2 of ``model``).
  B1 the potential along the chain is sum over cells c = 0..L-1 and nuclei nu
     of Z_(nu, c) w_q phi_q(x; X_c + a_nu), with Z_(nu, c) the defect charge
     on defect cells (every nucleus of a defect cell carries it) and Z_nu
     elsewhere; across the chain each nucleus's own factors.  No window, no
     replication, no defect correction: the lattice sum itself.
  B2 every block (k, m) uses the actual basis of cells k and m (exponents times
     the defect's scale factor on defect cells) on the box grid with its
     walls; blocks with |k - m| > L0 (L0 of reading T3) are zero (overlap
     below 1e-22); ``full=True`` computes them anyway.
"""

from __future__ import annotations

import numpy as np

from .model import cell_integral_gauss, fem_1d, sinc_rule
from .toeplitz import ChainModel, _factors, _grams, defect_charge, defect_scale


def finite_lattice_potential(inst, g):
    """[M0 R, n] chain factors of the finite lattice's potential (B1), Z w_q
    folded in, on the chain's box nodes g.x."""
    L, a = inst.L[0], inst.a
    t, w = sinc_rule(inst)
    out = np.zeros((inst.M0 * inst.R, g.n))
    centres = -0.5 * L * a + (np.arange(L) + 0.5) * a
    for nu in range(inst.M0):
        for c in range(L):
            zc = defect_charge(inst, c)
            z = float(inst.Z[nu]) if zc is None else zc
            A = centres[c] + float(inst.nuc[nu, 0])
            for q in range(inst.R):
                out[nu * inst.R + q] += z * w[q] * cell_integral_gauss(g.x, g.h, t[q], A)
    return out


class BoxChain:
    """The exact box operator of a Dirichlet chain (reading B1, B2)."""

    def __init__(self, inst):
        self.model = ChainModel(inst)          # grids, band, transverse Grams
        self.inst = inst
        self.L0 = self.model.L0
        g = self.model.gs[0]
        self.pot = finite_lattice_potential(inst, g)
        self._fem = fem_1d(g)

    def block(self, k, m):
        """H_box(k, m), S_box(k, m)."""
        inst, g = self.inst, self.model.gs[0]
        A, S = self._fem
        sk, sm = defect_scale(inst, k), defect_scale(inst, m)
        Gk = _factors(inst, g.x, self.model.centre(k), 0, sk)
        Gm = _factors(inst, g.x, self.model.centre(m), 0, sm)
        gx = _grams(Gk, Gm, A, S, self.pot)
        ty, tz = self.model.transverse(sk, sm)
        return self.model._combine(gx, ty, tz)

    def blocks(self, full=False):
        """{(k, m): (H, S)} for k <= m within the band (every pair if full)."""
        L = self.inst.L[0]
        out = {}
        for k in range(L):
            hi = L if full else min(L, k + self.L0 + 1)
            for m in range(k, hi):
                out[(k, m)] = self.block(k, m)
        return out

    def dense(self, full=False):
        """Dense H_box, S_box (N x N)."""
        L, m0 = self.inst.L[0], self.inst.m0
        H = np.zeros((L * m0, L * m0))
        S = np.zeros((L * m0, L * m0))
        for (k, m), (bh, bs) in self.blocks(full).items():
            H[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0] = bh
            S[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0] = bs
            H[m * m0:(m + 1) * m0, k * m0:(k + 1) * m0] = bh.T
            S[m * m0:(m + 1) * m0, k * m0:(k + 1) * m0] = bs.T
        return H, S
