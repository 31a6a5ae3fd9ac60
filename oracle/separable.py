"""The paper's route: 1D Gram matrices -> generator blocks -> Fourier blocks.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Steps, in the paper's order:
  1. 1D Gram matrices per dimension (Prop. 2.2, eqs. Mass_Gal_fact and
     Lapl_Gal_fact; the potential analogue of Lemma 2.1's proof):
       S^l[k] = G_k^T S G_0,  K^l[k] = G_k^T A G_0,
       M^l_(nu,q)[k] = G_k^T diag(P^l_(nu,q)) G_0
     with G_k the nodal factors of cell k (computed directly, every shift).
  2. Hadamard combination into the generator blocks A_k = block(k, 0) of the
     three-level block-circulant matrices (Lemma 3.4, eqs. BC-Core, BC-mass,
     BC-Laplace):
       S_k = S1[k1] o S2[k2] o S3[k3]
       H_k = 1/2 (K1 o S2 o S3 + S1 o K2 o S3 + S1 o S2 o K3)
             - sum_(nu,q) Z_nu w_q M1 o M2 o M3
  3. Fourier blocks  Hbar_j = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) A_k,
     w_l = exp(-2 pi i / L_l)  (Lemma 3.1, Prop. 5.1), by numpy's forward FFT
     over the three lattice axes.
  4. Per-block generalized eigenproblems Hbar_j u = lambda Sbar_j u
     (eq. HF-FSpace-Block), by Cholesky reduction and a Hermitian eigensolver.
No band truncation: every shift k is computed.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg

from .model import fem_1d, grid_1d, nodal_factor, potential_factor, sinc_rule


def gram_1d(inst, ell: int, shifts=None):
    """1D Grams of dimension ell for every shift (or the given list).

    Returns dict with S, K: [nshift, m0, m0] and M: [M0 R, nshift, m0, m0]
    (entry (mu, nu) = <factor of g_(k,mu), Op factor of g_(0,nu)>), plus the
    Grid1D.  The potential term index is nu * R + q."""
    g = grid_1d(inst, ell)
    A, S = fem_1d(g)
    t, _ = sinc_rule(inst)
    m0 = inst.m0
    if shifts is None:
        shifts = list(range(g.L))
    G0 = np.stack([nodal_factor(inst, g, ell, mu, 0) for mu in range(m0)])   # [m0, n]
    SG0 = np.asarray((S @ G0.T).T)
    AG0 = np.asarray((A @ G0.T).T)
    P = np.stack([potential_factor(inst, g, ell, nu, t[q])
                  for nu in range(inst.M0) for q in range(inst.R)])          # [M0 R, n]
    PG0 = P[:, None, :] * G0[None, :, :]                                      # [M0 R, m0, n]
    ns = len(shifts)
    Sg = np.empty((ns, m0, m0)); Kg = np.empty((ns, m0, m0))
    Mg = np.empty((P.shape[0], ns, m0, m0))
    for i, k in enumerate(shifts):
        Gk = np.stack([nodal_factor(inst, g, ell, mu, k % g.L) for mu in range(m0)])
        Sg[i] = Gk @ SG0.T
        Kg[i] = Gk @ AG0.T
        Mg[:, i] = np.einsum("mi,tni->tmn", Gk, PG0)
    return dict(S=Sg, K=Kg, M=Mg, grid=g, shifts=list(shifts))


def term_coefficients(inst):
    """Z_nu w_q for potential term index nu * R + q."""
    _, w = sinc_rule(inst)
    return np.concatenate([inst.Z[nu] * w for nu in range(inst.M0)])


def generator_stacks(inst, grams=None):
    """Generator stacks H_gen, S_gen of shape [L1, L2, L3, m0, m0] (real)."""
    if grams is None:
        grams = [gram_1d(inst, ell) for ell in range(3)]
    c = term_coefficients(inst)
    g1, g2, g3 = grams
    S1, S2, S3 = g1["S"], g2["S"], g3["S"]
    K1, K2, K3 = g1["K"], g2["K"], g3["K"]
    Sst = np.einsum("aij,bij,cij->abcij", S1, S2, S3)
    T = 0.5 * (np.einsum("aij,bij,cij->abcij", K1, S2, S3)
               + np.einsum("aij,bij,cij->abcij", S1, K2, S3)
               + np.einsum("aij,bij,cij->abcij", S1, S2, K3))
    V = np.einsum("t,taij,tbij,tcij->abcij", c, g1["M"], g2["M"], g3["M"])
    return T - V, Sst


def fourier_blocks(stack):
    """Hbar_j = sum_k w^(j.k) A_k over the three lattice axes (Prop. 5.1)."""
    return np.fft.fftn(stack, axes=(0, 1, 2))


def block_eigvals(Hb, Sb):
    """Ascending eigenvalues of every block pair; Hb, Sb: [..., m, m].

    Cholesky reduction Sbar = C C^H, Hbar -> C^-1 Hbar C^-H, then LAPACK's
    Hermitian eigensolver, batched over the leading axes."""
    C = np.linalg.cholesky(Sb)
    Y = np.linalg.solve(C, Hb)
    Red = np.linalg.solve(C, np.conj(np.swapaxes(Y, -1, -2)))
    Red = 0.5 * (Red + np.conj(np.swapaxes(Red, -1, -2)))
    return np.linalg.eigvalsh(Red)


def block_eigvals_scipy(Hb, Sb):
    """Same as block_eigvals, one LAPACK hegv call per block (for tiny cases)."""
    flat_h = Hb.reshape(-1, *Hb.shape[-2:])
    flat_s = Sb.reshape(-1, *Sb.shape[-2:])
    out = np.stack([scipy.linalg.eigh(h, s, eigvals_only=True) for h, s in zip(flat_h, flat_s)])
    return out.reshape(*Hb.shape[:-1])


def block_circulant_dense(stack):
    """Dense N x N matrix with block (k, m) = A_((k - m) mod L) (eq. BC-Core)."""
    L1, L2, L3, m0, _ = stack.shape
    cells = [(a, b, c) for a in range(L1) for b in range(L2) for c in range(L3)]
    N = len(cells) * m0
    out = np.empty((N, N), dtype=stack.dtype)
    for i, k in enumerate(cells):
        for j, m in enumerate(cells):
            d = ((k[0] - m[0]) % L1, (k[1] - m[1]) % L2, (k[2] - m[2]) % L3)
            out[i * m0:(i + 1) * m0, j * m0:(j + 1) * m0] = stack[d]
    return out


def solve(inst):
    """Full periodic pipeline: returns dict with grams, stacks, Fourier blocks
    and per-block eigenvalues [L1, L2, L3, m0]."""
    grams = [gram_1d(inst, ell) for ell in range(3)]
    Hg, Sg = generator_stacks(inst, grams)
    Hb, Sb = fourier_blocks(Hg), fourier_blocks(Sg)
    w = block_eigvals(Hb, Sb)
    return dict(grams=grams, H_gen=Hg, S_gen=Sg, H_bar=Hb, S_bar=Sb, eig=w)
