"""Three-level block-Toeplitz operator of a lattice in a box and its
three-level block-circulant embedding.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Paper passages followed:
  * Sec. 2.3, item (A) after Fig. 2.4: replicating the central cell's
    potential to every cell makes the box matrix shift invariant,
    V_km = V_(k-m), a block-Toeplitz form with (2 L0 + 1) block bands.
  * Lemma 2.1 / Prop. 2.2 (items (C)): the Galerkin matrices of a lattice
    in a box are symmetric three-level block-Toeplitz matrices; Def. 5.4
    (class BT_s(d, L, m0)) defines them level by level.
  * Remark 3.2: a block-Toeplitz matrix extends to a block-circulant one of
    about double size at each level, whose action is a multilevel FFT, one
    small product per frequency, and the inverse FFT.
  * Sec. 2.4 and Prop. 2.2: 1D FEM Grams, separable combination.

Readings (the 3D analogue of readings T1-T3 of ``toeplitz``):
  U1 every dimension is a box dimension.  A dimension with L >= 2 cells has
     cell-aligned nodes, n = nc L and pad = a / (2 nc); its generators are
     taken on the node set extended without walls.  A one-cell dimension is
     an ordinary box dimension with its walls (reading R2), shift 0 only.
  U2 generators A_s(mu, nu) = <g_(0,mu), H_rep g_(s,nu)>, s in
     [-L0_1, L0_1] x [-L0_2, L0_2] x [-L0_3, L0_3], H_rep with the potential
     replicated from the central cell: per multi-cell dimension the
     lattice-window factors of reading R4 at the node offsets of a cell,
     repeated with period a; per one-cell dimension the nucleus's own factor.
     They are Hadamard combinations of 1D Grams G_l[s_l] with
     G_l[-s] = G_l[s]^T (translation invariance; the 1D operators are
     symmetric).
  U3 L0_l of reading T3 on each multi-cell dimension (0 on one-cell ones);
     T(k, m) = A_(m-k), zero when some |m_l - k_l| > L0_l.
"""

from __future__ import annotations

import math

import numpy as np

from .model import angular_power, cell_integral_gauss, fem_1d, grids, gto_1d, sinc_rule, window
from .toeplitz import _fem, _grams


def bands(inst):
    """L0 per dimension (reading U3)."""
    amin = float(inst.alpha.min())
    jmax = float(np.abs(inst.centre).max())
    L0 = int(math.ceil((2.0 * jmax + math.sqrt(101.4 / amin)) / inst.a))
    return tuple(min(L0, L - 1) for L in inst.L)


def _check(inst):
    if inst.bc != "dirichlet":
        raise ValueError("the three-level Toeplitz operator is for a lattice in a box")
    for ell in range(3):
        L, n = inst.L[ell], inst.n[ell]
        if L >= 2:
            if n % L:
                raise ValueError("multi-cell dimensions need n a multiple of L")
            nc = n // L
            if abs(inst.pad[ell] - 0.5 * inst.a / nc) > 1e-12 * inst.a:
                raise ValueError("multi-cell dimensions need cell-aligned nodes: pad = a / (2 nc)")


def _factors(inst, x, centre, ell):
    out = np.empty((len(x), inst.m0))
    for mu in range(inst.m0):
        l = angular_power(int(inst.ang[mu]), ell)
        out[:, mu] = gto_1d(x, float(inst.alpha[mu]), l, centre + inst.centre[mu, ell])
    return out


def grams_1d(inst, ell, L0):
    """Grams of dimension ell for shifts s = 0..L0 (U1, U2): dict S, K [L0+1,
    m0, m0] and M [M0 R, L0+1, m0, m0], entry (mu, nu) = <g_(0,mu), O
    g_(s,nu)>; Z_nu w_q folded into dimension 1."""
    L, a = inst.L[ell], inst.a
    t, w = sinc_rule(inst)
    fold = ell == 0
    g = grids(inst)[ell]
    if L == 1:
        A, S = fem_1d(g)
        G = _factors(inst, g.x, g.centres[0], ell)
        P = []
        for nu in range(inst.M0):
            for q in range(inst.R):
                c = inst.Z[nu] * w[q] if fold else 1.0
                P.append(c * cell_integral_gauss(g.x, g.h, t[q], g.centres[0] + inst.nuc[nu, ell]))
        s, k, v = _grams(G, G, A, S, np.array(P))
        return dict(S=s[None], K=k[None], M=v[:, None])
    nc = inst.n[ell] // L
    h = a / nc
    amin = float(inst.alpha.min())
    jmax = float(np.abs(inst.centre).max())
    E = int(math.ceil((math.sqrt(80.6 / amin) + jmax) / a)) + 1
    # wall-free node set from E cells left of cell 0 to E cells right of cell L0
    i = np.arange(1 - E * nc, (L0 + 1 + E) * nc + 1)
    x = -0.5 * (L * a + 2.0 * inst.pad[ell]) + i * h
    A, S = _fem(x, h, L, a)
    centre = lambda k: -0.5 * L * a + (k + 0.5) * a
    # replicated window potential: node i of a cell sits at offset -a/2 + ((i - 1) mod nc + 1/2) h
    off = -0.5 * a + (((i - 1) % nc) + 0.5) * h
    ks, wk = window(L)
    P = []
    for nu in range(inst.M0):
        for q in range(inst.R):
            acc = np.zeros(len(x))
            for kk, wt in zip(ks, wk):
                acc += wt * cell_integral_gauss(off, h, t[q], inst.nuc[nu, ell] + kk * a)
            P.append((inst.Z[nu] * w[q] if fold else 1.0) * acc)
    P = np.array(P)
    G0 = _factors(inst, x, centre(0), ell)
    Sg, Kg, Mg = [], [], []
    for s in range(L0 + 1):
        Gs = _factors(inst, x, centre(s), ell)
        s_, k_, v_ = _grams(G0, Gs, A, S, P)
        Sg.append(s_); Kg.append(k_); Mg.append(v_)
    return dict(S=np.array(Sg), K=np.array(Kg), M=np.stack(Mg, axis=1))


def _signed(g, s):
    """G[s] for a signed shift (G[-s] = G[s]^T)."""
    return g[s] if s >= 0 else np.swapaxes(g[-s], -1, -2)


def generators(inst):
    """A_s of H and S for s in the signed band, arrays [2L0_1+1, 2L0_2+1,
    2L0_3+1, m0, m0] indexed by s + L0 (U2)."""
    _check(inst)
    L0 = bands(inst)
    gr = [grams_1d(inst, ell, L0[ell]) for ell in range(3)]
    shp = tuple(2 * b + 1 for b in L0) + (inst.m0, inst.m0)
    H = np.zeros(shp)
    Sm = np.zeros(shp)
    for a1 in range(-L0[0], L0[0] + 1):
        for a2 in range(-L0[1], L0[1] + 1):
            for a3 in range(-L0[2], L0[2] + 1):
                s = (a1, a2, a3)
                S1, S2, S3 = (_signed(gr[l]["S"], s[l]) for l in range(3))
                K1, K2, K3 = (_signed(gr[l]["K"], s[l]) for l in range(3))
                M1, M2, M3 = (_signed(np.swapaxes(gr[l]["M"], 0, 1), s[l]) for l in range(3))
                idx = (a1 + L0[0], a2 + L0[1], a3 + L0[2])
                Sm[idx] = S1 * S2 * S3
                H[idx] = 0.5 * (K1 * S2 * S3 + S1 * K2 * S3 + S1 * S2 * K3) - (M1 * M2 * M3).sum(axis=0)
    return H, Sm


def dense(gen, L):
    """Dense three-level block-Toeplitz matrix T(k, m) = A_(m-k) (U3), cells in
    C order k = (k1 L2 + k2) L3 + k3."""
    L0 = tuple((gen.shape[l] - 1) // 2 for l in range(3))
    m0 = gen.shape[-1]
    cells = [(a, b, c) for a in range(L[0]) for b in range(L[1]) for c in range(L[2])]
    N = len(cells) * m0
    T = np.zeros((N, N))
    for i, k in enumerate(cells):
        for j, m in enumerate(cells):
            d = tuple(m[l] - k[l] for l in range(3))
            if all(abs(d[l]) <= L0[l] for l in range(3)):
                T[i * m0:(i + 1) * m0, j * m0:(j + 1) * m0] = gen[d[0] + L0[0], d[1] + L0[1], d[2] + L0[2]]
    return T


def embedding_sizes(L, L0):
    """Smallest powers of two P_l >= L_l + L0_l (1 for one-cell dimensions)."""
    out = []
    for Ll, b in zip(L, L0):
        P = 1
        while P < Ll + b:
            P *= 2
        out.append(P)
    return tuple(out)


def embed_matvec(gen, L, x, P=None):
    """T x through the three-level block-circulant embedding (Remark 3.2),
    numpy's FFT: x is [L1, L2, L3, m0, nvec]; returns the same shape.
    y_k = sum_d B_d x_(k-d) with B_d = T(k, k - d) = A_(-d), placed at d mod P."""
    L0 = tuple((gen.shape[l] - 1) // 2 for l in range(3))
    m0 = gen.shape[-1]
    P = P or embedding_sizes(L, L0)
    c = np.zeros(tuple(P) + (m0, m0))
    for d1 in range(-L0[0], L0[0] + 1):
        for d2 in range(-L0[1], L0[1] + 1):
            for d3 in range(-L0[2], L0[2] + 1):
                c[d1 % P[0], d2 % P[1], d3 % P[2]] = gen[-d1 + L0[0], -d2 + L0[1], -d3 + L0[2]]
    xp = np.zeros(tuple(P) + x.shape[3:])
    xp[:L[0], :L[1], :L[2]] = x
    ax = (0, 1, 2)
    yh = np.einsum("abcmn,abcnv->abcmv", np.fft.fftn(c, axes=ax), np.fft.fftn(xp, axes=ax))
    return np.fft.ifftn(yh, axes=ax)[:L[0], :L[1], :L[2]].real
