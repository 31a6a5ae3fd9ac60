"""The plain definition: full Galerkin matrices by direct 3D grid quadrature.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

For the lattice basis {g_(k,mu)} (cell k, function mu; N = m0 L1 L2 L3) this
module builds, with no use of separability or block structure beyond what the
definitions themselves state,
  S  = G^T S_3 G                       (Sec. 2.4, eq. Lapl_Mass_Gal)
  T  = 1/2 G^T A_3 G                   (kinetic part of eq. Core_Ham)
  V  = G^T diag(p) G,  p_i = collocated lattice potential (eqs. nuc_pot,
       EwaldSumE / EwaldSumP), summed image by image in 3D
  H  = T - V                           (eq. Core_Ham, operator HFcore)
where G holds the nodal values of each 3D basis function evaluated directly
on the 3D grid, and A_3 = A x S x S + S x A x S + S x S x A, S_3 = S x S x S
act on the 3D nodal arrays (Kronecker action).  Then it solves H c = lambda S c
densely (generalized problem of Sec. 2.1).

With ``finite=True`` the potential is the finite lattice's own (eq.
EwaldSumE, the exact box case (B) of Sec. 2.3): every nucleus of every cell
k in {0..L1-1} x {0..L2-1} x {0..L3-1}, at its position, on every node, with
no window and no replication.

Defect cells (Dirichlet chains): the functions of a defect cell have their
exponents multiplied by its scale factor, and its nuclei carry the defect
charge: the change Z_def - Z_nu is added as the potential of an isolated
nucleus at its position, on every node (no window, no replication).

Basis order: cell index (k1 L2 + k2) L3 + k3, then mu.
Feasible for N * n1 n2 n3 up to ~1e9 (the 8-cell chain at 128^3 is the
largest case used).
"""

from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg

from .model import (angular_power, central_offsets, cell_integral_gauss, fem_1d,
                    gto_norm, grids, image_range, sinc_rule, window)


def _apply_along(M, arr, axis):
    moved = np.moveaxis(arr, axis, 0)
    shp = moved.shape
    out = M @ moved.reshape(shp[0], -1)
    return np.moveaxis(np.asarray(out).reshape(shp), 0, axis)


def basis_3d(inst, gs):
    """[N, n1 n2 n3] nodal values of every lattice basis function, each
    evaluated as a 3D Gaussian (summed over supercell translates on periodic
    dimensions)."""
    X = np.meshgrid(gs[0].x, gs[1].x, gs[2].x, indexing="ij")
    L1, L2, L3 = inst.L
    out = np.empty((inst.m0 * L1 * L2 * L3, X[0].size))
    scale = {int(c): float(f) for c, f in zip(inst.def_cells, inst.def_scale)}
    row = 0
    for k1, k2, k3 in itertools.product(range(L1), range(L2), range(L3)):
        kk = (k1, k2, k3)
        f_cell = scale.get(cell_index(inst.L, kk), 1.0)
        for mu in range(inst.m0):
            alpha = float(inst.alpha[mu]) * f_cell
            ls = [angular_power(int(inst.ang[mu]), ell) for ell in range(3)]
            nrm = np.prod([gto_norm(alpha, ls[ell]) for ell in range(3)])
            c = [gs[ell].centres[kk[ell]] + inst.centre[mu, ell] for ell in range(3)]
            ranges = [range(-image_range(gs[ell], alpha), image_range(gs[ell], alpha) + 1)
                      for ell in range(3)]
            acc = np.zeros(X[0].shape)
            for s in itertools.product(*ranges):
                d = [X[ell] - (c[ell] + s[ell] * gs[ell].period) for ell in range(3)]
                val = np.exp(-alpha * (d[0] ** 2 + d[1] ** 2 + d[2] ** 2))
                for ell in range(3):
                    if ls[ell]:
                        val = val * d[ell]
                acc += val
            out[row] = (nrm * acc).ravel()
            row += 1
    return out


def potential_3d(inst, gs, finite=False):
    """Collocated lattice potential on every node, summed image by image.

    For each nucleus, sinc node and lattice image k (product of the 1D windows
    of reading R4, weights multiplied), the collocated Gaussian term is the
    product of its three 1D cell integrals; the image sum is done explicitly
    over all 3D images (the form of eq. EwaldSumE), on node offsets relative to
    the centre of the cell holding them (replication of eq. EwaldSumP)."""
    t, w = sinc_rule(inst)
    ys, wins = [], []
    for g in gs:
        if finite:
            # every cell of the finite lattice: node positions relative to
            # cell 0's centre, images at the other cells' centres
            ys.append(g.x - g.centres[0])
            wins.append((np.arange(g.L), np.ones(g.L)))
        elif g.L == 1:
            ys.append(g.x - g.centres[0])
            wins.append(window(g.L))
        else:
            ys.append(central_offsets(g)[0])
            wins.append(window(g.L))
    p = np.zeros((gs[0].n, gs[1].n, gs[2].n))
    for nu in range(inst.M0):
        A = inst.nuc[nu]
        for q in range(inst.R):
            for (k1, w1), (k2, w2), (k3, w3) in itertools.product(
                    zip(*wins[0]), zip(*wins[1]), zip(*wins[2])):
                kk = (k1, k2, k3)
                f = [cell_integral_gauss(ys[ell], gs[ell].h, t[q], A[ell] + kk[ell] * gs[ell].a)
                     for ell in range(3)]
                p += (inst.Z[nu] * w[q] * w1 * w2 * w3) * np.einsum("i,j,k->ijk", f[0], f[1], f[2])
    # defect charges: isolated nuclei at their positions
    L1, L2, L3 = inst.L
    for c, zc in zip(inst.def_cells, inst.def_Z):
        c = int(c)
        kk = (c // (L2 * L3), (c // L3) % L2, c % L3)
        for nu in range(inst.M0):
            dz = float(zc) - float(inst.Z[nu])
            A = [gs[ell].centres[kk[ell]] + inst.nuc[nu, ell] for ell in range(3)]
            for q in range(inst.R):
                f = [cell_integral_gauss(gs[ell].x, gs[ell].h, t[q], A[ell]) for ell in range(3)]
                p += (dz * w[q]) * np.einsum("i,j,k->ijk", f[0], f[1], f[2])
    return p


def dense_matrices(inst, finite=False):
    """Dense (H, S, T, V), each N x N, by 3D quadrature (``finite``: the
    finite lattice's own potential, eq. EwaldSumE)."""
    gs = grids(inst)
    G = basis_3d(inst, gs)
    shp = (gs[0].n, gs[1].n, gs[2].n)
    ops = [fem_1d(g) for g in gs]   # (A, S) per dimension
    N = G.shape[0]
    SG = np.empty_like(G)
    AG = np.empty_like(G)
    for r in range(N):
        f = G[r].reshape(shp)
        s1 = _apply_along(ops[0][1], f, 0)
        s12 = _apply_along(ops[1][1], s1, 1)
        SG[r] = _apply_along(ops[2][1], s12, 2).ravel()
        a = _apply_along(ops[2][0], s12, 2)                                   # S x S x A
        a = a + _apply_along(ops[2][1], _apply_along(ops[1][0], s1, 1), 2)     # S x A x S
        a = a + _apply_along(ops[2][1],
                             _apply_along(ops[1][1], _apply_along(ops[0][0], f, 0), 1), 2)  # A x S x S
        AG[r] = a.ravel()
    p = potential_3d(inst, gs, finite).ravel()
    S = G @ SG.T
    T = 0.5 * (G @ AG.T)
    V = G @ (G * p).T
    H = T - V
    return H, S, T, V


def dense_eigvals(H, S):
    """All generalized eigenvalues of (H, S), ascending (LAPACK)."""
    return scipy.linalg.eigh(H, S, eigvals_only=True)


def block(Mat, m0, k, m):
    return Mat[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]


def cell_index(L, k):
    return (k[0] * L[1] + k[1]) * L[2] + k[2]
