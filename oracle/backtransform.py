"""Eigenvectors of the full lattice problem from the Fourier-block ones.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Prop. 5.1 (eq. eigvecA): with F = F_L1 x F_L2 x F_L3 the unitary Fourier
matrix of the lattice, (F_L)_(j,k) = w^(j k) / sqrt(L), w = exp(-2 pi i / L),
the block-circulant pair (H, S) is block-diagonalised by F x I_m0 (Lemma 3.1),
and its eigenvectors are U = (F^* x I_m0) bdiag(Ubar_j), where the columns of
Ubar_j are the eigenvectors of the Fourier block pair (Hbar_j, Sbar_j)
(eq. HF-FSpace-Block).  Column c of Ubar_j becomes the vector whose block on
cell k is
    U(k) = L^(-1/2) exp(+2 pi i (j1 k1 / L1 + j2 k2 / L2 + j3 k3 / L3)) Ubar_j(:, c),
(the column j of F^*), cells in C order k = (k1 L2 + k2) L3 + k3 as in the
dense matrices of dense3d and separable.block_circulant_dense.  If the columns
of Ubar_j are Sbar_j-orthonormal, the full set is S-orthonormal.
"""

from __future__ import annotations

import numpy as np


def block_eigenpairs(Hb, Sb):
    """Ascending eigenvalues and Sbar-orthonormal eigenvectors of every block
    pair; Hb, Sb: [..., m, m].  Cholesky reduction Sbar = C C^H, LAPACK's
    Hermitian eigensolver on C^-1 Hbar C^-H, back substitution u = C^-H v."""
    C = np.linalg.cholesky(Sb)
    Y = np.linalg.solve(C, Hb)
    Red = np.linalg.solve(C, np.conj(np.swapaxes(Y, -1, -2)))
    Red = 0.5 * (Red + np.conj(np.swapaxes(Red, -1, -2)))
    w, V = np.linalg.eigh(Red)
    U = np.linalg.solve(np.conj(np.swapaxes(C, -1, -2)), V)
    return w, U


def cell_phases(L, j):
    """Column j = (j1, j2, j3) of F^*: exp(+2 pi i sum_l j_l k_l / L_l) / sqrt(L)
    for every cell k in C order."""
    k1, k2, k3 = np.meshgrid(np.arange(L[0]), np.arange(L[1]), np.arange(L[2]), indexing="ij")
    arg = j[0] * k1 / L[0] + j[1] * k2 / L[1] + j[2] * k3 / L[2]
    return (np.exp(2j * np.pi * arg) / np.sqrt(L[0] * L[1] * L[2])).ravel()


def lattice_eigenvector(L, Ubar, j, c):
    """The full eigenvector (length L1 L2 L3 m0, cell-major) of column c of
    the Fourier block j; Ubar: [L1, L2, L3, m0, m0]."""
    ph = cell_phases(L, j)
    return (ph[:, None] * Ubar[j[0], j[1], j[2]][:, c][None, :]).ravel()


def all_lattice_eigenvectors(L, w, Ubar):
    """Every eigenpair of the full problem: eigenvalues [N] and eigenvectors
    [N, N] (column n), ordered by block j in C order, then column c."""
    vals, cols = [], []
    for j1 in range(L[0]):
        for j2 in range(L[1]):
            for j3 in range(L[2]):
                for c in range(Ubar.shape[-1]):
                    vals.append(w[j1, j2, j3, c])
                    cols.append(lattice_eigenvector(L, Ubar, (j1, j2, j3), c))
    return np.array(vals), np.stack(cols, axis=1)
