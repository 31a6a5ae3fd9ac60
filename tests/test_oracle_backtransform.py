"""Pins of the oracle's eigenvector back-transform (Prop. 5.1, eq. eigvecA).

The back-transformed vectors are checked against things other than the
formula that makes them:
  * they solve the dense generalized problem H u = lambda S u, with (H, S)
    assembled by direct 3D quadrature (dense3d), and are S-orthonormal;
  * they equal the explicit matrix product (F^* x I) bdiag(Ubar_j) with the
    unitary Fourier matrices written out entry by entry;
  * per eigenvalue cluster they span the same S-orthogonal projector as the
    eigenvectors of an independent dense LAPACK solve (several eigenvectors
    are correct inside a cluster: the conjugate pair j, -j always forms one);
  * a phase of the wrong sign, a missing 1/sqrt(L) or a reversed order of the
    lattice levels, planted in the oracle, fails the first check.
"""

import math

import numpy as np
import pytest
import scipy.linalg

from oracle import backtransform, dense3d, separable
from synth import tiny_instance

CASES = [
    dict(L=(5, 1, 1), n=(40, 18, 18), n_s=3, n_p=0, seed=81),      # odd chain
    dict(L=(4, 1, 1), n=(32, 20, 20), n_s=2, n_p=1, seed=82),      # even chain, s + p
    dict(L=(3, 2, 1), n=(24, 16, 14), n_s=2, n_p=1, seed=83),      # 2D sheet
    dict(L=(2, 3, 2), n=(16, 24, 16), n_s=2, n_p=0, seed=84),      # 3D
]
IDS = ["L" + "x".join(map(str, c["L"])) for c in CASES]


def _solve(case):
    inst = tiny_instance(R=5, **case)
    H, S, _, _ = dense3d.dense_matrices(inst)
    res = separable.solve(inst)
    w, Ub = backtransform.block_eigenpairs(res["H_bar"], res["S_bar"])
    return inst, H, S, w, Ub


def _residual_and_orthonormality(inst, H, S, w, Ub):
    vals, U = backtransform.all_lattice_eigenvectors(inst.L, w, Ub)
    scale = np.abs(H).max()
    res = np.abs(H @ U - (S @ U) * vals[None, :]).max()
    orth = np.abs(U.conj().T @ S @ U - np.eye(U.shape[1])).max()
    return res / scale, orth


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_backtransform_solves_the_dense_problem(case):
    inst, H, S, w, Ub = _solve(case)
    res, orth = _residual_and_orthonormality(inst, H, S, w, Ub)
    assert res < 1e-11, res
    assert orth < 1e-11, orth


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_backtransform_equals_explicit_kronecker_product(case):
    inst = tiny_instance(R=5, **case)
    res = separable.solve(inst)
    w, Ub = backtransform.block_eigenpairs(res["H_bar"], res["S_bar"])
    m0 = inst.m0

    def F(L):
        j = np.arange(L)
        return np.exp(-2j * np.pi * np.outer(j, j) / L) / math.sqrt(L)
    FL = np.kron(np.kron(F(inst.L[0]), F(inst.L[1])), F(inst.L[2]))
    big = np.kron(FL.conj().T, np.eye(m0))
    bdiag = scipy.linalg.block_diag(*Ub.reshape(-1, m0, m0))
    _, U = backtransform.all_lattice_eigenvectors(inst.L, w, Ub)
    assert np.abs(big @ bdiag - U).max() < 1e-13


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_backtransform_clusters_match_dense_solve(case):
    inst, H, S, w, Ub = _solve(case)
    vals, U = backtransform.all_lattice_eigenvectors(inst.L, w, Ub)
    order = np.argsort(vals)
    vals, U = vals[order], U[:, order]
    ev, Y = scipy.linalg.eigh(H, S)
    scale = max(1.0, np.abs(ev).max())
    assert np.abs(vals - ev).max() < 1e-10 * scale
    # clusters: runs of eigenvalues closer than 1e-7 of the scale
    start = 0
    nclusters = 0
    for i in range(1, len(ev) + 1):
        if i == len(ev) or ev[i] - ev[i - 1] > 1e-7 * scale:
            X, Yc = U[:, start:i], Y[:, start:i]
            k = i - start
            overlap = Yc.conj().T @ S @ X          # k x k, unitary when the spans agree
            assert abs(k - np.linalg.norm(overlap) ** 2) < 1e-9, (start, k)
            nclusters += 1
            start = i
    assert nclusters < len(ev)   # conjugate pairs j, -j do form clusters


def _wrong_sign(L, j):
    return np.conj(_ORIG(L, j))


def _no_norm(L, j):
    return _ORIG(L, j) * math.sqrt(L[0] * L[1] * L[2])


def _reversed_levels(L, j):
    k3, k2, k1 = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    arg = j[0] * k1 / L[0] + j[1] * k2 / L[1] + j[2] * k3 / L[2]
    return (np.exp(2j * np.pi * arg) / np.sqrt(L[0] * L[1] * L[2])).ravel()


_ORIG = backtransform.cell_phases


_LOPSIDED_3D = dict(L=(3, 1, 2), n=(24, 14, 16), n_s=2, n_p=0, seed=85)


@pytest.mark.parametrize("bad,case", [(_wrong_sign, CASES[0]), (_wrong_sign, CASES[2]), (_no_norm, CASES[1]),
                                      (_reversed_levels, CASES[2]), (_reversed_levels, _LOPSIDED_3D)],
                         ids=["sign-chain", "sign-sheet", "norm", "levels-sheet", "levels-3d"])
def test_planted_backtransform_mistakes_are_caught(monkeypatch, bad, case):
    inst, H, S, w, Ub = _solve(case)
    monkeypatch.setattr(backtransform, "cell_phases", bad)
    res, orth = _residual_and_orthonormality(inst, H, S, w, Ub)
    assert res > 1e-6 or orth > 1e-6, (res, orth)
