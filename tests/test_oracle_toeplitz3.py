"""Pins of the three-level block-Toeplitz operator (oracle.toeplitz3; Sec.
2.3 item (A), Def. 5.4, Remark 3.2) against independent routes:

* the generators equal the blocks of interior cell pairs of the direct 3D
  quadrature of the box lattice (oracle.dense3d, which replicates the
  central cell's window potential per dimension and truncates the stencils at
  the walls; interior functions never reach a wall), for every signed shift
  the interior allows, mixed signs included -- this pins the 1D Grams on the
  wall-free grids, the replicated potential, the transposition G[-s] =
  G[s]^T and the separable combination;
* the matrix is symmetric with A_(-s) = A_s^T, yet A_s != A_s^T (so a sign
  slip in the shift convention cannot hide);
* the three-level circulant-embedding matvec (numpy FFT) equals the dense
  three-level Toeplitz product, one-cell levels and lengths that are not
  powers of two included; a planted sign slip in the embedding fails.
"""

import itertools

import numpy as np
import pytest

from oracle import dense3d, toeplitz3
from synth import make_instance


def _box(L, nc=8, **kw):
    a = 5.0
    n = tuple(nc * x if x > 1 else 12 for x in L)
    pad = tuple(a / (2 * nc) if x > 1 else 4.0 for x in L)
    args = dict(name="box3", L=L, n=n, bc="dirichlet", a=a, pad=pad, n_s=2, n_p=0, exp_range=(2.0, 4.0), Z=2, R=6,
                seed=191)
    args.update(kw)
    return make_instance(**args)


@pytest.mark.parametrize("L,kw", [((8, 7, 1), dict(n_p=1)), ((6, 6, 6), dict())], ids=["sheet", "cube"])
def test_generators_equal_interior_blocks_of_3d_quadrature(L, kw):
    inst = _box(L, **kw)
    L0 = toeplitz3.bands(inst)
    assert L0[0] == 2
    gH, gS = toeplitz3.generators(inst)
    H, S, _, _ = dense3d.dense_matrices(inst)
    m0 = inst.m0
    interior = [range(b, Ll - b) if Ll > 1 else range(1) for Ll, b in zip(L, L0)]
    cells = list(itertools.product(*interior))
    idx = lambda k: (k[0] * L[1] + k[1]) * L[2] + k[2]
    seen = set()
    for k in cells:
        for m in cells:
            d = tuple(m[l] - k[l] for l in range(3))
            if any(abs(d[l]) > L0[l] for l in range(3)):
                continue
            g = tuple(d[l] + L0[l] for l in range(3))
            bh = H[idx(k) * m0:(idx(k) + 1) * m0, idx(m) * m0:(idx(m) + 1) * m0]
            bs = S[idx(k) * m0:(idx(k) + 1) * m0, idx(m) * m0:(idx(m) + 1) * m0]
            assert np.abs(bh - gH[g]).max() <= 1e-12 * np.abs(H).max(), (k, m)
            assert np.abs(bs - gS[g]).max() <= 1e-13 * np.abs(S).max(), (k, m)
            seen.add(d)
    # mixed-sign shifts are among those checked
    assert any(d[0] * d[1] < 0 for d in seen) or L[1] == 1


def test_symmetry_and_shift_convention():
    inst = _box((5, 4, 3), nc=6, exp_range=(0.6, 2.0), n_p=1)
    gH, gS = toeplitz3.generators(inst)
    L0 = toeplitz3.bands(inst)
    for gen in (gH, gS):
        neg = gen[::-1, ::-1, ::-1]
        assert np.abs(neg - np.swapaxes(gen, -1, -2)).max() <= 1e-14 * np.abs(gen).max()
        T = toeplitz3.dense(gen, inst.L)
        assert np.abs(T - T.T).max() <= 1e-14 * np.abs(T).max()
    one = gH[L0[0] + 1, L0[1], L0[2]]
    assert np.abs(one - one.T).max() > 1e-4 * np.abs(one).max()


@pytest.mark.parametrize("L", [(5, 4, 3), (7, 1, 1), (3, 1, 6), (6, 5, 1)])
def test_embedding_matvec_equals_dense(L):
    inst = _box(L, nc=6, exp_range=(1.5, 4.0))
    gH, gS = toeplitz3.generators(inst)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(tuple(L) + (inst.m0, 3))
    for gen in (gH, gS):
        T = toeplitz3.dense(gen, L)
        want = (T @ x.reshape(-1, 3)).reshape(x.shape)
        got = toeplitz3.embed_matvec(gen, L, x)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        # a larger embedding gives the same product
        P = tuple(2 * p for p in toeplitz3.embedding_sizes(L, toeplitz3.bands(inst)))
        assert np.abs(toeplitz3.embed_matvec(gen, L, x, P) - want).max() <= 1e-12 * np.abs(want).max()


def test_planted_embedding_sign_slip_fails():
    inst = _box((5, 4, 3), nc=6, exp_range=(0.6, 2.0), n_p=1)
    gH, _ = toeplitz3.generators(inst)
    T = toeplitz3.dense(gH, inst.L)
    x = np.random.default_rng(8).standard_normal(tuple(inst.L) + (inst.m0, 2))
    want = (T @ x.reshape(-1, 2)).reshape(x.shape)
    # B_d = A_d instead of A_(-d): the generators reversed in every level
    bad = toeplitz3.embed_matvec(gH[::-1, ::-1, ::-1], inst.L, x)
    assert np.abs(bad - want).max() > 1e-6 * np.abs(want).max()    # far above the 1e-12 of the check
