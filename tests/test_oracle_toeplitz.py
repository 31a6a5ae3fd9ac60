"""Pins of the Dirichlet-chain model (oracle.toeplitz) against independent
routes:

* with no defects, the model's H and S equal the direct 3D quadrature of the
  box chain (oracle.dense3d, which replicates the central cell's potential
  and truncates the stencils at the walls) -- this pins the pristine
  generators on the wall-free grid, the wall blocks, the replicated potential
  and the assembly indices;
* with one defect cell, S and the kinetic part equal the 3D quadrature
  everywhere, and H equals it on every block that touches the defect (where
  the model keeps the defect charge exactly);
* the block-circulant embedding matvec (numpy FFT) equals the dense
  block-Toeplitz product, also for L = 1 and a zero band;
* a pristine generator equals the exact block of an interior cell pair.
"""

import numpy as np
import pytest

from oracle import dense3d, toeplitz
from synth import make_instance


def _chain(L=10, ndef=0, **kw):
    nc = 8
    a = 5.0
    args = dict(name=f"box{L}", L=(L, 1, 1), n=(nc * L, 14, 14), bc="dirichlet", a=a,
                pad=(a / (2 * nc), 4.0, 4.0), n_s=2, n_p=0, exp_range=(0.8, 2.5), Z=2, R=8, seed=71)
    args.update(kw)
    return make_instance(**args)


def _blocks_close(A, B, m0, pairs, tol):
    for k, m in pairs:
        a = A[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]
        b = B[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]
        assert np.abs(a - b).max() <= tol, (k, m, np.abs(a - b).max())


@pytest.fixture(scope="module")
def pristine():
    inst = _chain()
    model = toeplitz.ChainModel(inst)
    H, S = toeplitz.model_dense(model)
    Hd, Sd, _, _ = dense3d.dense_matrices(inst)
    return inst, model, H, S, Hd, Sd


def test_model_has_interior_toeplitz_blocks(pristine):
    inst, model, H, S, _, _ = pristine
    assert model.L0 == 3
    assert list(model.X) == [0, 1, 2, 7, 8, 9]
    assert np.allclose(H, H.T, atol=0) and np.allclose(S, S.T, atol=0)
    assert np.linalg.eigvalsh(S).min() > 0


def test_pristine_model_equals_3d_quadrature(pristine):
    inst, model, H, S, Hd, Sd = pristine
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(Sd).max()
    assert np.abs(H - Hd).max() <= 1e-12 * np.abs(Hd).max()


def test_generator_equals_interior_exact_block(pristine):
    inst, model, _, _, _, _ = pristine
    h0, s0 = model.exact_block(4, 4)
    for s in range(model.L0 + 1):
        gh, gs = model.generator(s)
        bh, bs = model.exact_block(4, 4 + s)
        assert np.abs(gh - bh).max() <= 1e-13 * np.abs(h0).max()
        assert np.abs(gs - bs).max() <= 1e-14 * np.abs(s0).max()


def test_defect_blocks_equal_3d_quadrature():
    inst = _chain(L=10)
    inst.def_cells = np.asarray([5], np.int64)
    inst.def_Z = np.asarray([4.0])
    inst.def_scale = np.asarray([0.7])
    model = toeplitz.ChainModel(inst)
    assert 5 in model.X
    H, S = toeplitz.model_dense(model)
    Hd, Sd, Td, _ = dense3d.dense_matrices(inst)
    m0 = inst.m0
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(Sd).max()
    L0, L = model.L0, inst.L[0]
    touching = [(5, m) for m in range(max(0, 5 - L0), min(L, 6 + L0))]
    touching += [(m, 5) for m, _ in [(mm, 0) for mm in range(max(0, 5 - L0), min(L, 6 + L0))]]
    _blocks_close(H, Hd, m0, touching, 1e-12 * np.abs(Hd).max())
    # the model drops the defect charge on blocks that do not touch the cell:
    # there it differs from the quadrature by exactly that charge's potential
    Vd = np.zeros_like(Hd)
    inst0 = _chain(L=10)
    inst0.def_cells, inst0.def_Z, inst0.def_scale = inst.def_cells, np.asarray([2.0]), inst.def_scale
    _, _, _, V0 = dense3d.dense_matrices(inst0)        # same basis, no extra charge
    _, _, _, V1 = dense3d.dense_matrices(inst)
    Vd = V1 - V0
    far = [(3, 3), (7, 7), (3, 4)]
    for k, m in far:
        a = H[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]
        b = (Hd + Vd)[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]
        assert np.abs(a - b).max() <= 1e-12 * np.abs(Hd).max(), (k, m)
        assert np.abs(Vd[k * m0:(k + 1) * m0, m * m0:(m + 1) * m0]).max() > 1e-8


@pytest.mark.parametrize("L,L0", [(10, 3), (1, 0), (7, 0), (5, 4)])
def test_embedding_matvec_equals_dense(L, L0):
    rng = np.random.Generator(np.random.PCG64(7))
    m0 = 3
    gen = rng.standard_normal((L0 + 1, m0, m0))
    gen[0] = gen[0] + gen[0].T
    T = toeplitz.toeplitz_dense(gen, L)
    x = rng.standard_normal((L, m0, 4))
    y = toeplitz.embed_matvec(gen, L, x)
    ref = (T @ x.reshape(L * m0, 4)).reshape(L, m0, 4)
    assert np.abs(y - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    # any embedding size >= L + L0 gives the same product
    y2 = toeplitz.embed_matvec(gen, L, x, P=toeplitz.embedding_size(L, L0) * 2 + 3)
    assert np.abs(y2 - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
