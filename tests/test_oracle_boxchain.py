"""Pins of the exact box-case operator of a Dirichlet chain (oracle.boxchain;
Sec. 2.3, case (B), eq. EwaldSumE) against independent routes:

* every block equals the direct 3D quadrature with the finite lattice's own
  potential summed image by image in 3D (oracle.dense3d, finite=True), with
  and without a defect cell, odd and even L -- this pins the 1D Gram
  contraction, the finite-lattice potential factors, the defect charges and
  scales, and the assembly indices;
* the chain factor of the finite-lattice potential equals the sum over the
  L cells of the collocation integrals evaluated at 60 digits;
* a chain whose cell is mirror symmetric gives a mirror-symmetric operator,
  H(k, m) = H(L-1-k, L-1-m) (a one-sided or shifted lattice sum breaks it);
* blocks beyond the band L0 vanish (reading B2);
* the box operator differs from the perturbed block-Toeplitz model at O(1)
  in the wall blocks (item (B)) and by a smaller, non-local amount in the
  interior (item (A)), which the model neglects.
"""

import math

import numpy as np
import pytest

from oracle import boxchain, dense3d, model, toeplitz
from synth import make_instance


def _chain(L=6, ndef=0, **kw):
    nc = 8
    a = 5.0
    args = dict(name=f"boxB{L}", L=(L, 1, 1), n=(nc * L, 14, 14), bc="dirichlet", a=a,
                pad=(a / (2 * nc), 4.0, 4.0), n_s=2, n_p=1, exp_range=(0.8, 2.5), Z=2, R=8, seed=171,
                ndefect=ndef, defect_seed=172)
    args.update(kw)
    return make_instance(**args)


@pytest.mark.parametrize("L,ndef", [(5, 0), (6, 0), (6, 1), (7, 2)])
def test_box_operator_equals_3d_quadrature(L, ndef):
    inst = _chain(L, ndef)
    box = boxchain.BoxChain(inst)
    H, S = box.dense(full=True)
    Hd, Sd, _, _ = dense3d.dense_matrices(inst, finite=True)
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(Sd).max()
    assert np.abs(H - Hd).max() <= 1e-12 * np.abs(Hd).max(), np.abs(H - Hd).max()


@pytest.mark.parametrize("ndef", [0, 2])
def test_finite_lattice_potential_vs_brute_force(ndef):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    inst = _chain(5, ndef, R=3)
    g = model.grids(inst)[0]
    P = boxchain.finite_lattice_potential(inst, g)
    t, w = model.sinc_rule(inst)
    a, L = inst.a, inst.L[0]
    zc = {int(c): float(z) for c, z in zip(inst.def_cells, inst.def_Z)}
    for q in range(inst.R):
        ref = []
        for x in g.x:
            acc = mpmath.mpf(0)
            for c in range(L):
                A = -0.5 * L * a + (c + 0.5) * a + float(inst.nuc[0, 0])
                X, H, T, AA = (mpmath.mpf(v) for v in (x, g.h, t[q], A))
                phi = mpmath.sqrt(mpmath.pi) / (2 * T) * (mpmath.erf(T * (X + H / 2 - AA)) -
                                                          mpmath.erf(T * (X - H / 2 - AA)))
                acc += zc.get(c, float(inst.Z[0])) * phi
            ref.append(float(acc * w[q]))
        ref = np.array(ref)
        assert np.abs(P[q] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_mirror_symmetric_chain_gives_mirror_symmetric_operator():
    inst = _chain(7, 0, n_p=0, jitter=0.0)
    box = boxchain.BoxChain(inst)
    H, S = box.dense()
    L, m0 = inst.L[0], inst.m0
    J = np.zeros((L * m0, L * m0))
    for k in range(L):
        J[k * m0:(k + 1) * m0, (L - 1 - k) * m0:(L - k) * m0] = np.eye(m0)
    assert np.abs(J @ H @ J - H).max() <= 1e-12 * np.abs(H).max()
    assert np.abs(J @ S @ J - S).max() <= 1e-13 * np.abs(S).max()


def test_blocks_beyond_band_vanish():
    inst = _chain(9, 0, exp_range=(1.2, 2.5))
    box = boxchain.BoxChain(inst)
    assert box.L0 < 8
    scale = max(np.abs(h).max() for h, _ in box.blocks().values())
    for (k, m), (bh, bs) in box.blocks(full=True).items():
        if m - k > box.L0:
            assert np.abs(bh).max() <= 1e-20 * scale and np.abs(bs).max() <= 1e-20 * scale


def test_box_differs_from_toeplitz_model_as_items_A_and_B():
    inst = _chain(12, 0, exp_range=(1.2, 2.5))
    box = boxchain.BoxChain(inst)
    Hb, Sb = box.dense()
    cm = toeplitz.ChainModel(inst)
    Hm, Sm = toeplitz.model_dense(cm)
    m0, L0 = inst.m0, box.L0
    # S does not see the potential: identical (the model keeps the wall blocks exact)
    assert np.abs(Hb - Hm).max() > 1e-3
    assert np.abs(Sb - Sm).max() <= 1e-13 * np.abs(Sb).max()
    diff = [np.abs(Hb[k * m0:(k + 1) * m0, k * m0:(k + 1) * m0] - Hm[k * m0:(k + 1) * m0, k * m0:(k + 1) * m0]).max()
            for k in range(inst.L[0])]
    interior = max(diff[L0:inst.L[0] - L0])
    assert 0 < interior < max(diff[0], diff[-1])


def _shifted_sum(inst, g):
    """Lattice sum over cells 1..L instead of 0..L-1 (a plausible off-by-one)."""
    P = _ORIG(inst, g)
    t, w = model.sinc_rule(inst)
    L, a = inst.L[0], inst.a
    for q in range(inst.R):
        for c, sign in ((0, -1.0), (L, 1.0)):
            A = -0.5 * L * a + (c + 0.5) * a + float(inst.nuc[0, 0])
            P[q] += sign * float(inst.Z[0]) * w[q] * model.cell_integral_gauss(g.x, g.h, t[q], A)
    return P


def _no_defect_charge(inst, g):
    saved = inst.def_Z.copy()
    inst.def_Z[:] = inst.Z[0]
    try:
        return _ORIG(inst, g)
    finally:
        inst.def_Z[:] = saved


_ORIG = boxchain.finite_lattice_potential


@pytest.mark.parametrize("bad,ndef", [(_shifted_sum, 0), (_no_defect_charge, 2)], ids=["shifted", "defect-charge"])
def test_planted_box_mistakes_are_caught(monkeypatch, bad, ndef):
    monkeypatch.setattr(boxchain, "finite_lattice_potential", bad)
    with pytest.raises(AssertionError):
        test_box_operator_equals_3d_quadrature(6, ndef)
