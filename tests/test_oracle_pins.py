"""Pins of the CPU oracle against things other than itself.

The paper prints no eigenvalue, energy or matrix entry, so no value of the
paper can pin the oracle.  Instead each piece is checked against mathematics:
closed-form Gaussian integrals (continuum limit of the grid Galerkin matrices,
extrapolated in h), adaptive quadrature, the explicit Fourier matrices of
Lemma 3.1 / Prop. 5.1, the union-of-spectra identity, and the symmetries of
symmetric block-circulant matrices (Cor. 5.2).  A plausible mistake anywhere in
the oracle (a dropped kinetic term, a sign of the potential, a transposed
generator, a wrong FFT sign or level order, a missing periodic image, a wrong
sinc weight) fails at least one of these.
"""

import math

import numpy as np
import pytest
import scipy.integrate

import closed_form as cf
from oracle import dense3d, model, separable
from synth import make_instance, tiny_instance


# ----------------------------------------------------------------------------- helpers

def _inst_1d(n0, L0=1, bc="periodic", pad=12.0, R=2, t=(0.5, 1.0), **kw):
    """Instance whose dimension 0 is the one under test; other dims tiny."""
    inst = make_instance(name="pin", L=(L0, 1, 1), n=(n0, 6, 6), a=5.0, bc=bc,
                         pad=(pad, 3.0, 3.0), R=R, **kw)
    inst.sinc_u0 = math.log(t[0])
    inst.sinc_step = math.log(t[1] / t[0]) if R > 1 else 1.0
    return inst


# ----------------------------------------------------------------------------- the pin helpers themselves

def test_closed_form_helpers_vs_quadrature():
    for (a1, l1, A1, a2, l2, A2) in [(0.7, 0, 0.2, 1.3, 1, -0.4), (0.4, 1, 0.0, 0.9, 1, 0.7)]:
        f1 = lambda x: cf._norm(a1, l1) * (x - A1) ** l1 * math.exp(-a1 * (x - A1) ** 2)
        f2 = lambda x: cf._norm(a2, l2) * (x - A2) ** l2 * math.exp(-a2 * (x - A2) ** 2)
        ov = scipy.integrate.quad(lambda x: f1(x) * f2(x), -30, 30, epsabs=1e-15, limit=200)[0]
        assert abs(ov - cf.overlap_1d(a1, l1, A1, a2, l2, A2)) < 1e-12
        h = 1e-5
        d = lambda f, x: (f(x + h) - f(x - h)) / (2 * h)
        dd = scipy.integrate.quad(lambda x: d(f1, x) * d(f2, x), -30, 30, epsabs=1e-13, limit=200)[0]
        assert abs(dd - cf.dd_1d(a1, l1, A1, a2, l2, A2)) < 1e-7
        tg = scipy.integrate.quad(lambda x: f1(x) * f2(x) * math.exp(-0.64 * (x - 0.3) ** 2),
                                  -30, 30, epsabs=1e-15, limit=200)[0]
        assert abs(tg - cf.three_gauss_1d(a1, l1, A1, a2, l2, A2, 0.8, 0.3)) < 1e-12


# ----------------------------------------------------------------------------- potential collocation (eq. galten)

@pytest.mark.parametrize("x,h,t,A", [(0.1, 0.2, 1.0, 0.0), (3.0, 0.1, 2.0, 0.0), (-4.0, 0.3, 1.5, 0.5),
                                     (0.05, 0.1, 30.0, 0.0), (12.0, 0.5, 0.2, -1.0),
                                     # cells much narrower than the Gaussian (small sinc nodes)
                                     (5.0, 0.066, 3.7e-6, 0.0), (1.0, 0.066, 3.7e-6, 0.0),
                                     (40.0, 0.625, 2e-3, 0.3), (-7.0, 0.3, 0.05, 0.1), (0.0, 0.02, 1.0, 0.0)])
def test_cell_integral_vs_high_precision(x, h, t, A):
    """Against the erf difference evaluated with 100 significant digits."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 100
    X, Hh, T, AA = (mpmath.mpf(v) for v in (x, h, t, A))
    ref = float(mpmath.sqrt(mpmath.pi) / (2 * T) * (mpmath.erf(T * (X + Hh / 2 - AA)) - mpmath.erf(T * (X - Hh / 2 - AA))))
    got = model.cell_integral_gauss(np.array([x]), h, t, A)[0]
    assert abs(got - ref) <= 2e-14 * abs(ref), (got, ref)


def test_sinc_rule_converges_to_inverse_distance():
    inst = tiny_instance()
    inst.R = 420
    inst.sinc_u0 = math.log(1e-15)
    inst.sinc_step = 0.1
    t, w = model.sinc_rule(inst)
    rho = np.geomspace(0.05, 100.0, 60)
    approx = (w[None, :] * np.exp(-np.outer(rho * rho, t * t))).sum(1)
    assert np.max(np.abs(approx * rho - 1.0)) < 1e-11


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_config_sinc_rule_model_error(name):
    """Model error of the configs' rank-R rules (not a parity tolerance)."""
    from synth import make_config
    inst = make_config(name)
    t, w = model.sinc_rule(inst)
    gs = model.grids(inst)
    rmin = 0.5 * min(g.h for g in gs)
    rho = np.geomspace(2 * rmin, 100.0, 200)
    approx = (w[None, :] * np.exp(-np.outer(rho * rho, t * t))).sum(1)
    err = np.max(np.abs(approx * rho - 1.0))
    print(f"{name}: R={inst.R} max relative error of the sinc rule on [{2*rmin:.3g}, 100] = {err:.2e}")
    assert err < 2e-2


# ----------------------------------------------------------------------------- 1D Grams vs continuum (Prop. 2.2 factors)

def _box_grams(n0, **kw):
    inst = _inst_1d(n0, L0=1, bc="dirichlet", **kw)
    g = separable.gram_1d(inst, 0)
    return inst, g


def test_gram_1d_box_richardson_vs_closed_form():
    kw = dict(n_s=2, n_p=1, exp_range=(0.4, 2.5), seed=21)
    inst, g1 = _box_grams(499, **kw)
    _, g2 = _box_grams(999, **kw)
    _, g4 = _box_grams(1999, **kw)
    h1, h2 = g1["grid"].h, g2["grid"].h
    assert abs(h1 / h2 - 2.0) < 1e-12
    rex = lambda key, *idx: cf.richardson3(g1[key][idx], g2[key][idx], g4[key][idx])
    t, _ = model.sinc_rule(inst)
    m0 = inst.m0
    for mu in range(m0):
        for nu in range(m0):
            lm = model.angular_power(int(inst.ang[mu]), 0)
            ln = model.angular_power(int(inst.ang[nu]), 0)
            am, an = inst.alpha[mu], inst.alpha[nu]
            cm, cn = inst.centre[mu, 0], inst.centre[nu, 0]
            S = cf.overlap_1d(am, lm, cm, an, ln, cn)
            K = cf.dd_1d(am, lm, cm, an, ln, cn)
            s_ex = rex("S", 0, mu, nu)
            k_ex = rex("K", 0, mu, nu)
            assert abs(s_ex - S) < 1e-10, (mu, nu, s_ex, S)
            assert abs(k_ex - K) < 1e-9, (mu, nu, k_ex, K)
            for q in range(inst.R):
                M = cf.three_gauss_1d(am, lm, cm, an, ln, cn, t[q], inst.nuc[0, 0])
                m_ex = rex("M", q, 0, mu, nu)
                assert abs(m_ex - M) < 1e-10, (q, mu, nu, m_ex, M)


def test_gram_1d_periodic_richardson_vs_closed_form():
    """Periodic dimension: shift-k Grams equal the continuum integrals summed
    over supercell translates, with the potential an infinite a-periodic sum."""
    L0 = 6
    kw = dict(n_s=2, n_p=1, exp_range=(0.4, 2.5), seed=22)
    inst1 = _inst_1d(L0 * 100, L0=L0, **kw)
    g1 = separable.gram_1d(inst1, 0)
    g2 = separable.gram_1d(_inst_1d(L0 * 200, L0=L0, **kw), 0)
    g4 = separable.gram_1d(_inst_1d(L0 * 400, L0=L0, **kw), 0)
    rex = lambda key, *idx: cf.richardson3(g1[key][idx], g2[key][idx], g4[key][idx])
    a, P = inst1.a, L0 * inst1.a
    Xc = lambda k: (k + 0.5) * a
    t, _ = model.sinc_rule(inst1)
    for k in range(L0):
        for mu in range(inst1.m0):
            for nu in range(inst1.m0):
                lm = model.angular_power(int(inst1.ang[mu]), 0)
                ln = model.angular_power(int(inst1.ang[nu]), 0)
                am, an = inst1.alpha[mu], inst1.alpha[nu]
                cm, cn = Xc(k) + inst1.centre[mu, 0], Xc(0) + inst1.centre[nu, 0]
                S = sum(cf.overlap_1d(am, lm, cm + s * P, an, ln, cn) for s in range(-3, 4))
                K = sum(cf.dd_1d(am, lm, cm + s * P, an, ln, cn) for s in range(-3, 4))
                assert abs(rex("S", k, mu, nu) - S) < 1e-10
                assert abs(rex("K", k, mu, nu) - K) < 1e-9
                for q in range(inst1.R):
                    M = sum(cf.three_gauss_1d(am, lm, cm + s * P, an, ln, cn, t[q],
                                              Xc(m) + inst1.nuc[0, 0])
                            for s in range(-3, 4) for m in range(-12, 13))
                    got = rex("M", q, k, mu, nu)
                    assert abs(got - M) < 1e-10, (k, q, mu, nu, got, M)


# ----------------------------------------------------------------------------- 3D single cell vs continuum (eq. Core_Ham)

@pytest.mark.slow
def test_single_cell_3d_dense_vs_closed_form():
    """Dense 3D quadrature of one box cell (s and p functions) converges to the
    continuum S, T = 1/2 int grad g grad g, V = sum_q Z w_q int g g exp(-t_q^2 r^2),
    H = T - V."""
    def inst_at(n):
        inst = make_instance(name="cell", L=(1, 1, 1), n=(n, n, n), a=5.0, bc="dirichlet",
                             pad=(6.0, 6.0, 6.0), n_s=1, n_p=1, exp_range=(0.5, 1.5), Z=2,
                             R=2, seed=31)
        inst.sinc_u0, inst.sinc_step = math.log(0.5), math.log(2.0)
        inst.nuc[0] = [0.2, -0.1, 0.15]
        return inst
    i1, i2 = inst_at(84), inst_at(169)
    H1, S1, T1, V1 = dense3d.dense_matrices(i1)
    H2, S2, T2, V2 = dense3d.dense_matrices(i2)
    t, w = model.sinc_rule(i1)
    m0 = i1.m0
    for mu in range(m0):
        for nu in range(m0):
            s = []; d = []; pot = []
            for ell in range(3):
                lm = model.angular_power(int(i1.ang[mu]), ell)
                ln = model.angular_power(int(i1.ang[nu]), ell)
                args = (i1.alpha[mu], lm, i1.centre[mu, ell], i1.alpha[nu], ln, i1.centre[nu, ell])
                s.append(cf.overlap_1d(*args)); d.append(cf.dd_1d(*args))
                pot.append([cf.three_gauss_1d(*args, t[q], i1.nuc[0, ell]) for q in range(i1.R)])
            S = s[0] * s[1] * s[2]
            T = 0.5 * (d[0] * s[1] * s[2] + s[0] * d[1] * s[2] + s[0] * s[1] * d[2])
            V = sum(i1.Z[0] * w[q] * pot[0][q] * pot[1][q] * pot[2][q] for q in range(i1.R))
            rex = lambda A, B: cf.richardson(A[mu, nu], B[mu, nu])
            # two-level extrapolation leaves an O(h^4) residual of ~1e-4 here;
            # a dropped term, a factor or a sign error is O(1)
            assert abs(rex(S1, S2) - S) < 1e-3
            assert abs(rex(T1, T2) - T) < 1e-3
            assert abs(rex(V1, V2) - V) < 1e-3
            assert abs(rex(H1, H2) - (T - V)) < 2e-3
            assert abs(H2[mu, nu] - (T - V)) < 3e-2


# ----------------------------------------------------------------------------- separable route vs the plain definition

CASES = [
    dict(L=(4, 1, 1), n=(32, 20, 20), n_s=2, n_p=1, seed=41),      # even chain, s + p
    dict(L=(5, 1, 1), n=(40, 18, 18), n_s=3, n_p=0, seed=42),      # odd chain
    dict(L=(3, 2, 1), n=(24, 16, 14), n_s=2, n_p=1, seed=43),      # 2D sheet
    dict(L=(2, 3, 2), n=(16, 24, 16), n_s=2, n_p=0, seed=44),      # 3D
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "L" + "x".join(map(str, c["L"])))
def test_dense_equals_separable_generators(case):
    inst = tiny_instance(R=5, **case)
    H, S, T, V = dense3d.dense_matrices(inst)
    Hg, Sg = separable.generator_stacks(inst)
    L, m0 = inst.L, inst.m0
    scale_h, scale_s = np.abs(H).max(), np.abs(S).max()
    cells = [(a, b, c) for a in range(L[0]) for b in range(L[1]) for c in range(L[2])]
    for k in cells:
        for m in cells:
            d = tuple((k[i] - m[i]) % L[i] for i in range(3))
            bk = dense3d.cell_index(L, k); bm = dense3d.cell_index(L, m)
            assert np.abs(dense3d.block(H, m0, bk, bm) - Hg[d]).max() < 1e-13 * scale_h
            assert np.abs(dense3d.block(S, m0, bk, bm) - Sg[d]).max() < 1e-13 * scale_s


@pytest.mark.parametrize("case", CASES + [dict(L=(6, 4, 3), n=(48, 32, 24), n_s=2, n_p=1, seed=45)],
                         ids=lambda c: "L" + "x".join(map(str, c["L"])))
def test_fourier_blocks_from_transformed_grams(case):
    """Theorem 3.3 / Remark 3.5: the Fourier blocks are the same Hadamard
    combination of the per-dimension 1D DFTs of the Grams,
      Sbar_j = S^1 o S^2 o S^3,  Hbar_j = 1/2 (K^1 S^2 S^3 + S^1 K^2 S^3 + S^1 S^2 K^3) - sum_t c_t M^1_t M^2_t M^3_t,
    as the 3D DFT of the generator stacks (a lost kinetic term, a transposed
    factor or a wrong sign fails)."""
    inst = tiny_instance(R=5, **case)
    grams = [separable.gram_1d(inst, ell) for ell in range(3)]
    Hg, Sg = separable.generator_stacks(inst, grams)
    Hb, Sb = separable.fourier_blocks(Hg), separable.fourier_blocks(Sg)
    c = separable.term_coefficients(inst)
    hat = [{k: np.fft.fft(g[k], axis=-3) for k in ("S", "K", "M")} for g in grams]
    S1, S2, S3 = (h["S"] for h in hat)
    K1, K2, K3 = (h["K"] for h in hat)
    Sb_sep = np.einsum("aij,bij,cij->abcij", S1, S2, S3)
    Hb_sep = 0.5 * (np.einsum("aij,bij,cij->abcij", K1, S2, S3) + np.einsum("aij,bij,cij->abcij", S1, K2, S3)
                    + np.einsum("aij,bij,cij->abcij", S1, S2, K3))
    Hb_sep -= np.einsum("t,taij,tbij,tcij->abcij", c, hat[0]["M"], hat[1]["M"], hat[2]["M"])
    assert np.abs(Sb_sep - Sb).max() <= 1e-13 * np.abs(Sb).max()
    assert np.abs(Hb_sep - Hb).max() <= 1e-13 * np.abs(Hb).max()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "L" + "x".join(map(str, c["L"])))
def test_explicit_fourier_matrices_block_diagonalise(case):
    """(F_L x I) A (F_L^* x I) = bdiag(Abar_j), F_L = F_L1 x F_L2 x F_L3 unitary
    with omega = exp(-2 pi i / L) (Lemma 3.1, Prop. 5.1) on the dense matrix."""
    inst = tiny_instance(R=5, **case)
    H, S, _, _ = dense3d.dense_matrices(inst)
    res = separable.solve(inst)
    m0 = inst.m0

    def F(L):
        j = np.arange(L)
        return np.exp(-2j * np.pi * np.outer(j, j) / L) / math.sqrt(L)
    FL = np.kron(np.kron(F(inst.L[0]), F(inst.L[1])), F(inst.L[2]))
    big = np.kron(FL, np.eye(m0))
    for Mat, bars in ((H, res["H_bar"]), (S, res["S_bar"])):
        D = big @ Mat @ big.conj().T
        nb = inst.ncells
        flat = bars.reshape(nb, m0, m0)
        for i in range(nb):
            for j in range(nb):
                blk = D[i * m0:(i + 1) * m0, j * m0:(j + 1) * m0]
                if i == j:
                    assert np.abs(blk - flat[i]).max() < 1e-12 * np.abs(Mat).max()
                else:
                    assert np.abs(blk).max() < 1e-12 * np.abs(Mat).max()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "L" + "x".join(map(str, c["L"])))
def test_union_of_block_spectra_equals_dense_spectrum(case):
    inst = tiny_instance(R=5, **case)
    H, S, _, _ = dense3d.dense_matrices(inst)
    ev = dense3d.dense_eigvals(H, S)
    res = separable.solve(inst)
    eb = np.sort(res["eig"].ravel())
    assert np.abs(ev - eb).max() < 1e-10 * max(1.0, np.abs(ev).max())
    e2 = separable.block_eigvals_scipy(res["H_bar"], res["S_bar"])
    assert np.abs(np.sort(e2.ravel()) - eb).max() < 1e-11 * max(1.0, np.abs(ev).max())


def test_one_function_per_cell_is_scalar_circulant():
    """m0 = 1: the Fourier blocks are the DFT of the first column, and the
    generalized spectrum is {Hbar_j / Sbar_j} (Appendix, eq. circDiag)."""
    inst = tiny_instance(L=(6, 1, 1), n=(48, 16, 16), n_s=1, R=4, seed=51)
    H, S, _, _ = dense3d.dense_matrices(inst)
    col_h, col_s = H[:, 0], S[:, 0]
    dft = lambda c: np.array([sum(c[k] * np.exp(-2j * np.pi * j * k / len(c)) for k in range(len(c)))
                              for j in range(len(c))])
    res = separable.solve(inst)
    assert np.abs(res["H_bar"].ravel() - dft(col_h)).max() < 1e-12 * np.abs(col_h).max()
    lam = np.sort((dft(col_h) / dft(col_s)).real)
    assert np.abs(lam - dense3d.dense_eigvals(H, S)).max() < 1e-11 * np.abs(lam).max()


# ----------------------------------------------------------------------------- symmetric block-circulant structure (Cor. 5.2)

@pytest.mark.parametrize("L", [(6, 1, 1), (5, 1, 1), (4, 3, 2)])
def test_generator_symmetry_and_hermitian_blocks(L):
    inst = tiny_instance(L=L, n=tuple(8 * x if x > 1 else 12 for x in L), n_s=2, n_p=1, R=4, seed=61)
    res = separable.solve(inst)
    for stack in (res["H_gen"], res["S_gen"]):
        neg = stack[(-np.arange(L[0])) % L[0]][:, (-np.arange(L[1])) % L[1]][:, :, (-np.arange(L[2])) % L[2]]
        assert np.abs(neg - np.swapaxes(stack, -1, -2)).max() < 1e-14 * np.abs(stack).max()
        if L[0] % 2 == 0:
            half = stack[L[0] // 2, 0, 0]
            assert np.abs(half - half.T).max() < 1e-14 * np.abs(stack).max()
    for bars in (res["H_bar"], res["S_bar"]):
        assert np.abs(bars - np.conj(np.swapaxes(bars, -1, -2))).max() < 1e-13 * np.abs(bars).max()
        negj = bars[(-np.arange(L[0])) % L[0]][:, (-np.arange(L[1])) % L[1]][:, :, (-np.arange(L[2])) % L[2]]
        assert np.abs(negj - np.conj(bars)).max() < 1e-13 * np.abs(bars).max()


@pytest.mark.slow
def test_c1_full_size_dense_equals_separable():
    """The 8-cell chain at full size (N = 32 on the 128^3 grid): the plain
    definition (dense 3D quadrature, image-by-image potential, dense LAPACK
    solve) against the separable route: every block of H and S, and the
    spectrum against the union of the Fourier-block spectra (Prop. 5.1)."""
    from synth import make_config
    inst = make_config("c1")
    H, S, _, _ = dense3d.dense_matrices(inst)
    res = separable.solve(inst)
    Hd = separable.block_circulant_dense(res["H_gen"])
    Sd = separable.block_circulant_dense(res["S_gen"])
    assert np.abs(H - Hd).max() <= 1e-13 * np.abs(H).max()
    assert np.abs(S - Sd).max() <= 1e-13 * np.abs(S).max()
    ev = dense3d.dense_eigvals(H, S)
    eb = np.sort(res["eig"].ravel())
    assert np.abs(ev - eb).max() <= 1e-12 * max(1.0, np.abs(ev).max())


@pytest.mark.parametrize("M0", [2, 3])
def test_dense_equals_separable_several_nuclei(M0):
    """Several off-centre nuclei per cell (sum over nuclei of the rank-R
    potential, each with its own lattice window): the separable generators
    equal the dense 3D quadrature, which sums every nucleus image by image."""
    inst = tiny_instance(L=(3, 2, 1), n=(24, 16, 14), n_s=2, n_p=1, R=5, seed=47)
    inst.Z = np.array([1.0, 2.0, 0.5][:M0])
    inst.nuc = np.array([[0.4, -0.3, 0.2], [-2.1, 1.3, -0.6], [1.7, 2.2, 0.9]][:M0])
    H, S, _, _ = dense3d.dense_matrices(inst)
    Hg, _ = separable.generator_stacks(inst)
    Hd = separable.block_circulant_dense(Hg)
    assert np.abs(H - Hd).max() < 1e-13 * np.abs(H).max()
    # the extra nuclei matter: dropping all but the first changes H at O(1)
    one = tiny_instance(L=(3, 2, 1), n=(24, 16, 14), n_s=2, n_p=1, R=5, seed=47)
    one.Z, one.nuc = inst.Z[:1].copy(), inst.nuc[:1].copy()
    H1 = separable.block_circulant_dense(separable.generator_stacks(one)[0])
    assert np.abs(H1 - Hd).max() > 1e-2 * np.abs(H).max()
