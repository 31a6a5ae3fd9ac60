"""GPU parity of the three-level block-Toeplitz operator of a lattice in a box
(lhf_toeplitz3_create; Sec. 2.3 item (A), Def. 5.4, Remark 3.2) against the
CPU oracle (oracle.toeplitz3), through the C ABI.

Tolerances (derived from the arithmetic):
  * generators (FP64 Grams, same definitions, sums in another order): 1e-12
    of the largest entry of their kind;
  * FP64 matvec (complex128 three-level transform, round-off ~ eps log P
    relative to |T| |x|): 1e-12 relative to the largest entry of the product;
    FP32 matvec (complex64 transform): 2e-5 relative;
  * eigenvalues from block LOBPCG (FP64 Rayleigh-Ritz after FP64 matvecs):
    1e-8 hartree absolute against LAPACK on the oracle's dense operator.
"""

import numpy as np
import pytest
import scipy.linalg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import toeplitz3  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from synth import make_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _box(L, nc=6, **kw):
    a = 5.0
    n = tuple(nc * x if x > 1 else 14 for x in L)
    pad = tuple(a / (2 * nc) if x > 1 else 4.0 for x in L)
    args = dict(name="box3g", L=L, n=n, bc="dirichlet", a=a, pad=pad, n_s=2, n_p=1, exp_range=(0.6, 2.0), Z=2,
                R=6, seed=201)
    args.update(kw)
    return make_instance(**args)


CASES = [(5, 4, 3), (6, 5, 1), (7, 1, 1), (3, 1, 6), (2, 2, 2)]


@pytest.mark.parametrize("L", CASES, ids=lambda L: "x".join(map(str, L)))
def test_generators_match_oracle(L):
    inst = _box(L)
    gH, gS = toeplitz3.generators(inst)
    op = lhf.Toeplitz(inst, levels=3)
    L0 = toeplitz3.bands(inst)
    info = op.info
    assert info.L == L[0] * L[1] * L[2] and info.L0 == max(L0) and info.N == info.L * inst.m0
    P = toeplitz3.embedding_sizes(L, L0)
    assert info.P == P[0] * P[1] * P[2]
    GH = torch.empty(gH.shape, dtype=torch.float64, device="cuda")
    GS = torch.empty(gS.shape, dtype=torch.float64, device="cuda")
    op.lhf_toeplitz3_generators(GH, GS)
    torch.cuda.synchronize()
    assert np.abs(GH.cpu().numpy() - gH).max() <= 1e-12 * np.abs(gH).max()
    assert np.abs(GS.cpu().numpy() - gS).max() <= 1e-12 * np.abs(gS).max()
    with pytest.raises(lhf.LhfError):
        op.lhf_toeplitz_blocks(None, None, None, None, None)


@pytest.mark.parametrize("L", CASES, ids=lambda L: "x".join(map(str, L)))
@pytest.mark.parametrize("ncols,ld", [(7, 7), (3, 5)])
def test_matvec_matches_dense(L, ncols, ld):
    inst = _box(L)
    gH, gS = toeplitz3.generators(inst)
    H, S = toeplitz3.dense(gH, L), toeplitz3.dense(gS, L)
    op = lhf.Toeplitz(inst, levels=3)
    N = H.shape[0]
    x = np.random.default_rng(ncols + sum(L)).standard_normal((N, ncols))
    X = torch.zeros((N, ld), dtype=torch.float64, device="cuda")
    X[:, :ncols] = torch.from_numpy(x)
    ws = op.matvec_workspace(ncols)
    yH_ref, yS_ref = H @ x, S @ x
    for prec, tol in ((lhf.LHF_PREC_FP64, 1e-12), (lhf.LHF_PREC_MIXED, 2e-5)):
        YH = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        YS = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        op.lhf_toeplitz_matvec(prec, X[:, :ncols], YH[:, :ncols], YS[:, :ncols], ws)
        torch.cuda.synchronize()
        yh, ys = YH[:, :ncols].cpu().numpy(), YS[:, :ncols].cpu().numpy()
        assert np.abs(yh - yH_ref).max() <= tol * np.abs(yH_ref).max(), prec
        assert np.abs(ys - yS_ref).max() <= tol * np.abs(yS_ref).max(), prec
        if ld > ncols:
            assert torch.isnan(YH[:, ncols:]).all()


def test_matvec_f32_interface_refused():
    """The FP32-interface matvec takes one-level and exact box operators only."""
    op = lhf.Toeplitz(_box(CASES[0]), levels=3)
    N = op.info.N
    X = torch.zeros((N, 2), dtype=torch.float32, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(lhf.LhfError):
        op.lhf_toeplitz_matvec_f32(X, Y, None, op.matvec_workspace(2))


def test_eigs_match_lapack():
    # wide enough exponents that neighbouring cells couple: the lowest band
    # spreads over 1.3 Ha with a 0.06 Ha gap after the 12th eigenvalue (a
    # band of nearly decoupled cells would leave LOBPCG gaps of 1e-4 Ha)
    inst = _box((6, 5, 4), n_p=0, exp_range=(0.12, 0.6))
    gH, gS = toeplitz3.generators(inst)
    H, S = toeplitz3.dense(gH, inst.L), toeplitz3.dense(gS, inst.L)
    nev = 12
    ref = scipy.linalg.eigh(H, S, subset_by_index=[0, nev - 1], eigvals_only=True)
    op = lhf.Toeplitz(inst, levels=3)
    w = torch.empty(nev, dtype=torch.float64, device="cuda")
    V = torch.empty((H.shape[0], nev), dtype=torch.float64, device="cuda")
    it, res = op.lhf_toeplitz_eigs(nev, w, V, maxit=300, tol=1e-6, seed=5)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    print(f"three-level box 6x5x4: {it} iterations, residual {res:.2e}, max eig error {np.abs(got - ref).max():.2e} Ha",
          flush=True)
    assert res < 1e-6
    assert np.abs(got - ref).max() <= 1e-8, (got, ref)
    v = V.cpu().numpy()
    assert np.abs(v.T @ S @ v - np.eye(nev)).max() <= 1e-10


def test_cube_16_sampled_against_oracle_embedding():
    """A 16 x 16 x 16 box of the cube workload's cell (8 s functions,
    log-U[0.2, 8] exponents): the matvec of two columns against the oracle's
    three-level embedding product (numpy FFT), every entry."""
    inst = make_instance(name="cube16", L=(16, 16, 16), n=(128, 128, 128), bc="dirichlet", a=5.0,
                         pad=(5.0 / 16,) * 3, n_s=8, n_p=0, exp_range=(0.2, 8.0), Z=(1, 3), R=24, seed=3)
    gH, gS = toeplitz3.generators(inst)
    op = lhf.Toeplitz(inst, levels=3)
    L, m0 = inst.L, inst.m0
    x = np.random.default_rng(9).standard_normal(tuple(L) + (m0, 2))
    xt = torch.from_numpy(x.reshape(-1, 2).copy()).cuda()
    yH = torch.empty_like(xt)
    yS = torch.empty_like(xt)
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_FP64, xt, yH, yS, op.matvec_workspace(2))
    torch.cuda.synchronize()
    for y, gen in ((yH, gH), (yS, gS)):
        want = toeplitz3.embed_matvec(gen, L, x).reshape(-1, 2)
        assert np.abs(y.cpu().numpy() - want).max() <= 1e-12 * np.abs(want).max()
