"""GPU parity of the Dirichlet-chain operator against the CPU oracle (through
the C ABI).

Tolerances (derived from the arithmetic):
  * blocks (FP64 Grams, same definitions, sums in another order): 1e-12 of
    the largest entry of the pristine diagonal block;
  * FP64 matvec (complex128 embedding transform, round-off ~ eps log P
    relative to |T| |x|): 1e-12 of max|H| max|x| N-scaled norm; the FP32
    path (complex64 transform): 2e-5 relative;
  * eigenvalues from block LOBPCG (FP64 Rayleigh-Ritz after FP64 matvecs):
    1e-8 hartree absolute against LAPACK on the oracle's dense model.
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import toeplitz  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from synth import make_config, make_instance  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _small():
    inst = make_instance(name="box14", L=(14, 1, 1), n=(112, 14, 14), bc="dirichlet", pad=(5.0 / 16, 4.0, 4.0),
                         n_s=2, n_p=1, exp_range=(0.8, 2.5), Z=2, R=8, seed=81)
    inst.def_cells = np.asarray([1, 6, 7], np.int64)     # near a wall, and two neighbours
    inst.def_Z = np.asarray([3.0, 1.0, 4.0])
    inst.def_scale = np.asarray([0.8, 1.3, 0.9])
    return inst


@pytest.fixture(scope="module")
def small():
    inst = _small()
    model = toeplitz.ChainModel(inst)
    gens = model.generators()
    cross = model.cross_blocks()
    H, S = toeplitz.model_dense(model, gens, cross)
    return inst, model, gens, cross, H, S


def test_blocks_match_oracle(small):
    inst, model, (gH, gS), cross, _, _ = small
    op = lhf.Toeplitz(inst)
    info = op.info
    m0, L0 = inst.m0, model.L0
    assert (info.L0, info.m0, info.N, info.ncross) == (L0, m0, inst.L[0] * m0, len(model.X))
    assert info.ncross_blocks == len(cross)
    dev = "cuda"
    GH = torch.empty((L0 + 1, m0, m0), dtype=torch.float64, device=dev)
    GS = torch.empty_like(GH)
    km = torch.empty((len(cross), 2), dtype=torch.int32, device=dev)
    CH = torch.empty((len(cross), m0, m0), dtype=torch.float64, device=dev)
    CS = torch.empty_like(CH)
    op.lhf_toeplitz_blocks(GH, GS, km, CH, CS)
    torch.cuda.synchronize()
    scale_h, scale_s = np.abs(gH[0]).max(), np.abs(gS[0]).max()
    assert np.abs(GH.cpu().numpy() - gH).max() <= 1e-12 * scale_h
    assert np.abs(GS.cpu().numpy() - gS).max() <= 1e-12 * scale_s
    keys = sorted(cross)
    assert [tuple(r) for r in km.cpu().numpy().tolist()] == keys
    ch, cs = CH.cpu().numpy(), CS.cpu().numpy()
    for i, key in enumerate(keys):
        bh, bs = cross[key]
        assert np.abs(ch[i] - bh).max() <= 1e-12 * scale_h, key
        assert np.abs(cs[i] - bs).max() <= 1e-12 * scale_s, key


@pytest.mark.parametrize("ncols,ld", [(7, 7), (5, 9), (1, 1)])
def test_matvec_matches_dense(small, ncols, ld):
    inst, model, _, _, H, S = small
    op = lhf.Toeplitz(inst)
    N = H.shape[0]
    rng = np.random.Generator(np.random.PCG64(ncols))
    x = rng.standard_normal((N, ncols))
    X = torch.zeros((N, ld), dtype=torch.float64, device="cuda")
    X[:, :ncols] = torch.from_numpy(x)
    xs = X[:, :ncols]
    ws = op.matvec_workspace(ncols)
    yH_ref, yS_ref = H @ x, S @ x
    for prec, tol in ((lhf.LHF_PREC_FP64, 1e-12), (lhf.LHF_PREC_MIXED, 2e-5)):
        YH = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        YS = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        op.lhf_toeplitz_matvec(prec, xs, YH[:, :ncols], YS[:, :ncols], ws)
        torch.cuda.synchronize()
        yh, ys = YH[:, :ncols].cpu().numpy(), YS[:, :ncols].cpu().numpy()
        assert np.abs(yh - yH_ref).max() <= tol * np.abs(yH_ref).max()
        assert np.abs(ys - yS_ref).max() <= tol * np.abs(yS_ref).max()
        if ld > ncols:   # columns beyond ncols are left alone
            assert torch.isnan(YH[:, ncols:]).all()
    # H only
    YH = torch.empty((N, ld), dtype=torch.float64, device="cuda")
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_FP64, xs, YH[:, :ncols], None, ws)
    torch.cuda.synchronize()
    assert np.abs(YH[:, :ncols].cpu().numpy() - yH_ref).max() <= 1e-12 * np.abs(yH_ref).max()


@pytest.mark.parametrize("ncols,ld", [(7, 7), (5, 9)])
def test_matvec_f32_interface_matches_dense(small, ncols, ld):
    """lhf_toeplitz_matvec_f32: FP32 x and y, the FP32 route's arithmetic.
    Against the dense model on the FP32-rounded input within the FP32 route's
    2e-5, and against the FP64-interface FP32 route on the same input within
    FP32 output rounding (1e-6 relative)."""
    inst, model, _, _, H, S = small
    op = lhf.Toeplitz(inst)
    N = H.shape[0]
    rng = np.random.Generator(np.random.PCG64(100 + ncols))
    x32 = rng.standard_normal((N, ncols)).astype(np.float32)
    x = x32.astype(np.float64)
    X = torch.zeros((N, ld), dtype=torch.float32, device="cuda")
    X[:, :ncols] = torch.from_numpy(x32)
    ws = op.matvec_workspace(ncols)
    YH = torch.full((N, ld), float("nan"), dtype=torch.float32, device="cuda")
    YS = torch.full((N, ld), float("nan"), dtype=torch.float32, device="cuda")
    op.lhf_toeplitz_matvec_f32(X[:, :ncols], YH[:, :ncols], YS[:, :ncols], ws)
    X64 = torch.from_numpy(x).cuda()
    RH = torch.empty((N, ncols), dtype=torch.float64, device="cuda")
    RS = torch.empty_like(RH)
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_MIXED, X64, RH, RS, ws)
    torch.cuda.synchronize()
    yH_ref, yS_ref = H @ x, S @ x
    yh, ys = YH[:, :ncols].double().cpu().numpy(), YS[:, :ncols].double().cpu().numpy()
    assert np.abs(yh - yH_ref).max() <= 2e-5 * np.abs(yH_ref).max()
    assert np.abs(ys - yS_ref).max() <= 2e-5 * np.abs(yS_ref).max()
    assert np.abs(yh - RH.cpu().numpy()).max() <= 1e-6 * np.abs(yH_ref).max()
    assert np.abs(ys - RS.cpu().numpy()).max() <= 1e-6 * np.abs(yS_ref).max()
    if ld > ncols:
        assert torch.isnan(YH[:, ncols:]).all() and torch.isnan(YS[:, ncols:]).all()
    # H only (x and y share the leading dimension ld)
    YH2 = torch.empty((N, ld), dtype=torch.float32, device="cuda")
    op.lhf_toeplitz_matvec_f32(X[:, :ncols], YH2[:, :ncols], None, ws)
    torch.cuda.synchronize()
    assert torch.equal(YH2[:, :ncols], YH[:, :ncols])


def test_eigs_small_matches_lapack(small):
    inst, model, _, _, H, S = small
    op = lhf.Toeplitz(inst)
    nev = 6
    ref, _ = toeplitz.lowest_eigenpairs(H, S, nev)
    w = torch.empty(nev, dtype=torch.float64, device="cuda")
    V = torch.empty((H.shape[0], nev), dtype=torch.float64, device="cuda")
    it, res = op.lhf_toeplitz_eigs(nev, w, V, maxit=200, tol=1e-6, seed=3)
    torch.cuda.synchronize()
    assert it < 200 and res < 1e-6
    got = w.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-8, (got, ref)
    v = V.cpu().numpy()
    assert np.abs(v.T @ S @ v - np.eye(nev)).max() <= 1e-10
    r = H @ v - (S @ v) * got[None, :]
    assert np.abs(r).max() <= 1e-5


def test_c5_lowest32_and_sampled_rows():
    """Config c5 at full size: the 32 lowest eigenvalues against the stored
    oracle values, and sampled block rows of the matvec against the oracle's
    blocks (a wall row, a defect row, an interior row)."""
    inst = make_config("c5")
    op = lhf.Toeplitz(inst)
    print(inst.summary(), "L0", op.info.L0, "X", op.info.ncross, "P", op.info.P, flush=True)
    gold = np.loadtxt(os.path.join(HERE, "golden", "c5_lowest32.txt"))
    assert op.info.L0 == 9 and op.info.ncross == 44
    w = torch.empty(32, dtype=torch.float64, device="cuda")
    it, res = op.lhf_toeplitz_eigs(32, w, None, maxit=150, tol=1e-5, seed=1)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    err = np.abs(got - gold).max()
    print(f"c5 LOBPCG: {it} iterations, residual {res:.2e}, max eig error {err:.2e} Ha", flush=True)
    assert err <= 1e-8
    # sampled rows
    model = toeplitz.ChainModel(inst)
    gH, gS = model.generators()
    L, m0, L0 = inst.L[0], inst.m0, model.L0
    X = set(int(c) for c in model.X)
    interior = next(k for k in range(L0, L - L0) if all(abs(k - c) > L0 for c in X))
    rows = [0, int(inst.def_cells[0]), interior]
    N = L * m0
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.standard_normal((N, 3))
    xt = torch.from_numpy(x).cuda()
    yH = torch.empty_like(xt)
    yS = torch.empty_like(xt)
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_FP64, xt, yH, yS, op.matvec_workspace(3))
    torch.cuda.synchronize()
    yh, ys = yH.cpu().numpy(), yS.cpu().numpy()
    for k in rows:
        rh = np.zeros((m0, 3))
        rs = np.zeros((m0, 3))
        for m in range(max(0, k - L0), min(L, k + L0 + 1)):
            if k in X or m in X:
                a, b = min(k, m), max(k, m)
                bh, bs = model.exact_block(a, b)
                if k > m:
                    bh, bs = bh.T, bs.T
            else:
                bh, bs = (gH[m - k], gS[m - k]) if m >= k else (gH[k - m].T, gS[k - m].T)
            rh += bh @ x[m * m0:(m + 1) * m0]
            rs += bs @ x[m * m0:(m + 1) * m0]
        sl = slice(k * m0, (k + 1) * m0)
        assert np.abs(yh[sl] - rh).max() <= 1e-11 * np.abs(rh).max(), k
        assert np.abs(ys[sl] - rs).max() <= 1e-11 * np.abs(rs).max(), k
