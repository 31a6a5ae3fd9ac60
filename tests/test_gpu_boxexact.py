"""GPU parity of the exact box operator of a Dirichlet chain (Sec. 2.3, case
(B); lhf_box_exact_create) against the CPU oracle (oracle.boxchain), through
the C ABI.

Tolerances (derived from the arithmetic, as for the block-Toeplitz model):
  * blocks (FP64 Grams, same definitions, sums in another order): 1e-12 of
    the largest entry of their kind;
  * block-sparse matvec (FP64 products of the blocks, in either precision
    argument): 1e-12 relative to the largest entry of the product;
  * eigenvalues from block LOBPCG (FP64 Rayleigh-Ritz after FP64 matvecs):
    1e-8 hartree absolute against LAPACK on the oracle's dense operator.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import boxchain, toeplitz  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from synth import make_config, make_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _small():
    inst = make_instance(name="boxB14", L=(14, 1, 1), n=(112, 14, 14), bc="dirichlet", pad=(5.0 / 16, 4.0, 4.0),
                         n_s=2, n_p=1, exp_range=(0.8, 2.5), Z=2, R=8, seed=181)
    inst.def_cells = np.asarray([0, 6, 7], np.int64)     # at a wall, and two neighbours
    inst.def_Z = np.asarray([3.0, 1.0, 4.0])
    inst.def_scale = np.asarray([0.8, 1.3, 0.9])
    return inst


@pytest.fixture(scope="module")
def small():
    inst = _small()
    box = boxchain.BoxChain(inst)
    blocks = box.blocks()
    H, S = box.dense()
    return inst, box, blocks, H, S


def test_exact_blocks_match_oracle(small):
    inst, box, blocks, _, _ = small
    op = lhf.Toeplitz(inst, exact=True)
    info = op.info
    m0, L = inst.m0, inst.L[0]
    assert (info.L0, info.m0, info.N, info.ncross) == (box.L0, m0, L * m0, L)
    assert info.ncross_blocks == len(blocks)
    km = torch.empty((len(blocks), 2), dtype=torch.int32, device="cuda")
    CH = torch.empty((len(blocks), m0, m0), dtype=torch.float64, device="cuda")
    CS = torch.empty_like(CH)
    op.lhf_toeplitz_blocks(None, None, km, CH, CS)
    torch.cuda.synchronize()
    keys = sorted(blocks)
    assert [tuple(r) for r in km.cpu().numpy().tolist()] == keys
    ch, cs = CH.cpu().numpy(), CS.cpu().numpy()
    scale_h = max(np.abs(b[0]).max() for b in blocks.values())
    scale_s = max(np.abs(b[1]).max() for b in blocks.values())
    for i, key in enumerate(keys):
        bh, bs = blocks[key]
        assert np.abs(ch[i] - bh).max() <= 1e-12 * scale_h, key
        assert np.abs(cs[i] - bs).max() <= 1e-12 * scale_s, key


@pytest.mark.parametrize("ncols,ld", [(7, 7), (5, 9), (1, 1), (40, 41)])
def test_exact_matvec_matches_dense(small, ncols, ld):
    inst, _, _, H, S = small
    op = lhf.Toeplitz(inst, exact=True)
    N = H.shape[0]
    rng = np.random.Generator(np.random.PCG64(ncols + 100))
    x = rng.standard_normal((N, ncols))
    X = torch.zeros((N, ld), dtype=torch.float64, device="cuda")
    X[:, :ncols] = torch.from_numpy(x)
    xs = X[:, :ncols]
    ws = op.matvec_workspace(ncols)
    yH_ref, yS_ref = H @ x, S @ x
    for prec in (lhf.LHF_PREC_FP64, lhf.LHF_PREC_MIXED):
        YH = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        YS = torch.full((N, ld), float("nan"), dtype=torch.float64, device="cuda")
        op.lhf_toeplitz_matvec(prec, xs, YH[:, :ncols], YS[:, :ncols], ws)
        torch.cuda.synchronize()
        yh, ys = YH[:, :ncols].cpu().numpy(), YS[:, :ncols].cpu().numpy()
        assert np.abs(yh - yH_ref).max() <= 1e-12 * np.abs(yH_ref).max()
        assert np.abs(ys - yS_ref).max() <= 1e-12 * np.abs(yS_ref).max()
        if ld > ncols:
            assert torch.isnan(YH[:, ncols:]).all()
    YH = torch.empty((N, ld), dtype=torch.float64, device="cuda")
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_FP64, xs, YH[:, :ncols], None, ws)
    torch.cuda.synchronize()
    assert np.abs(YH[:, :ncols].cpu().numpy() - yH_ref).max() <= 1e-12 * np.abs(yH_ref).max()


@pytest.mark.parametrize("ncols,ld", [(7, 7), (40, 41)])
def test_exact_matvec_f32_interface(small, ncols, ld):
    """lhf_toeplitz_matvec_f32 on the exact box operator (block-sparse
    product, FP64 accumulation, FP32 input and output): against the dense
    operator on the FP32-rounded input within FP32 output rounding."""
    inst, _, _, H, S = small
    op = lhf.Toeplitz(inst, exact=True)
    N = H.shape[0]
    rng = np.random.Generator(np.random.PCG64(ncols + 300))
    x32 = rng.standard_normal((N, ncols)).astype(np.float32)
    X = torch.zeros((N, ld), dtype=torch.float32, device="cuda")
    X[:, :ncols] = torch.from_numpy(x32)
    ws = op.matvec_workspace(ncols)
    YH = torch.full((N, ld), float("nan"), dtype=torch.float32, device="cuda")
    YS = torch.full((N, ld), float("nan"), dtype=torch.float32, device="cuda")
    op.lhf_toeplitz_matvec_f32(X[:, :ncols], YH[:, :ncols], YS[:, :ncols], ws)
    torch.cuda.synchronize()
    x = x32.astype(np.float64)
    yH_ref, yS_ref = H @ x, S @ x
    assert np.abs(YH[:, :ncols].double().cpu().numpy() - yH_ref).max() <= 1e-6 * np.abs(yH_ref).max()
    assert np.abs(YS[:, :ncols].double().cpu().numpy() - yS_ref).max() <= 1e-6 * np.abs(yS_ref).max()
    if ld > ncols:
        assert torch.isnan(YH[:, ncols:]).all()


def test_exact_eigs_small_matches_lapack(small):
    inst, _, _, H, S = small
    op = lhf.Toeplitz(inst, exact=True)
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


def test_exact_eigs_64_cells_lowest32():
    """A 64-cell chain of the 512-cell workload's cell (4 s + 4 p shells,
    log-U[0.1, 10] exponents, R = 30) with three defect cells: the 32 lowest
    eigenvalues against LAPACK on the oracle's dense exact operator, beside
    those of the block-Toeplitz model of the same chain."""
    inst = make_instance(name="boxB64", L=(64, 1, 1), n=(512, 48, 48), bc="dirichlet", pad=(5.0 / 16, 6.0, 6.0),
                         n_s=4, n_p=4, exp_range=(0.1, 10.0), Z=(1, 6), R=30, seed=182, ndefect=3,
                         defect_seed=183)
    H, S = boxchain.BoxChain(inst).dense()
    ref, _ = toeplitz.lowest_eigenpairs(H, S, 32)
    op = lhf.Toeplitz(inst, exact=True)
    w = torch.empty(32, dtype=torch.float64, device="cuda")
    it, res = op.lhf_toeplitz_eigs(32, w, None, maxit=200, tol=1e-5, seed=4)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    err = np.abs(got - ref).max()
    model = lhf.Toeplitz(inst)
    wm = torch.empty(32, dtype=torch.float64, device="cuda")
    model.lhf_toeplitz_eigs(32, wm, None, maxit=200, tol=1e-5, seed=4)
    torch.cuda.synchronize()
    dmodel = np.abs(wm.cpu().numpy() - got).max()
    print(f"exact box, 64 cells: {it} iterations, residual {res:.2e}, max eig error {err:.2e} Ha; "
          f"block-Toeplitz model differs by up to {dmodel:.2e} Ha", flush=True)
    assert err <= 1e-8
    assert dmodel > 1e-6          # the model's neglected asymmetry and wall terms are visible


def test_exact_c5_chain_sampled_rows_and_residuals():
    """The 512-cell chain with 26 defect cells as an exact box operator: its
    lowest 32 pairs by LOBPCG, and on sampled block rows (a wall row, a defect
    row, an interior row) the product with the oracle's blocks -- both of a
    random block and of the eigenvectors, whose row residuals must vanish."""
    inst = make_config("c5")
    op = lhf.Toeplitz(inst, exact=True)
    L, m0, L0 = inst.L[0], inst.m0, op.info.L0
    N = L * m0
    w = torch.empty(32, dtype=torch.float64, device="cuda")
    V = torch.empty((N, 32), dtype=torch.float64, device="cuda")
    it, res = op.lhf_toeplitz_eigs(32, w, V, maxit=150, tol=1e-5, seed=1)
    torch.cuda.synchronize()
    print(f"exact c5 chain: {it} iterations, residual {res:.2e}", flush=True)
    assert res < 1e-5
    rng = np.random.Generator(np.random.PCG64(6))
    x = np.concatenate([rng.standard_normal((N, 2)), V.cpu().numpy()[:, :4]], axis=1)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yH = torch.empty_like(xt)
    yS = torch.empty_like(xt)
    op.lhf_toeplitz_matvec(lhf.LHF_PREC_FP64, xt, yH, yS, op.matvec_workspace(x.shape[1]))
    torch.cuda.synchronize()
    yh, ys = yH.cpu().numpy(), yS.cpu().numpy()
    box = boxchain.BoxChain(inst)
    lam = w.cpu().numpy()[:4]
    for k in (0, int(inst.def_cells[0]), L // 2):
        rh = np.zeros((m0, x.shape[1]))
        rs = np.zeros((m0, x.shape[1]))
        for m in range(max(0, k - L0), min(L, k + L0 + 1)):
            bh, bs = box.block(min(k, m), max(k, m))
            if k > m:
                bh, bs = bh.T, bs.T
            rh += bh @ x[m * m0:(m + 1) * m0]
            rs += bs @ x[m * m0:(m + 1) * m0]
        sl = slice(k * m0, (k + 1) * m0)
        assert np.abs(yh[sl] - rh).max() <= 1e-11 * np.abs(rh).max(), k
        assert np.abs(ys[sl] - rs).max() <= 1e-11 * np.abs(rs).max(), k
        # eigenvector rows of the oracle's operator: H v - lambda S v
        r = rh[:, 2:] - rs[:, 2:] * lam[None, :]
        assert np.abs(r).max() <= 1e-4 * max(1.0, np.abs(lam).max()), k
