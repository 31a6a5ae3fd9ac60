"""GPU parity of the periodic hot path against the CPU oracle (through the C ABI).

Tolerances (from the arithmetic: FP64 rounding of O(1) terms, the FP32
solve's error removed by the FP64 refinement):
  * FP64 pipeline: eigenvalues within 1e-10 max(|lambda|, 1 Ha) of the oracle;
    Grams / generator stacks / Fourier blocks within 1e-12 of the largest
    entry of their kind (the GPU band drops generators below 1e-22 relative).
  * mixed pipeline: eigenvalues within 1e-8 Ha absolute after FP64 refinement;
    the FP32 generator stacks within, relative to their largest entry, 1e-6
    from FP64 Grams (FP32 rounding), 2e-6 from FP32-operand and FP16 hi+lo
    Grams (22- to 24-bit operands, FP32 accumulation) and 1e-4 from bf16
    hi+lo Grams (16-bit operands).
Every case uses the oracle's seeded instances; the oracle computes every
shift, so any effect of the GPU's band truncation shows up here.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import separable  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from paper_1702_00339_amd.pipeline import Pipeline  # noqa: E402
from synth import make_config, make_instance, tiny_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _run(inst, prec, **kw):
    pipe = Pipeline(inst, prec=prec, **kw)
    pipe.step()
    torch.cuda.synchronize()
    return pipe


def _eig_ref(inst):
    res = separable.solve(inst)
    return res, np.sort(res["eig"], axis=-1)


TINY = [
    dict(L=(6, 1, 1), n=(48, 24, 24), n_s=2, n_p=1, seed=101),                   # chain, full band
    dict(L=(16, 1, 1), n=(96, 20, 20), n_s=3, n_p=0, seed=102, exp_range=(0.6, 3.0)),  # banded chain
    dict(L=(5, 4, 1), n=(40, 32, 14), n_s=2, n_p=1, seed=103),                   # 2D, odd/even
    dict(L=(4, 3, 2), n=(32, 24, 16), n_s=4, n_p=0, seed=104),                   # 3D
    dict(L=(1, 1, 1), n=(20, 22, 18), n_s=2, n_p=1, seed=105),                   # one cell
    dict(L=(2, 1, 1), n=(24, 16, 16), n_s=1, n_p=0, seed=106),                   # m0 = 1, self-conjugate blocks
    dict(L=(7, 1, 1), n=(70, 12, 12), n_s=5, n_p=0, seed=107),                   # m0 = 5 (padded to 8), ragged K
    dict(L=(9, 2, 1), n=(90, 18, 12), n_s=3, n_p=4, seed=108, R=6),              # m0 = 15 (padded to 16)
    dict(L=(4, 1, 1), n=(32, 12, 12), n_s=8, n_p=8, seed=109, R=4),              # m0 = 32
    dict(L=(6, 3, 1), n=(48, 24, 12), n_s=2, n_p=0, seed=110),                   # 2D, L1 = 2 mod 4
    dict(L=(12, 2, 2), n=(96, 16, 16), n_s=3, n_p=0, seed=111, exp_range=(0.8, 3.0)),  # 3D, banded L1 = 0 mod 4
]


def _ids(c):
    return f"L{'x'.join(map(str, c['L']))}_m{c.get('n_s', 2) + 3 * c.get('n_p', 0)}"


@pytest.mark.parametrize("case", TINY, ids=_ids)
@pytest.mark.parametrize("fourier", ["dft", "sep"])
def test_fp64_pipeline_matches_oracle(case, fourier):
    inst = tiny_instance(**{"R": 8, **case})
    print(inst.summary(), fourier, flush=True)
    res, ref = _eig_ref(inst)
    pipe = _run(inst, lhf.LHF_PREC_FP64, fourier=fourier)
    assert pipe.separable() == (fourier == "sep")
    info = pipe.info.cpu().numpy()
    assert (info == 0).all(), info
    # generator stacks (block DFT route) and Fourier blocks
    if fourier == "dft":
        Hg, Sg = pipe.stacks("H_gen")[0], pipe.stacks("S_gen")[0]
        assert np.abs(Hg - res["H_gen"]).max() <= 1e-12 * np.abs(res["H_gen"]).max()
        assert np.abs(Sg - res["S_gen"]).max() <= 1e-12 * np.abs(res["S_gen"]).max()
    Hb, Sb = pipe.stacks("H_bar")[0], pipe.stacks("S_bar")[0]
    assert np.abs(Hb - res["H_bar"]).max() <= 1e-12 * np.abs(res["H_bar"]).max()
    assert np.abs(Sb - res["S_bar"]).max() <= 1e-12 * np.abs(res["S_bar"]).max()
    got = pipe.eigenvalues()[0]
    tol = 1e-10 * np.maximum(np.abs(ref), 1.0)
    assert (np.abs(got - ref) <= tol).all(), np.abs(got - ref).max()


# lattices with one cell along the first axis: the dimension-1 Grams keep
# every image shift while the band has one slot (m0^2 a multiple of 8 takes
# the asynchronous staging, the others the synchronous one)
FIRST_AXIS_ONE = [
    dict(L=(1, 4, 3), n=(14, 32, 24), n_s=2, n_p=1, seed=112),                   # 3D
    dict(L=(1, 5, 1), n=(16, 40, 12), n_s=3, n_p=0, seed=113),                   # 2D, odd L2
    dict(L=(1, 4, 3), n=(14, 32, 24), n_s=4, n_p=0, seed=114),                   # m0 = 4: asynchronous staging
]


@pytest.mark.parametrize("case", FIRST_AXIS_ONE, ids=_ids)
def test_separable_one_cell_first_axis(case):
    """Separable Fourier blocks (Theorem 3.3) when the first axis is one cell:
    the staged dimension-1 rows then step by whole shift blocks instead of
    slots.  Blocks and eigenvalues against the oracle, as in the TINY cases."""
    inst = tiny_instance(**{"R": 8, **case})
    print(inst.summary(), flush=True)
    res, ref = _eig_ref(inst)
    pipe = _run(inst, lhf.LHF_PREC_FP64, fourier="sep")
    assert pipe.separable()
    Hb, Sb = pipe.stacks("H_bar")[0], pipe.stacks("S_bar")[0]
    assert np.abs(Hb - res["H_bar"]).max() <= 1e-12 * np.abs(res["H_bar"]).max()
    assert np.abs(Sb - res["S_bar"]).max() <= 1e-12 * np.abs(res["S_bar"]).max()
    got = pipe.eigenvalues()[0]
    tol = 1e-10 * np.maximum(np.abs(ref), 1.0)
    assert (np.abs(got - ref) <= tol).all(), np.abs(got - ref).max()


@pytest.mark.parametrize("case", TINY, ids=_ids)
@pytest.mark.parametrize("gram", [lhf.LHF_GRAM_BF16X3, lhf.LHF_GRAM_FP16X3, lhf.LHF_GRAM_FP32, lhf.LHF_GRAM_FP64])
def test_mixed_pipeline_matches_oracle(case, gram):
    inst = tiny_instance(**{"R": 8, **case})
    print(inst.summary(), "gram", gram, flush=True)
    res, ref = _eig_ref(inst)
    for src, fourier in (("band", "auto"), ("bar64", "auto"), ("dual", "auto"), ("direct", "dft"), ("direct", "sep")):
        pipe = _run(inst, lhf.LHF_PREC_MIXED, gram=gram, refine_src=src, fourier=fourier)
        info = pipe.info.cpu().numpy()
        assert (info == 0).all(), (src, info)
        got = pipe.eigenvalues()[0]
        err = np.abs(got - ref).max()
        assert err <= 1e-8, (src, err)
        if src == "direct":
            continue
        if src == "dual":
            # the complex64 blocks are the roundings of the complex128 ones
            assert torch.equal(pipe.H_bar, pipe.H_bar64.to(torch.complex64))
            assert torch.equal(pipe.S_bar, pipe.S_bar64.to(torch.complex64))
            continue
        Hg = pipe.stacks("H_gen")[0]
        rel = np.abs(Hg - res["H_gen"]).max() / np.abs(res["H_gen"]).max()
        bound = {lhf.LHF_GRAM_FP64: 1e-6, lhf.LHF_GRAM_FP32: 2e-6, lhf.LHF_GRAM_FP16X3: 2e-6,
                 lhf.LHF_GRAM_BF16X3: 1e-4}[gram]
        assert rel <= bound, rel


def test_grams64_layout_and_values():
    """FP64 1D Grams in the documented layout [term][slot][mu][nu], Z w_q on dim 1."""
    inst = tiny_instance(L=(12, 3, 1), n=(96, 24, 20), n_s=2, n_p=1, R=5, seed=111)
    L0 = (2, 2, 2)
    pipe = Pipeline(inst, prec=lhf.LHF_PREC_FP64, L0=L0)
    pipe.step()
    torch.cuda.synchronize()
    g = pipe.grams64.cpu().numpy()
    m0, T = inst.m0, 2 + inst.R
    coef = separable.term_coefficients(inst)
    off = 0
    for ell in range(3):
        Ld = inst.L[ell]
        if Ld == 1:
            shifts = [0]
        elif 2 * L0[ell] + 1 >= Ld:
            shifts = list(range(Ld))
        else:
            shifts = [k % Ld for k in range(-L0[ell], L0[ell] + 1)]
        ref = separable.gram_1d(inst, ell, shifts)
        ns = len(shifts)
        blk = g[off:off + T * ns * m0 * m0].reshape(T, ns, m0, m0)
        off += T * ns * m0 * m0
        sc = np.abs(ref["S"]).max()
        assert np.abs(blk[0] - ref["S"]).max() <= 1e-13 * sc
        assert np.abs(blk[1] - ref["K"]).max() <= 1e-12 * np.abs(ref["K"]).max()
        M = ref["M"] * (coef[:, None, None, None] if ell == 0 else 1.0)
        assert np.abs(blk[2:] - M).max() <= 1e-13 * np.abs(M).max()


def test_several_lattices_in_one_plan():
    insts = [tiny_instance(L=(6, 1, 1), n=(48, 16, 16), n_s=2, seed=121),
             tiny_instance(L=(3, 2, 2), n=(24, 16, 16), n_s=3, n_p=1, seed=122),
             tiny_instance(L=(10, 1, 1), n=(80, 16, 16), n_s=1, seed=123)]
    for prec, tol_abs in ((lhf.LHF_PREC_FP64, None), (lhf.LHF_PREC_MIXED, 1e-8)):
        pipe = _run(insts, prec)
        assert (pipe.info.cpu().numpy() == 0).all()
        for inst, got in zip(insts, pipe.eigenvalues()):
            _, ref = _eig_ref(inst)
            tol = tol_abs if tol_abs else 1e-10 * np.maximum(np.abs(ref), 1.0)
            assert (np.abs(got - ref) <= tol).all()


def test_grouped_plan_mixes_every_class():
    """One plan whose lattices differ in everything the grouped launches split
    on: eigensolver size class (m0 = 1, 5, 6, 15), DFT band class and number
    of DFT passes (1 to 3, the one-cell lattice being a copy).  The band
    half-width 17 is forced on every lattice (it only adds zero generators),
    so the chain's band has 35 slots and takes the wide kernel."""
    insts = [tiny_instance(L=(40, 1, 1), n=(320, 12, 12), n_s=1, seed=151, exp_range=(0.3, 0.6)),
             tiny_instance(L=(3, 2, 2), n=(24, 16, 16), n_s=3, n_p=1, seed=152),
             tiny_instance(L=(1, 1, 1), n=(20, 16, 16), n_s=2, seed=153),
             tiny_instance(L=(5, 4, 1), n=(40, 32, 12), n_s=2, n_p=1, seed=154),
             tiny_instance(L=(9, 1, 1), n=(72, 12, 12), n_s=3, n_p=4, R=6, seed=155)]
    for prec, tol_abs in ((lhf.LHF_PREC_FP64, None), (lhf.LHF_PREC_MIXED, 1e-8)):
        pipe = _run(insts, prec, L0=(17, 17, 17))
        nshift, _, full = pipe.plan.lhf_plan_band(0)
        assert nshift[0] == 35 and full[0] == 0
        assert (pipe.info.cpu().numpy() == 0).all()
        for inst, got in zip(insts, pipe.eigenvalues()):
            _, ref = _eig_ref(inst)
            tol = tol_abs if tol_abs else 1e-10 * np.maximum(np.abs(ref), 1.0)
            assert (np.abs(got - ref) <= tol).all(), inst.name


def test_separable_blocks_match_block_dft():
    """lhf_fourier_blocks (separable formation from the Grams, Theorem 3.3)
    against the block DFT of the FP64 generator stacks, on one plan holding
    every TINY shape (chains, 2D, 3D, one cell, full and banded axes, odd and
    even lengths, m0 from 1 to 32); a plan with a 35-slot band is refused."""
    insts = [tiny_instance(**{"R": 8, **c}) for c in TINY]
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64, fourier="dft")
    pipe.step()
    Hd, Sd = pipe.H_bar.clone(), pipe.S_bar.clone()
    pipe.H_bar.zero_()
    pipe.S_bar.zero_()
    pipe.plan.lhf_fourier_blocks(pipe.grams64, pipe.H_bar, pipe.S_bar, pipe.ws)
    torch.cuda.synchronize()
    for a, b in ((pipe.H_bar, Hd), (pipe.S_bar, Sd)):
        off = 0
        for inst in insts:
            n = inst.ncells * inst.m0 * inst.m0
            x, y = a[off:off + n], b[off:off + n]
            assert (x - y).abs().max().item() <= 1e-13 * y.abs().max().item(), inst.name
            off += n
    wide = Pipeline(tiny_instance(L=(40, 1, 1), n=(320, 12, 12), n_s=1, seed=151, exp_range=(0.3, 0.6)),
                    prec=lhf.LHF_PREC_FP64, L0=(17, 17, 17))
    assert not wide.separable()
    with pytest.raises(lhf.LhfError):
        wide.plan.lhf_fourier_blocks(wide.grams64, wide.H_bar, wide.S_bar, wide.ws)


@pytest.mark.parametrize("mask", [0b0101, 0b1010, 0b1111])
@pytest.mark.parametrize("src", ["direct", "bar64", "band"])
def test_mixed_fp64_classes(mask, src):
    """Mixed plans solving some size classes by the FP64 solve alone (tuning
    field heev_fp64): every class meets the mixed bound, a class taken by
    FP64 solve meets the FP64 one, and a refined solve without complex128
    blocks ("band") keeps the FP32 solve and refinement for every class."""
    insts = [tiny_instance(**{"R": 8, **c}) for c in TINY]
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_MIXED, refine_src=src, want_vectors=True)
    t = pipe.plan.lhf_plan_get_tuning()
    t.heev_fp64 = mask
    pipe.plan.lhf_plan_set_tuning(t)
    assert pipe.plan.lhf_plan_get_tuning().heev_fp64 == mask
    pipe.step()
    torch.cuda.synchronize()
    assert (pipe.info.cpu().numpy() == 0).all()
    for inst, got, V in zip(insts, pipe.eigenvalues(), pipe.stacks("V")):
        res, ref = _eig_ref(inst)
        cls = 0 if inst.m0 <= 4 else 1 if inst.m0 <= 8 else 2 if inst.m0 <= 16 else 3
        assert np.abs(got - ref).max() <= 1e-8, inst.name
        if src != "band" and (mask >> cls) & 1:
            assert (np.abs(got - ref) <= 1e-10 * np.maximum(np.abs(ref), 1.0)).all(), inst.name
        Hb, Sb = res["H_bar"], res["S_bar"]
        Rz = Hb @ V - (Sb @ V) * got[..., None, :]
        assert np.abs(Rz).max() <= 1e-9 * max(1.0, np.abs(got).max()), inst.name


@pytest.mark.parametrize("wide", [15, 0], ids=["wide", "four"])
def test_eigenvectors_fp64_and_refined(wide):
    inst = tiny_instance(L=(5, 2, 1), n=(40, 16, 14), n_s=2, n_p=1, R=6, seed=131)
    res, ref = _eig_ref(inst)
    m0 = inst.m0
    for prec in (lhf.LHF_PREC_FP64, lhf.LHF_PREC_MIXED):
        pipe = Pipeline(inst, prec=prec, want_vectors=True)
        t = pipe.plan.lhf_plan_get_tuning()
        t.heev_wide = wide
        pipe.plan.lhf_plan_set_tuning(t)
        pipe.step()
        torch.cuda.synchronize()
        V = pipe.stacks("V")[0]
        w = pipe.eigenvalues()[0]
        Hb, Sb = res["H_bar"], res["S_bar"]
        R = Hb @ V - (Sb @ V) * w[..., None, :]
        assert np.abs(R).max() <= 1e-9 * max(1.0, np.abs(w).max())
        G = np.conj(np.swapaxes(V, -1, -2)) @ Sb @ V
        assert np.abs(G - np.eye(m0)).max() <= 1e-8


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_full_config_fp64_and_mixed(name):
    """The configurations at full size: every Fourier block entry and every
    block's eigenvalues (the oracle's separable route equals the dense 3D
    quadrature at the 8-cell chain's full size: test_oracle_pins)."""
    inst = make_config(name)
    print(inst.summary(), flush=True)
    res, ref = _eig_ref(inst)
    pipe = _run(inst, lhf.LHF_PREC_FP64)
    assert (pipe.info.cpu().numpy() == 0).all()
    for key, want in (("H_bar", res["H_bar"]), ("S_bar", res["S_bar"])):
        d = np.abs(pipe.stacks(key)[0] - want).max()
        print(f"{name} fp64: max |d{key}| = {d:.2e} Ha", flush=True)
        assert d <= 1e-12 * np.abs(want).max()
    got = pipe.eigenvalues()[0]
    err64 = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    print(f"{name} fp64: max relative eig error {err64.max():.2e}", flush=True)
    assert err64.max() <= 1e-10
    pipe = _run(inst, lhf.LHF_PREC_MIXED)
    assert (pipe.info.cpu().numpy() == 0).all()
    got = pipe.eigenvalues()[0]
    errm = np.abs(got - ref).max()
    print(f"{name} mixed: max abs eig error {errm:.2e} Ha", flush=True)
    assert errm <= 1e-8


def test_heev_info_codes():
    """Non-HPD overlap and non-finite input are reported per block."""
    inst = tiny_instance(L=(4, 1, 1), n=(32, 16, 16), n_s=2, seed=141)
    pipe = _run(inst, lhf.LHF_PREC_FP64)
    m0 = inst.m0
    H = pipe.H_bar.clone().view(4, m0, m0)
    S = pipe.S_bar.clone().view(4, m0, m0)
    S[1] = -torch.eye(m0, dtype=S.dtype, device=S.device)
    H[2, 0, 0] = float("nan")
    w = torch.empty_like(pipe.w)
    info = torch.empty_like(pipe.info)
    pipe.plan.lhf_heev_batched(0, H.view(-1), S.view(-1), w, info, pipe.ws)
    torch.cuda.synchronize()
    got = info.cpu().numpy()
    assert got[1] == 1 and got[2] == -2 and got[0] == 0, got
    # blocks 1 and 3 are a conjugate pair: the pair is solved once, from block 1
    assert got[3] == got[1]


# ----------------------------------------------------------------------------- the 64-lattice mix at full size

# the cheapest lattice of every (L2, L3) pair (all four size classes, prime L1 = 23 and 61) and the
# largest L1 (512 x 4 x 4)
C4_COVER = (41, 59, 20, 28, 2, 47, 24, 62, 39, 31)


@pytest.fixture(scope="module")
def c4_plans():
    from synth import config_c4_lattices
    insts = config_c4_lattices()
    out = {}
    for prec in (lhf.LHF_PREC_FP64, lhf.LHF_PREC_MIXED):
        pipe = _run(insts, prec)
        info = pipe.info.cpu().numpy()
        blocks = {k: pipe.stacks(k) for k in ("H_bar", "S_bar")} if prec == lhf.LHF_PREC_FP64 else None
        out[prec] = (pipe.eigenvalues(), info, blocks)
        del pipe
    return insts, out


@pytest.mark.parametrize("idx", C4_COVER)
def test_c4_mix_lattice(c4_plans, idx):
    """One grouped plan of all 64 lattices (one launch per stage and size
    class); lattice idx against the oracle: Fourier blocks and eigenvalues
    (FP64), eigenvalues (mixed).  The error is printed beside the condition
    number of the overlap blocks, which bounds how block errors reach the
    eigenvalues."""
    insts, out = c4_plans
    inst = insts[idx]
    res, ref = _eig_ref(inst)
    w64, info64, blocks = out[lhf.LHF_PREC_FP64]
    wmx, infomx, _ = out[lhf.LHF_PREC_MIXED]
    sb = res["S_bar"].reshape(-1, inst.m0, inst.m0)
    ev = np.linalg.eigvalsh(sb)
    kappa = float((ev[:, -1] / ev[:, 0]).max())
    off = sum(i.ncells for i in insts[:idx])
    assert (info64[off:off + inst.ncells] == 0).all() and (infomx[off:off + inst.ncells] == 0).all()
    for key in ("H_bar", "S_bar"):
        d = np.abs(blocks[key][idx] - res[key]).max()
        assert d <= 1e-12 * np.abs(res[key]).max(), (key, d)
    rel = (np.abs(w64[idx] - ref) / np.maximum(np.abs(ref), 1.0)).max()
    err = np.abs(wmx[idx] - ref).max()
    print(f"{inst.summary()}: fp64 rel {rel:.2e}, mixed abs {err:.2e} Ha, max kappa(Sbar) {kappa:.3g}", flush=True)
    assert rel <= 1e-10
    assert err <= 1e-8


# ----------------------------------------------------------------------------- several nuclei per cell, off centre

MULTI_NUC = [
    (dict(L=(6, 1, 1), n=(48, 20, 20), n_s=3, n_p=1, seed=171), [1.0, 2.0], [[0.4, -0.3, 0.2], [-1.9, 0.5, -0.6]]),
    (dict(L=(4, 3, 1), n=(32, 24, 16), n_s=2, n_p=1, seed=172), [3.0, 1.0, 1.0],
     [[0.0, 0.0, 0.0], [2.2, -1.1, 0.4], [-2.3, 1.7, -0.9]]),
    (dict(L=(3, 2, 2), n=(24, 16, 16), n_s=4, n_p=0, seed=173), [1.0, 1.0, 2.0, 0.5],
     [[1.2, 1.2, -0.8], [-1.2, -1.2, 0.8], [2.4, 0.1, 2.4], [-0.2, -2.4, 0.3]]),
]


@pytest.mark.parametrize("case,Z,pos", MULTI_NUC, ids=["M0=2 chain", "M0=3 sheet", "M0=4 3D"])
def test_several_off_centre_nuclei(case, Z, pos):
    """M0 = 2, 3, 4 nuclei per cell at off-centre positions (up to 2.4 bohr of
    the 2.5 bohr half-cell), through the ABI's lhf_cell.M0, Z and nuc: both
    Fourier-block routes on the FP64 path, and the mixed path."""
    inst = tiny_instance(**{"R": 8, **case})
    inst.Z = np.asarray(Z, np.float64)
    inst.nuc = np.asarray(pos, np.float64)
    assert inst.M0 == len(Z)
    res, ref = _eig_ref(inst)
    for fourier in ("dft", "sep"):
        pipe = _run(inst, lhf.LHF_PREC_FP64, fourier=fourier)
        assert (pipe.info.cpu().numpy() == 0).all()
        Hb = pipe.stacks("H_bar")[0]
        assert np.abs(Hb - res["H_bar"]).max() <= 1e-12 * np.abs(res["H_bar"]).max(), fourier
        got = pipe.eigenvalues()[0]
        assert (np.abs(got - ref) <= 1e-10 * np.maximum(np.abs(ref), 1.0)).all(), fourier
    pipe = _run(inst, lhf.LHF_PREC_MIXED)
    assert (pipe.info.cpu().numpy() == 0).all()
    assert np.abs(pipe.eigenvalues()[0] - ref).max() <= 1e-8
