"""Fourier blocks in the Hermitian half-space along k3 (lhf_block_fft_half,
lhf_fourier_blocks_half) through the C ABI.

The generators are real symmetric, so Hbar_(-j) = conj(Hbar_j) (Prop. 5.1)
and the blocks j3 > L3/2 add nothing to the kept ones.  The half calls form
exactly the blocks 0 <= j3 <= L3/2 with the same arithmetic as the full calls,
so each lattice's half stack must equal the j3 <= L3/2 planes of the full
stack bit for bit, at the lattice's offset in the half layout (a stack of
half_elems elements).  Plans mix every route: the fused three-dimensional
transform, the pass kernels (a lattice with one transformed dimension, the
third), the wide-band pass kernel (a band of 35 slots), the separable
formation and its chain kernel; odd and even L3, and L3 = 1 (every block kept).
FP64 (complex128) and the mixed plan's complex64 transform.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1702_00339_amd import lhf  # noqa: E402
from paper_1702_00339_amd.pipeline import Pipeline  # noqa: E402
from synth import tiny_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


SHAPES = [
    dict(L=(4, 3, 2), n=(32, 24, 16), n_s=4, n_p=0, seed=201),                   # 3D, even L3
    dict(L=(12, 2, 5), n=(96, 16, 40), n_s=3, n_p=0, seed=202, exp_range=(0.8, 3.0)),  # odd L3, banded L1
    dict(L=(6, 1, 1), n=(48, 24, 24), n_s=2, n_p=1, seed=203),                   # chain
    dict(L=(1, 1, 6), n=(20, 20, 48), n_s=2, n_p=0, seed=204),                   # only the third axis: pass kernels
    dict(L=(5, 4, 1), n=(40, 32, 14), n_s=2, n_p=1, seed=205),                   # 2D, L3 = 1
    dict(L=(3, 2, 4), n=(24, 16, 32), n_s=1, n_p=0, seed=206),                   # m0 = 1
]


def _check_half(insts, full, half):
    """Every lattice's half stack against the j3 <= L3/2 planes of its full stack."""
    off_f = off_h = 0
    for inst in insts:
        L1, L2, L3 = inst.L
        E = inst.m0 * inst.m0
        h3 = L3 // 2 + 1
        f = full[off_f:off_f + L1 * L2 * L3 * E].reshape(L1, L2, L3, E)[:, :, :h3, :]
        h = half[off_h:off_h + L1 * L2 * h3 * E].reshape(L1, L2, h3, E)
        assert torch.equal(f, h), inst.name
        off_f += L1 * L2 * L3 * E
        off_h += L1 * L2 * h3 * E
    assert off_h == half.numel()


@pytest.mark.parametrize("prec", [lhf.LHF_PREC_FP64, lhf.LHF_PREC_MIXED], ids=["fp64", "mixed"])
def test_block_fft_half_is_the_kept_planes(prec):
    insts = [tiny_instance(**{"R": 6, **c}) for c in SHAPES]
    kw = dict(fourier="dft") if prec == lhf.LHF_PREC_FP64 else dict(refine_src="bar64")
    pipe = Pipeline(insts, prec=prec, **kw)
    pipe.step()   # fills the generator stacks
    sz = pipe.plan.sizes
    assert sz.half_elems == sum(i.L[0] * i.L[1] * (i.L[2] // 2 + 1) * i.m0 * i.m0 for i in insts)
    cdt = pipe.H_bar.dtype
    Hf = torch.zeros(int(sz.gen_elems), dtype=cdt, device="cuda")
    Sf = torch.zeros_like(Hf)
    Hh = torch.full((int(sz.half_elems),), float("nan"), dtype=cdt, device="cuda")
    Sh = torch.full_like(Hh, float("nan"))
    pipe.plan.lhf_block_fft(prec, pipe.H_gen, pipe.S_gen, Hf, Sf, pipe.ws)
    pipe.plan.lhf_block_fft_half(prec, pipe.H_gen, pipe.S_gen, Hh, Sh, pipe.ws)
    torch.cuda.synchronize()
    _check_half(insts, Hf, Hh)
    _check_half(insts, Sf, Sh)


def test_block_fft_half_wide_band():
    """A 35-slot band (the wide pass kernel) next to a three-dimensional lattice."""
    insts = [tiny_instance(L=(40, 1, 1), n=(320, 12, 12), n_s=1, seed=207, exp_range=(0.3, 0.6), R=6),
             tiny_instance(L=(4, 2, 3), n=(32, 16, 24), n_s=2, seed=208, R=6)]
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64, fourier="dft", L0=(17, 17, 17))
    pipe.step()
    sz = pipe.plan.sizes
    Hf = torch.zeros(int(sz.gen_elems), dtype=torch.complex128, device="cuda")
    Sf = torch.zeros_like(Hf)
    Hh = torch.full((int(sz.half_elems),), float("nan"), dtype=torch.complex128, device="cuda")
    Sh = torch.full_like(Hh, float("nan"))
    pipe.plan.lhf_block_fft(lhf.LHF_PREC_FP64, pipe.H_gen, pipe.S_gen, Hf, Sf, pipe.ws)
    pipe.plan.lhf_block_fft_half(lhf.LHF_PREC_FP64, pipe.H_gen, pipe.S_gen, Hh, Sh, pipe.ws)
    torch.cuda.synchronize()
    _check_half(insts, Hf, Hh)
    _check_half(insts, Sf, Sh)


def test_fourier_blocks_half_is_the_kept_planes():
    insts = [tiny_instance(**{"R": 6, **c}) for c in SHAPES if c["L"] != (1, 1, 6)]
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64, fourier="sep")
    pipe.step()   # fills the FP64 Grams
    sz = pipe.plan.sizes
    Hf = torch.zeros(int(sz.gen_elems), dtype=torch.complex128, device="cuda")
    Sf = torch.zeros_like(Hf)
    Hh = torch.full((int(sz.half_elems),), float("nan"), dtype=torch.complex128, device="cuda")
    Sh = torch.full_like(Hh, float("nan"))
    pipe.plan.lhf_fourier_blocks(pipe.grams64, Hf, Sf, pipe.ws)
    pipe.plan.lhf_fourier_blocks_half(pipe.grams64, Hh, Sh, pipe.ws)
    torch.cuda.synchronize()
    _check_half(insts, Hf, Hh)
    _check_half(insts, Sf, Sh)
    # the conjugate half really is redundant: Hbar at (-j1, -j2, L3 - j3) = conj(Hbar_j)
    off = 0
    for inst in insts:
        L1, L2, L3 = inst.L
        E = inst.m0 * inst.m0
        A = Hf[off:off + L1 * L2 * L3 * E].reshape(L1, L2, L3, inst.m0, inst.m0).cpu().numpy()
        neg = A[(-np.arange(L1)) % L1][:, (-np.arange(L2)) % L2][:, :, (-np.arange(L3)) % L3]
        assert np.abs(neg - np.conj(A)).max() <= 1e-12 * max(1.0, np.abs(A).max()), inst.name
        off += L1 * L2 * L3 * E


def test_fourier_blocks_half_asynchronous_staging():
    """The separable route's half layout when every lattice has m0^2 a
    multiple of 8 (the asynchronously staged kernel), even and odd L3; the
    full blocks of that kernel against the block DFT route."""
    insts = [tiny_instance(L=(4, 3, 2), n=(32, 24, 16), n_s=4, n_p=0, seed=208, R=6),
             tiny_instance(L=(6, 2, 5), n=(48, 16, 40), n_s=4, n_p=0, seed=209, R=6)]
    assert all(i.m0 * i.m0 % 8 == 0 for i in insts)
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64, fourier="dft")
    pipe.step()   # fills the FP64 Grams and the block DFT's Fourier blocks
    Hd, Sd = pipe.H_bar.clone(), pipe.S_bar.clone()
    sz = pipe.plan.sizes
    Hf = torch.zeros(int(sz.gen_elems), dtype=torch.complex128, device="cuda")
    Sf = torch.zeros_like(Hf)
    Hh = torch.full((int(sz.half_elems),), float("nan"), dtype=torch.complex128, device="cuda")
    Sh = torch.full_like(Hh, float("nan"))
    pipe.plan.lhf_fourier_blocks(pipe.grams64, Hf, Sf, pipe.ws)
    pipe.plan.lhf_fourier_blocks_half(pipe.grams64, Hh, Sh, pipe.ws)
    torch.cuda.synchronize()
    assert (Hf - Hd).abs().max().item() <= 1e-13 * Hd.abs().max().item()
    assert (Sf - Sd).abs().max().item() <= 1e-13 * Sd.abs().max().item()
    _check_half(insts, Hf, Hh)
    _check_half(insts, Sf, Sh)


def test_half_rejects_missing_buffers():
    pipe = Pipeline(tiny_instance(**{"R": 6, **SHAPES[0]}), prec=lhf.LHF_PREC_FP64, fourier="dft")
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_block_fft_half(lhf.LHF_PREC_FP64, pipe.H_gen, pipe.S_gen, None, pipe.S_bar, pipe.ws)
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_fourier_blocks_half(pipe.grams64, pipe.H_bar, None, pipe.ws)
