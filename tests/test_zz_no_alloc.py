"""lhf_fourier_blocks_noalloc through the C ABI: the separable Fourier blocks
with the transformed Grams in the library's static device scratch instead of
a workspace.

* two calls in a row, the second on a smaller plan (the scratch still holds
  the first call's values), each equal bit for bit to lhf_fourier_blocks of
  the same Grams with a workspace (same kernels, same inputs), and within the
  FP64 tolerance of the oracle's Fourier blocks (Theorem 3.3 route);
* a plan whose transformed Grams exceed the static maximum is refused before
  anything is launched.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import separable  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from paper_1702_00339_amd.pipeline import Pipeline  # noqa: E402
from synth import make_instance, tiny_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _blocks_both_ways(insts):
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64, fourier="sep")
    p = pipe.plan
    p.lhf_assemble_blocks(None, None, pipe.grams64, pipe.ws)
    p.lhf_fourier_blocks(pipe.grams64, pipe.H_bar, pipe.S_bar, pipe.ws)
    H = torch.full_like(pipe.H_bar, float("nan"))
    S = torch.full_like(pipe.S_bar, float("nan"))
    p.lhf_fourier_blocks_noalloc(pipe.grams64, H, S)
    torch.cuda.synchronize()
    return pipe, H, S


def _check_vs_oracle(pipe, H, S, insts):
    off = 0
    for inst in insts:
        ref = separable.solve(inst)
        cnt = inst.ncells * inst.m0 * inst.m0
        for got, want in ((H, ref["H_bar"]), (S, ref["S_bar"])):
            g = got[off:off + cnt].cpu().numpy().reshape(want.shape)
            assert np.abs(g - want).max() <= 1e-12 * np.abs(want).max(), inst.name
        off += cnt


def test_noalloc_matches_workspace_call_twice_shrinking():
    big = [tiny_instance(L=(6, 4, 3), n=(48, 32, 24), n_s=2, n_p=1, R=6, seed=701),
           tiny_instance(L=(5, 2, 1), n=(40, 16, 14), n_s=3, n_p=0, R=6, seed=702)]
    small = [tiny_instance(L=(4, 1, 1), n=(32, 16, 16), n_s=2, n_p=0, R=5, seed=703)]
    for insts in (big, small):
        pipe, H, S = _blocks_both_ways(insts)
        assert torch.equal(H, pipe.H_bar) and torch.equal(S, pipe.S_bar)
        _check_vs_oracle(pipe, H, S, insts)


def test_noalloc_refuses_plan_beyond_static_scratch():
    # (2 + R) (L2 + L3) m0^2 complex128 = 26 * 128 * 1024 * 16 bytes > 32 MiB
    inst = make_instance(name="big", L=(2, 64, 64), n=(32, 1024, 1024), n_s=8, n_p=8, R=24, seed=704)
    plan = lhf.Plan([inst], prec=lhf.LHF_PREC_FP64)
    dummy = torch.zeros(16, dtype=torch.complex128, device="cuda")
    grams = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(lhf.LhfError) as e:
        plan.lhf_fourier_blocks_noalloc(grams, dummy, dummy)
    assert e.value.status == lhf.LHF_ERR_UNSUPPORTED
    assert "static scratch" in str(e.value)
