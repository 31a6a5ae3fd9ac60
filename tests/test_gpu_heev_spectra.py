"""Batched eigensolver on blocks with known spectra (through the C ABI).

Each canonical block is a generalized pair (H, S) = (C Q diag(lam) Q^H C^H,
C C^H) with a random unitary Q and a well-conditioned C, so its eigenvalues
are lam exactly, by construction.  The spectra carry exact degeneracies and
clusters split by 1e-9, 1e-6 and 1e-3 Ha, where a perturbative shortcut
would be wrong, next to well-separated spectra with a wide spread, where
the solvers may stop early.  Tolerances as for the pipelines: FP64 within
1e-10 max(|lambda|, 1), mixed (FP32 solve + FP64 refinement) within 1e-8 Ha.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1702_00339_amd import lhf  # noqa: E402
from paper_1702_00339_amd.pipeline import Pipeline  # noqa: E402
from synth import tiny_instance  # noqa: E402

NBLK = 8   # chain of 8 cells: canonical blocks 0..4, blocks 5..7 are conjugates of 3..1


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _spectrum(kind, m0, rng):
    base = np.sort(rng.uniform(-3.0, 10.0, m0))
    if kind == "degenerate":
        lam = np.repeat(base[: (m0 + 2) // 3], 3)[:m0]
    elif kind in ("c1e-9", "c1e-6", "c1e-3"):
        delta = float(kind[1:])
        lam = base.copy()
        lam[1::2] = lam[0::2][: m0 // 2] + delta
    elif kind == "spread":
        lam = np.sort(np.concatenate([rng.uniform(-5.0, 1000.0, m0 - 2), [1000.0, 1000.0]]))[:m0]
    else:
        raise ValueError(kind)
    return np.sort(lam)


def _pair(lam, rng):
    m0 = lam.size
    q, _ = np.linalg.qr(rng.standard_normal((m0, m0)) + 1j * rng.standard_normal((m0, m0)))
    c = np.eye(m0) + 0.3 * (rng.standard_normal((m0, m0)) + 1j * rng.standard_normal((m0, m0))) / np.sqrt(m0)
    h = c @ q @ np.diag(lam) @ q.conj().T @ c.conj().T
    h = 0.5 * (h + h.conj().T)
    s = c @ c.conj().T
    s = 0.5 * (s + s.conj().T)
    return h, s


KINDS = ["degenerate", "c1e-9", "c1e-6", "c1e-3", "spread"]


def _blocks(m0, seed):
    rng = np.random.default_rng(seed)
    lams, hs, ss = [], [], []
    for j in range(NBLK // 2 + 1):
        lam = _spectrum(KINDS[j], m0, rng)
        h, s = _pair(lam, rng)
        lams.append(lam)
        hs.append(h)
        ss.append(s)
    for j in range(NBLK // 2 + 1, NBLK):
        lams.append(lams[NBLK - j])
        hs.append(hs[NBLK - j].conj())
        ss.append(ss[NBLK - j].conj())
    return np.array(lams), np.array(hs), np.array(ss)


# m0 -> (n_s, n_p) of a chain instance with that many functions per cell
SIZES = {4: (4, 0), 8: (2, 2), 16: (4, 4), 32: (8, 8)}


@pytest.mark.parametrize("m0", sorted(SIZES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("layout", ["wide", "four"])
def test_known_spectra(m0, prec, layout):
    n_s, n_p = SIZES[m0]
    inst = tiny_instance(L=(NBLK, 1, 1), n=(64, 12, 12), n_s=n_s, n_p=n_p, seed=170 + m0, R=4)
    assert inst.m0 == m0
    p = lhf.LHF_PREC_FP64 if prec == "fp64" else lhf.LHF_PREC_MIXED
    pipe = Pipeline(inst, prec=p, gram=lhf.LHF_GRAM_FP64)
    # both eigensolver layouts: one matrix entry per thread, or four
    t = pipe.plan.lhf_plan_get_tuning()
    t.heev_wide = 15 if layout == "wide" else 0
    pipe.plan.lhf_plan_set_tuning(t)
    lam, h, s = _blocks(m0, seed=1000 + m0)
    dev = pipe.H_bar.device
    h128 = torch.from_numpy(h.reshape(-1)).to(dev)
    s128 = torch.from_numpy(s.reshape(-1)).to(dev)
    w = torch.empty_like(pipe.w)
    info = torch.empty_like(pipe.info)
    if prec == "fp64":
        pipe.plan.lhf_heev_batched(0, h128, s128, w, info, pipe.ws)
    else:
        h64, s64 = h128.to(torch.complex64), s128.to(torch.complex64)
        pipe.plan.lhf_heev_batched(lhf.LHF_HEEV_REFINE_FP64, h64, s64, w, info, pipe.ws, H_bar64=h128,
                                   S_bar64=s128)
    torch.cuda.synchronize()
    got = w.cpu().numpy().reshape(NBLK, m0)
    assert (info.cpu().numpy() == 0).all(), info.cpu().numpy()
    err = np.abs(got - lam)
    for j in range(NBLK):
        print(f"m0={m0} {prec} block {j} ({KINDS[min(j, NBLK - j)]}): max err {err[j].max():.2e}", flush=True)
    if prec == "fp64":
        assert (err <= 1e-10 * np.maximum(np.abs(lam), 1.0)).all()
    else:
        assert err.max() <= 1e-8
