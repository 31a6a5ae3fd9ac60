"""The whole-step entry points on the GPU: lhf_step, its hipGraph capture and
the autotuner (through the C ABI).

* lhf_step gives bit-identical results to the three stage calls (the same
  kernels in the same order; every kernel is deterministic);
* a captured step replayed several times, with eager work and host
  synchronisations between the replays, rewrites every output each time and
  matches the eager step bit for bit;
* autotuned settings stay in range, keep the eigenvalues within the
  parity tolerance of the oracle, and a second plan with the same work reads
  them back from the cache file.
"""

import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import separable  # noqa: E402
from paper_1702_00339_amd import lhf  # noqa: E402
from paper_1702_00339_amd.pipeline import Pipeline  # noqa: E402
from synth import tiny_instance  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _mix():
    return [tiny_instance(L=(6, 1, 1), n=(48, 16, 16), n_s=2, seed=161),
            tiny_instance(L=(3, 2, 2), n=(24, 16, 16), n_s=3, n_p=1, seed=162),
            tiny_instance(L=(10, 1, 1), n=(80, 16, 16), n_s=5, seed=163),
            tiny_instance(L=(1, 1, 1), n=(20, 16, 16), n_s=2, seed=164)]


def _blocks(pipe):
    """The Fourier block buffers the pipeline's step writes."""
    out = [] if pipe.refine_src == "direct" else [pipe.H_bar, pipe.S_bar]
    if pipe.H_bar64 is not None:
        out += [pipe.H_bar64, pipe.S_bar64]
    return out


def _outputs(pipe):
    out = [pipe.w.clone(), pipe.info.clone()] + [b.clone() for b in _blocks(pipe)]
    if pipe.V is not None:
        out.append(pipe.V.clone())
    return out


def _poison(pipe):
    pipe.w.fill_(float("nan"))
    pipe.info.fill_(99)
    for b in _blocks(pipe):
        b.zero_()
    if pipe.V is not None:
        pipe.V.zero_()


PRECS = [(lhf.LHF_PREC_FP64, False), (lhf.LHF_PREC_MIXED, False), (lhf.LHF_PREC_MIXED, True)]


@pytest.mark.parametrize("fourier", ["dft", "sep"])
@pytest.mark.parametrize("prec,vec", PRECS, ids=["fp64", "mixed", "mixed_vectors"])
def test_native_step_matches_stage_calls(prec, vec, fourier):
    pipe = Pipeline(_mix(), prec=prec, want_vectors=vec, fourier=fourier)
    pipe.step()
    torch.cuda.synchronize()
    ref = _outputs(pipe)
    _poison(pipe)
    pipe.step_native()
    torch.cuda.synchronize()
    for a, b in zip(ref, _outputs(pipe)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("fourier", ["dft", "sep"])
@pytest.mark.parametrize("prec,vec", PRECS, ids=["fp64", "mixed", "mixed_vectors"])
def test_graph_replays_match_eager(prec, vec, fourier):
    pipe = Pipeline(_mix(), prec=prec, want_vectors=vec, fourier=fourier)
    pipe.step_native()
    torch.cuda.synchronize()
    ref = _outputs(pipe)
    graph = pipe.capture()
    for rep in range(4):
        _poison(pipe)
        torch.cuda.synchronize()
        graph.lhf_graph_launch()
        torch.cuda.synchronize()
        got = _outputs(pipe)
        for a, b in zip(ref, got):
            assert torch.equal(a, b), f"replay {rep}"
        # eager work of the program between replays
        pipe.step_native()
        scratch = torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
    graph.close()


def test_autotune_keeps_results_and_caches(tmp_path):
    insts = _mix()
    cache = str(tmp_path / "tune.json")
    pipe = Pipeline(insts, prec=lhf.LHF_PREC_MIXED)
    t = pipe.autotune(cache)
    assert t.from_cache == 0 and t.step_ms > 0
    assert t.gram_split in (16, 32, 64, 128, 256) and t.gram_grid in (1024, 2048, 4096, 8192)
    assert t.dft_threads in (32768, 65536, 131072, 262144, 524288) and t.tol32_scale in (1, 16, 256, 4096)
    got = pipe.plan.lhf_plan_get_tuning()
    assert (got.dft_threads, got.gram_split, got.gram_grid, got.tol32_scale, got.heev_wide, got.fourier_sep,
            got.heev_fp64, got.gram_tile) == \
        (t.dft_threads, t.gram_split, t.gram_grid, t.tol32_scale, t.heev_wide, t.fourier_sep, t.heev_fp64,
         t.gram_tile)
    assert 0 <= t.heev_wide <= 15 and t.fourier_sep in (0, 1) and 0 <= t.heev_fp64 <= 15 and t.gram_tile in (64, 32)
    entries = json.load(open(cache))
    assert len(entries) == 1
    pipe.step_native()
    torch.cuda.synchronize()
    assert (pipe.info.cpu().numpy() == 0).all()
    for inst, w in zip(insts, pipe.eigenvalues()):
        ref = np.sort(separable.solve(inst)["eig"], axis=-1)
        assert np.abs(w - ref).max() <= 1e-8, inst.name
    # same work in a new plan: settings come from the cache
    again = Pipeline(insts, prec=lhf.LHF_PREC_MIXED)
    t2 = again.autotune(cache)
    assert t2.from_cache == 1
    assert (t2.dft_threads, t2.gram_split, t2.gram_grid, t2.tol32_scale, t2.heev_wide, t2.fourier_sep,
            t2.heev_fp64, t2.gram_tile) == \
        (t.dft_threads, t.gram_split, t.gram_grid, t.tol32_scale, t.heev_wide, t.fourier_sep, t.heev_fp64,
         t.gram_tile)
    # a different plan adds its own entry
    Pipeline(insts[:2], prec=lhf.LHF_PREC_FP64).autotune(cache)
    assert len(json.load(open(cache))) == 2


def test_set_tuning_extremes_keep_parity():
    """The smallest and largest launch shapes still give the oracle's eigenvalues."""
    insts = _mix()
    refs = [np.sort(separable.solve(i)["eig"], axis=-1) for i in insts]
    for dft, split, grid, wide, sep, tile in ((32768, 1, 1, 0, 0, 32), (1 << 24, 256, 1 << 20, 15, 1, 64),
                                              (32768, 256, 1 << 20, 15, 1, 32)):
        pipe = Pipeline(insts, prec=lhf.LHF_PREC_FP64)
        t = pipe.plan.lhf_plan_get_tuning()
        t.dft_threads, t.gram_split, t.gram_grid, t.heev_wide, t.fourier_sep, t.gram_tile = dft, split, grid, wide, sep, tile
        pipe.plan.lhf_plan_set_tuning(t)
        pipe.step_native()
        torch.cuda.synchronize()
        for w, ref in zip(pipe.eigenvalues(), refs):
            assert (np.abs(w - ref) <= 1e-10 * np.maximum(np.abs(ref), 1.0)).all()
    # the 32 tile in the FP32, bf16 and FP16 hi+lo Gram modes of mixed plans
    for gram in (lhf.LHF_GRAM_FP32, lhf.LHF_GRAM_BF16X3, lhf.LHF_GRAM_FP16X3):
        mix = Pipeline(insts, prec=lhf.LHF_PREC_MIXED, gram=gram, refine_src="band")
        t = mix.plan.lhf_plan_get_tuning()
        t.gram_tile = 32
        mix.plan.lhf_plan_set_tuning(t)
        mix.step()
        torch.cuda.synchronize()
        for w, ref in zip(mix.eigenvalues(), refs):
            assert np.abs(w - ref).max() <= 1e-8
    bad = pipe.plan.lhf_plan_get_tuning()
    bad.gram_split = 257
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_plan_set_tuning(bad)
    bad = pipe.plan.lhf_plan_get_tuning()
    bad.heev_wide = 16
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_plan_set_tuning(bad)
    bad = pipe.plan.lhf_plan_get_tuning()
    bad.fourier_sep = 2
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_plan_set_tuning(bad)
    bad = pipe.plan.lhf_plan_get_tuning()
    bad.heev_fp64 = 16
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_plan_set_tuning(bad)
    bad = pipe.plan.lhf_plan_get_tuning()
    bad.gram_tile = 48
    with pytest.raises(lhf.LhfError):
        pipe.plan.lhf_plan_set_tuning(bad)
    # an FP64 plan accepts the mask and reads 0: its classes all take the FP64 solve
    t = pipe.plan.lhf_plan_get_tuning()
    t.heev_fp64 = 15
    pipe.plan.lhf_plan_set_tuning(t)
    assert pipe.plan.lhf_plan_get_tuning().heev_fp64 == 0


def test_graph_is_stale_after_tuning_change():
    """A graph bakes in the plan's launch shapes and work tables: after the
    tuning changes, launching it is refused (no launch), a new capture runs
    and matches the eager step, and setting the same tuning again keeps
    graphs valid."""
    pipe = Pipeline(_mix(), prec=lhf.LHF_PREC_FP64)
    graph = pipe.capture()
    t = pipe.plan.lhf_plan_get_tuning()
    pipe.plan.lhf_plan_set_tuning(t)          # unchanged: still valid
    graph.lhf_graph_launch()
    torch.cuda.synchronize()
    t.gram_tile = 32 if t.gram_tile == 64 else 64
    pipe.plan.lhf_plan_set_tuning(t)
    with pytest.raises(lhf.LhfError):
        graph.lhf_graph_launch()
    graph.close()
    pipe.step_native()
    torch.cuda.synchronize()
    ref = _outputs(pipe)
    _poison(pipe)
    again = pipe.capture()
    again.lhf_graph_launch()
    torch.cuda.synchronize()
    for a, b in zip(ref, _outputs(pipe)):
        assert torch.equal(a, b)
    again.close()
