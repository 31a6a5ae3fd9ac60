"""Host-side checks of the C ABI (no GPU needed).

* liblhf.so loads and exports every function include/lhf.h declares;
* descriptor validation rejects bad input with a status code before any HIP
  call is made (so it runs on a machine without a GPU).
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1702_00339_amd import lhf
from synth import tiny_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lhf.LIB_PATH):
        from paper_1702_00339_amd import build_lib
        build_lib.build()
    return lhf.load()


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lhf_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_hot_path():
    names = _declared_functions()
    for required in ("lhf_assemble_blocks", "lhf_block_fft", "lhf_fourier_blocks", "lhf_heev_batched",
                     "lhf_workspace_size", "lhf_plan_create", "lhf_status_string", "lhf_last_error"):
        assert required in names, required


def test_library_exports_every_declared_symbol(lib):
    raw = C.CDLL(lhf.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert lib.lhf_status_string(lhf.LHF_OK) == b"ok"
    assert lib.lhf_status_string(lhf.LHF_ERR_WORKSPACE) == b"workspace too small"
    assert lib.lhf_version() >= 1


def _create(lib, inst, prec=lhf.LHF_PREC_FP64, gram=lhf.LHF_GRAM_FP64, mutate=None):
    lat, keep = lhf.lattice_from_instance(inst)
    if mutate:
        mutate(lat)
    arr = (lhf.lhf_lattice * 1)(lat)
    h = C.c_void_p()
    st = lib.lhf_plan_create(arr, 1, prec, gram, C.byref(h))
    return st, h, keep


@pytest.mark.parametrize("mutate,expect", [
    (lambda l: setattr(l, "a", -1.0), lhf.LHF_ERR_INVALID),
    (lambda l: l.L.__setitem__(0, 0), lhf.LHF_ERR_INVALID),
    (lambda l: l.n.__setitem__(0, 33), lhf.LHF_ERR_INVALID),          # n not a multiple of L on a periodic dim
    (lambda l: setattr(l, "R", 0), lhf.LHF_ERR_INVALID),
    (lambda l: setattr(l, "R", 65), lhf.LHF_ERR_UNSUPPORTED),
    (lambda l: setattr(l, "sinc_step", 0.0), lhf.LHF_ERR_INVALID),
    (lambda l: setattr(l, "bc", 7), lhf.LHF_ERR_INVALID),
    (lambda l: setattr(l.cell, "m0", 33), lhf.LHF_ERR_UNSUPPORTED),
    (lambda l: setattr(l.cell, "M0", 0), lhf.LHF_ERR_INVALID),
    (lambda l: setattr(l, "bc", lhf.LHF_BC_DIRICHLET), lhf.LHF_ERR_UNSUPPORTED),  # multi-cell box dim
])
def test_plan_validation_rejects_bad_descriptors(lib, mutate, expect):
    inst = tiny_instance(L=(4, 1, 1), n=(32, 16, 16))
    st, h, _ = _create(lib, inst, mutate=mutate)
    assert st == expect, (st, lib.lhf_last_error())
    assert not h.value
    assert lib.lhf_last_error()


def test_plan_validation_rejects_nonpositive_exponent(lib):
    inst = tiny_instance(L=(4, 1, 1), n=(32, 16, 16))
    inst.alpha = inst.alpha.copy()
    inst.alpha[0] = -0.5
    st, h, _ = _create(lib, inst)
    assert st == lhf.LHF_ERR_INVALID
    assert b"exponent" in lib.lhf_last_error()


def test_bad_precision_and_null_output(lib):
    inst = tiny_instance()
    lat, keep = lhf.lattice_from_instance(inst)
    arr = (lhf.lhf_lattice * 1)(lat)
    h = C.c_void_p()
    assert lib.lhf_plan_create(arr, 1, 5, 0, C.byref(h)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_create(arr, 1, 0, 9, C.byref(h)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_create(arr, 1, 1, lhf.LHF_GRAM_FP16X3 + 1, C.byref(h)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_create(arr, 1, 1, -1, C.byref(h)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_create(arr, 0, 0, 0, C.byref(h)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_create(arr, 1, 0, 0, None) == lhf.LHF_ERR_INVALID


def test_hot_calls_reject_null_plan(lib):
    assert lib.lhf_assemble_blocks(None, None, None, None, None, None, None, 0, None) == lhf.LHF_ERR_INVALID
    assert lib.lhf_block_fft(None, 0, None, None, None, None, None, 0, None) == lhf.LHF_ERR_INVALID
    assert lib.lhf_fourier_blocks(None, None, None, None, None, 0, None) == lhf.LHF_ERR_INVALID
    assert lib.lhf_heev_batched(None, 0, None, None, None, None, None, None, None, None, None, None, 0,
                                None) == lhf.LHF_ERR_INVALID


def test_step_graph_and_tuning_reject_null(lib):
    args = lhf.lhf_step_args()
    assert lib.lhf_step(None, C.byref(args), None) == lhf.LHF_ERR_INVALID
    h = C.c_void_p()
    assert lib.lhf_graph_create(None, C.byref(args), C.byref(h)) == lhf.LHF_ERR_INVALID
    assert h.value is None
    assert lib.lhf_graph_launch(None, None) == lhf.LHF_ERR_INVALID
    assert lib.lhf_graph_destroy(None) == lhf.LHF_OK
    t = lhf.lhf_tuning()
    assert lib.lhf_plan_get_tuning(None, C.byref(t)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_set_tuning(None, C.byref(t)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_plan_autotune(None, C.byref(args), None, None, None) == lhf.LHF_ERR_INVALID


def _box(lib, inst, mutate=None):
    box, keep = lhf.box_from_instance(inst)
    if mutate:
        mutate(box)
    h = C.c_void_p()
    st = lib.lhf_toeplitz_create(C.byref(box), C.byref(h))
    return st, h


def _chain(**kw):
    from synth import make_instance
    args = dict(name="box", L=(12, 1, 1), n=(96, 12, 12), bc="dirichlet", pad=(5.0 / 16, 4.0, 4.0), n_s=2,
                exp_range=(0.8, 2.5), Z=2, R=8, seed=3)
    args.update(kw)
    return make_instance(**args)


def test_toeplitz_create_rejects_bad_chains(lib):
    st, h = _box(lib, _chain(bc="periodic"))
    assert st == lhf.LHF_ERR_UNSUPPORTED and h.value is None
    st, _ = _box(lib, _chain(pad=(1.0, 4.0, 4.0)))          # nodes not cell aligned
    assert st == lhf.LHF_ERR_UNSUPPORTED
    assert b"cell aligned" in lib.lhf_last_error()
    st, _ = _box(lib, _chain(L=(12, 2, 1), n=(96, 24, 12)))
    assert st == lhf.LHF_ERR_UNSUPPORTED
    inst = _chain()
    inst.def_cells = np.asarray([3, 3]); inst.def_Z = np.asarray([1.0, 2.0]); inst.def_scale = np.asarray([1.0, 1.0])
    st, _ = _box(lib, inst)
    assert st == lhf.LHF_ERR_INVALID and b"distinct" in lib.lhf_last_error()
    inst.def_cells = np.asarray([12]); inst.def_Z = np.asarray([1.0]); inst.def_scale = np.asarray([1.0])
    assert _box(lib, inst)[0] == lhf.LHF_ERR_INVALID
    inst.def_cells = np.asarray([2]); inst.def_Z = np.asarray([1.0]); inst.def_scale = np.asarray([0.0])
    assert _box(lib, inst)[0] == lhf.LHF_ERR_INVALID
    h = C.c_void_p()
    assert lib.lhf_toeplitz_create(None, C.byref(h)) == lhf.LHF_ERR_INVALID
    info = lhf.lhf_toeplitz_info()
    assert lib.lhf_toeplitz_get_info(None, C.byref(info)) == lhf.LHF_ERR_INVALID
    assert lib.lhf_toeplitz_matvec_workspace(None, 4) == 0
    assert lib.lhf_toeplitz_eigs_workspace(None, 4) == 0
    assert lib.lhf_toeplitz_destroy(None) == lhf.LHF_OK
