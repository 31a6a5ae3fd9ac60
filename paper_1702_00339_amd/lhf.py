"""ctypes binding of liblhf.so (argument marshalling only).

The functions keep the C names and signatures of include/lhf.h; ``Plan``
wraps a plan handle and passes torch tensors' device pointers and the current
torch stream.  Every computation runs in the HIP library: there is no CPU
fallback, and loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LHF_LIB selects another build of the same library (the host tests run the
# sanitizer build through it)
LIB_PATH = os.environ.get("LHF_LIB") or os.path.join(HERE, "lib", "liblhf.so")

LHF_OK, LHF_ERR_INVALID, LHF_ERR_UNSUPPORTED, LHF_ERR_WORKSPACE, LHF_ERR_HIP, LHF_ERR_ALLOC = 0, -1, -2, -3, -4, -5
LHF_PREC_FP64, LHF_PREC_MIXED = 0, 1
LHF_GRAM_FP64, LHF_GRAM_FP32, LHF_GRAM_BF16X3, LHF_GRAM_FP16X3 = 0, 1, 2, 3
LHF_BC_PERIODIC, LHF_BC_DIRICHLET = 0, 1
LHF_HEEV_VECTORS, LHF_HEEV_REFINE_FP64, LHF_HEEV_FP32_SOLVE = 1, 2, 4


class lhf_cell(C.Structure):
    _fields_ = [("m0", C.c_int32), ("alpha", C.POINTER(C.c_double)), ("centre", C.POINTER(C.c_double)),
                ("ang", C.POINTER(C.c_int32)), ("M0", C.c_int32), ("Z", C.POINTER(C.c_double)),
                ("nuc", C.POINTER(C.c_double))]


class lhf_lattice(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("n", C.c_int32 * 3), ("a", C.c_double), ("pad", C.c_double * 3),
                ("bc", C.c_int32), ("R", C.c_int32), ("sinc_u0", C.c_double), ("sinc_step", C.c_double),
                ("L0", C.c_int32 * 3), ("cell", lhf_cell)]


class lhf_sizes(C.Structure):
    _fields_ = [("nlat", C.c_int64), ("nblocks", C.c_int64), ("gen_elems", C.c_int64),
                ("w_elems", C.c_int64), ("grams_elems", C.c_int64), ("ws_bytes", C.c_size_t),
                ("half_elems", C.c_int64)]


class lhf_step_args(C.Structure):
    _fields_ = [("H_gen", C.c_void_p), ("S_gen", C.c_void_p), ("grams64", C.c_void_p), ("H_gen64", C.c_void_p),
                ("S_gen64", C.c_void_p), ("H_bar", C.c_void_p), ("S_bar", C.c_void_p), ("H_bar64", C.c_void_p),
                ("S_bar64", C.c_void_p), ("w", C.c_void_p), ("V", C.c_void_p), ("info", C.c_void_p),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t), ("heev_flags", C.c_uint32)]


class lhf_tuning(C.Structure):
    _fields_ = [("dft_threads", C.c_int32), ("gram_split", C.c_int32), ("gram_grid", C.c_int32),
                ("tol32_scale", C.c_int32), ("heev_wide", C.c_int32), ("fourier_sep", C.c_int32),
                ("heev_fp64", C.c_int32), ("gram_tile", C.c_int32), ("step_ms", C.c_double),
                ("from_cache", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class lhf_box(C.Structure):
    _fields_ = [("lat", lhf_lattice), ("ndef", C.c_int32), ("def_cells", C.POINTER(C.c_int32)),
                ("def_Z", C.POINTER(C.c_double)), ("def_scale", C.POINTER(C.c_double))]


class lhf_toeplitz_info(C.Structure):
    _fields_ = [("L", C.c_int32), ("m0", C.c_int32), ("L0", C.c_int32), ("N", C.c_int32), ("P", C.c_int32),
                ("ncross", C.c_int32), ("ncross_blocks", C.c_int32), ("sigma", C.c_double)]


class LhfError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"lhf status {status}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load liblhf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its bundled HIP runtime has the same soname as the system
    # one, so the library then binds to the runtime that owns torch's streams
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it first (python -m paper_1702_00339_amd.build_lib)")
    lib = C.CDLL(path)
    vp, i32, u32, sz = C.c_void_p, C.c_int32, C.c_uint32, C.c_size_t
    sig = {
        "lhf_plan_create": (i32, [C.POINTER(lhf_lattice), i32, i32, i32, C.POINTER(vp)]),
        "lhf_plan_sizes": (i32, [vp, C.POINTER(lhf_sizes)]),
        "lhf_plan_band": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "lhf_workspace_size": (sz, [vp]),
        "lhf_plan_destroy": (i32, [vp]),
        "lhf_assemble_blocks": (i32, [vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "lhf_block_fft": (i32, [vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "lhf_block_fft_half": (i32, [vp, i32, vp, vp, vp, vp, vp, sz, vp]),
        "lhf_block_fft_dual": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "lhf_fourier_blocks": (i32, [vp, vp, vp, vp, vp, sz, vp]),
        "lhf_fourier_blocks_half": (i32, [vp, vp, vp, vp, vp, sz, vp]),
        "lhf_fourier_blocks_noalloc": (i32, [vp, vp, vp, vp, vp]),
        "lhf_heev_batched": (i32, [vp, u32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]),
        "lhf_eigvecs_lattice": (i32, [vp, i32, vp, i32, vp, vp, vp]),
        "lhf_step": (i32, [vp, C.POINTER(lhf_step_args), vp]),
        "lhf_graph_create": (i32, [vp, C.POINTER(lhf_step_args), C.POINTER(vp)]),
        "lhf_graph_launch": (i32, [vp, vp]),
        "lhf_graph_destroy": (i32, [vp]),
        "lhf_plan_get_tuning": (i32, [vp, C.POINTER(lhf_tuning)]),
        "lhf_plan_set_tuning": (i32, [vp, C.POINTER(lhf_tuning)]),
        "lhf_plan_autotune": (i32, [vp, C.POINTER(lhf_step_args), vp, C.c_char_p, C.POINTER(lhf_tuning)]),
        "lhf_toeplitz_create": (i32, [C.POINTER(lhf_box), C.POINTER(vp)]),
        "lhf_box_exact_create": (i32, [C.POINTER(lhf_box), C.POINTER(vp)]),
        "lhf_toeplitz3_create": (i32, [C.POINTER(lhf_lattice), C.POINTER(vp)]),
        "lhf_toeplitz3_generators": (i32, [vp, vp, vp]),
        "lhf_toeplitz_get_info": (i32, [vp, C.POINTER(lhf_toeplitz_info)]),
        "lhf_toeplitz_blocks": (i32, [vp, vp, vp, vp, vp, vp]),
        "lhf_toeplitz_matvec_workspace": (sz, [vp, i32]),
        "lhf_toeplitz_matvec": (i32, [vp, i32, i32, vp, vp, vp, i32, vp, sz, vp]),
        "lhf_toeplitz_matvec_f32": (i32, [vp, i32, vp, vp, vp, i32, vp, sz, vp]),
        "lhf_toeplitz_eigs_workspace": (sz, [vp, i32]),
        "lhf_toeplitz_eigs": (i32, [vp, i32, i32, C.c_double, C.c_uint64, vp, vp, C.POINTER(i32),
                                    C.POINTER(C.c_double), vp, sz, vp]),
        "lhf_toeplitz_destroy": (i32, [vp]),
        "lhf_dense_syev": (i32, [i32, i32, vp, i32, vp, vp, i32, vp]),
        "lhf_status_string": (C.c_char_p, [i32]),
        "lhf_last_error": (C.c_char_p, []),
        "lhf_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names the binding expects the library to export."""
    return ["lhf_plan_create", "lhf_plan_sizes", "lhf_plan_band", "lhf_workspace_size", "lhf_plan_destroy",
            "lhf_assemble_blocks", "lhf_block_fft", "lhf_block_fft_half", "lhf_block_fft_dual", "lhf_fourier_blocks",
            "lhf_fourier_blocks_half",
            "lhf_fourier_blocks_noalloc", "lhf_heev_batched", "lhf_eigvecs_lattice", "lhf_step", "lhf_graph_create",
            "lhf_graph_launch", "lhf_graph_destroy", "lhf_plan_get_tuning", "lhf_plan_set_tuning",
            "lhf_plan_autotune", "lhf_toeplitz_create", "lhf_box_exact_create", "lhf_toeplitz3_create",
            "lhf_toeplitz3_generators", "lhf_toeplitz_get_info", "lhf_toeplitz_blocks",
            "lhf_toeplitz_matvec_workspace", "lhf_toeplitz_matvec", "lhf_toeplitz_matvec_f32",
            "lhf_toeplitz_eigs_workspace",
            "lhf_toeplitz_eigs", "lhf_toeplitz_destroy", "lhf_dense_syev",
            "lhf_status_string", "lhf_last_error", "lhf_version"]


def _check(st):
    if st != LHF_OK:
        lib = load()
        raise LhfError(st, lib.lhf_last_error().decode())


def lattice_from_instance(inst, L0=(-1, -1, -1)):
    """Fill an lhf_lattice from a synth Instance; returns (struct, keepalive)."""
    keep = []

    def arr(x, dt, ct):
        a = np.ascontiguousarray(np.asarray(x, dtype=dt).ravel())
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(ct))

    lat = lhf_lattice()
    lat.L[:] = [int(v) for v in inst.L]
    lat.n[:] = [int(v) for v in inst.n]
    lat.a = float(inst.a)
    lat.pad[:] = [float(v) for v in inst.pad]
    lat.bc = LHF_BC_PERIODIC if inst.bc == "periodic" else LHF_BC_DIRICHLET
    lat.R = int(inst.R)
    lat.sinc_u0 = float(inst.sinc_u0)
    lat.sinc_step = float(inst.sinc_step)
    lat.L0[:] = [int(v) for v in L0]
    cell = lhf_cell()
    cell.m0 = inst.m0
    cell.alpha = arr(inst.alpha, np.float64, C.c_double)
    cell.centre = arr(inst.centre, np.float64, C.c_double)
    cell.ang = arr(inst.ang, np.int32, C.c_int32)
    cell.M0 = inst.M0
    cell.Z = arr(inst.Z, np.float64, C.c_double)
    cell.nuc = arr(inst.nuc, np.float64, C.c_double)
    lat.cell = cell
    return lat, keep


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def lhf_dense_syev(m, k, A, lda, w, V, ldv):
    """The k lowest eigenpairs of the symmetric m x m matrix A (device FP64
    tensors; V row-major m x k)."""
    lib = load()
    _check(lib.lhf_dense_syev(m, k, _ptr(A), lda, _ptr(w), _ptr(V), ldv, _stream()))


class Plan:
    """A plan over one or more lattices (lhf_plan_create / lhf_plan_destroy)."""

    def __init__(self, instances, prec=LHF_PREC_FP64, gram=LHF_GRAM_FP64, L0=None):
        lib = load()
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        arr = (lhf_lattice * len(instances))()
        self._keep = []
        for i, inst in enumerate(instances):
            lat, keep = lattice_from_instance(inst, L0 if L0 is not None else (-1, -1, -1))
            arr[i] = lat
            self._keep.append(keep)
        h = C.c_void_p()
        _check(lib.lhf_plan_create(arr, len(instances), prec, gram, C.byref(h)))
        self.handle = h
        self.prec = prec
        self.gram = gram
        self.instances = list(instances)
        s = lhf_sizes()
        _check(lib.lhf_plan_sizes(h, C.byref(s)))
        self.sizes = s

    def close(self):
        if getattr(self, "handle", None):
            load().lhf_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lhf_plan_band(self, index=0):
        """(nshift, L0, full) per dimension of lattice ``index``."""
        ns, l0, fu = (C.c_int32 * 3)(), (C.c_int32 * 3)(), (C.c_int32 * 3)()
        _check(load().lhf_plan_band(self.handle, index, ns, l0, fu))
        return list(ns), list(l0), list(fu)

    # ----------------------------------------------------------------- buffers
    def workspace(self, device="cuda"):
        import torch
        return torch.empty(max(1, int(self.sizes.ws_bytes)), dtype=torch.uint8, device=device)

    # ----------------------------------------------------------------- calls
    def lhf_assemble_blocks(self, H_gen, S_gen, grams64, ws, H_gen64=None, S_gen64=None):
        _check(load().lhf_assemble_blocks(self.handle, _ptr(H_gen), _ptr(S_gen), _ptr(grams64),
                                          _ptr(H_gen64), _ptr(S_gen64), _ptr(ws), ws.numel(), _stream()))

    def lhf_block_fft(self, prec, H_gen, S_gen, H_bar, S_bar, ws):
        _check(load().lhf_block_fft(self.handle, prec, _ptr(H_gen), _ptr(S_gen), _ptr(H_bar), _ptr(S_bar),
                                    _ptr(ws), ws.numel(), _stream()))

    def lhf_block_fft_half(self, prec, H_gen, S_gen, H_half, S_half, ws):
        _check(load().lhf_block_fft_half(self.handle, prec, _ptr(H_gen), _ptr(S_gen), _ptr(H_half), _ptr(S_half),
                                         _ptr(ws), ws.numel(), _stream()))

    def lhf_block_fft_dual(self, H_gen64, S_gen64, H_bar64, S_bar64, H_bar32, S_bar32, ws):
        _check(load().lhf_block_fft_dual(self.handle, _ptr(H_gen64), _ptr(S_gen64), _ptr(H_bar64), _ptr(S_bar64),
                                         _ptr(H_bar32), _ptr(S_bar32), _ptr(ws), ws.numel(), _stream()))

    def lhf_fourier_blocks(self, grams64, H_bar64, S_bar64, ws):
        _check(load().lhf_fourier_blocks(self.handle, _ptr(grams64), _ptr(H_bar64), _ptr(S_bar64), _ptr(ws),
                                         ws.numel(), _stream()))

    def lhf_fourier_blocks_half(self, grams64, H_half64, S_half64, ws):
        _check(load().lhf_fourier_blocks_half(self.handle, _ptr(grams64), _ptr(H_half64), _ptr(S_half64),
                                              _ptr(ws), ws.numel(), _stream()))

    def lhf_fourier_blocks_noalloc(self, grams64, H_bar64, S_bar64):
        _check(load().lhf_fourier_blocks_noalloc(self.handle, _ptr(grams64), _ptr(H_bar64), _ptr(S_bar64),
                                                 _stream()))

    def lhf_eigvecs_lattice(self, lattice, V, sel, U):
        """sel: device int32 tensor [nsel, 2] of (block, column); U: complex128 [nsel, ncells, m0]."""
        _check(load().lhf_eigvecs_lattice(self.handle, int(lattice), _ptr(V), int(sel.shape[0]), _ptr(sel), _ptr(U),
                                          _stream()))

    def lhf_heev_batched(self, flags, H_bar, S_bar, w, info, ws, V=None, H_bar64=None, S_bar64=None,
                         H_gen64=None, S_gen64=None):
        _check(load().lhf_heev_batched(self.handle, flags, _ptr(H_bar), _ptr(S_bar), _ptr(H_bar64),
                                       _ptr(S_bar64), _ptr(H_gen64), _ptr(S_gen64), _ptr(w), _ptr(V),
                                       _ptr(info), _ptr(ws), ws.numel(), _stream()))

    def lhf_step(self, args):
        _check(load().lhf_step(self.handle, C.byref(args), _stream()))

    def lhf_plan_get_tuning(self):
        t = lhf_tuning()
        _check(load().lhf_plan_get_tuning(self.handle, C.byref(t)))
        return t

    def lhf_plan_set_tuning(self, tuning):
        _check(load().lhf_plan_set_tuning(self.handle, C.byref(tuning)))

    def lhf_plan_autotune(self, args, cache_path=None):
        t = lhf_tuning()
        path = cache_path.encode() if cache_path else None
        _check(load().lhf_plan_autotune(self.handle, C.byref(args), _stream(), path, C.byref(t)))
        return t

    def lhf_graph_create(self, args):
        return Graph(self, args)


class Graph:
    """A captured step (lhf_graph_create); keeps its plan and args alive."""

    def __init__(self, plan, args):
        self.plan, self.args = plan, args
        h = C.c_void_p()
        _check(load().lhf_graph_create(plan.handle, C.byref(args), C.byref(h)))
        self.handle = h

    def lhf_graph_launch(self):
        _check(load().lhf_graph_launch(self.handle, _stream()))

    def close(self):
        if getattr(self, "handle", None):
            load().lhf_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def box_from_instance(inst):
    """Fill an lhf_box from a synth Instance (Dirichlet chain with defects);
    returns (struct, keepalive)."""
    lat, keep = lattice_from_instance(inst)
    box = lhf_box()
    box.lat = lat
    cells = np.ascontiguousarray(inst.def_cells, dtype=np.int32)
    dz = np.ascontiguousarray(inst.def_Z, dtype=np.float64)
    ds = np.ascontiguousarray(inst.def_scale, dtype=np.float64)
    keep = list(keep) + [cells, dz, ds]
    box.ndef = len(cells)
    box.def_cells = cells.ctypes.data_as(C.POINTER(C.c_int32))
    box.def_Z = dz.ctypes.data_as(C.POINTER(C.c_double))
    box.def_scale = ds.ctypes.data_as(C.POINTER(C.c_double))
    return box, keep


class Toeplitz:
    """A Dirichlet-chain operator: the perturbed block-Toeplitz model
    (lhf_toeplitz_create) or, with exact=True, the exact box operator
    (lhf_box_exact_create); freed by lhf_toeplitz_destroy."""

    def __init__(self, inst, exact=False, levels=1):
        self.inst = inst
        self.exact = exact
        h = C.c_void_p()
        if levels == 3:
            lat, self._keep = lattice_from_instance(inst)
            _check(load().lhf_toeplitz3_create(C.byref(lat), C.byref(h)))
        else:
            box, self._keep = box_from_instance(inst)
            create = load().lhf_box_exact_create if exact else load().lhf_toeplitz_create
            _check(create(C.byref(box), C.byref(h)))
        self.handle = h
        info = lhf_toeplitz_info()
        _check(load().lhf_toeplitz_get_info(self.handle, C.byref(info)))
        self.info = info

    def close(self):
        if getattr(self, "handle", None):
            load().lhf_toeplitz_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def lhf_toeplitz3_generators(self, gen_H, gen_S):
        _check(load().lhf_toeplitz3_generators(self.handle, _ptr(gen_H), _ptr(gen_S)))

    def lhf_toeplitz_blocks(self, gen_H=None, gen_S=None, cross_km=None, cross_H=None, cross_S=None):
        _check(load().lhf_toeplitz_blocks(self.handle, _ptr(gen_H), _ptr(gen_S), _ptr(cross_km), _ptr(cross_H),
                                          _ptr(cross_S)))

    def matvec_workspace(self, ncols, device="cuda"):
        import torch
        n = int(load().lhf_toeplitz_matvec_workspace(self.handle, ncols))
        return torch.empty(max(1, n), dtype=torch.uint8, device=device)

    def lhf_toeplitz_matvec(self, prec, x, y_H, y_S, ws):
        ncols = x.shape[1]
        _check(load().lhf_toeplitz_matvec(self.handle, prec, ncols, _ptr(x), _ptr(y_H), _ptr(y_S), x.stride(0),
                                          _ptr(ws), ws.numel(), _stream()))

    def lhf_toeplitz_matvec_f32(self, x, y_H, y_S, ws):
        ncols = x.shape[1]
        _check(load().lhf_toeplitz_matvec_f32(self.handle, ncols, _ptr(x), _ptr(y_H), _ptr(y_S), x.stride(0),
                                              _ptr(ws), ws.numel(), _stream()))

    def eigs_workspace(self, nev, device="cuda"):
        import torch
        n = int(load().lhf_toeplitz_eigs_workspace(self.handle, nev))
        if n == 0:
            raise LhfError(LHF_ERR_INVALID, "unsupported nev")
        return torch.empty(n, dtype=torch.uint8, device=device)

    def lhf_toeplitz_eigs(self, nev, w, V=None, maxit=200, tol=1e-6, seed=1, ws=None):
        ws = ws if ws is not None else self.eigs_workspace(nev, w.device)
        it = C.c_int32()
        res = C.c_double()
        _check(load().lhf_toeplitz_eigs(self.handle, nev, maxit, tol, seed, _ptr(w), _ptr(V), C.byref(it),
                                        C.byref(res), _ptr(ws), ws.numel(), _stream()))
        return it.value, res.value
