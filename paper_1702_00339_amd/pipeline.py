"""The periodic hot path on device buffers: assemble -> block DFT -> eigensolve.

``Pipeline`` owns the plan and every device buffer of one configuration and
runs one step with three (FP64) or four-plus (mixed) C-ABI calls on the
current torch stream.  All arithmetic happens in the HIP library.
"""

from __future__ import annotations

import torch

from . import lhf


class Pipeline:
    """prec: lhf.LHF_PREC_FP64 or lhf.LHF_PREC_MIXED.  For the mixed path
    ``refine_src`` picks where the FP64 refinement gets its blocks:
      "direct" (default) the assembly writes only the FP64 stacks, one FP64
              block DFT writes the complex128 blocks, and the FP32 solve
              reads them (rounding on load);
      "dual"  the assembly writes only the FP64 stacks and one FP64 block
              DFT writes the complex128 blocks and their complex64 copies
              for the FP32 solve;
      "bar64" FP32 stacks and a complex64 DFT for the FP32 solve, plus a
              separate complex128 DFT of the FP64 stacks;
      "band"  FP32 stacks and a complex64 DFT; refinement regenerates each
              block from the FP64 generator band.
    ``fourier`` picks how the complex128 Fourier blocks of FP64 plans and of
    the "direct" mixed path are made: "sep" separably from the FP64 Grams
    (lhf_fourier_blocks; no generator stacks are written), "dft" generator
    stacks and a block DFT, "auto" the plan's setting (separable where the
    plan qualifies; the autotuner may change it).  The choice is the plan's
    tuning field fourier_sep, which lhf_step follows as well.
    ``fp32_solve`` (mixed path): every size class takes the FP32 solve and
    the FP64 refinement (LHF_HEEV_FP32_SOLVE), never the FP64 solve alone."""

    def __init__(self, instances, prec=lhf.LHF_PREC_FP64, gram=lhf.LHF_GRAM_BF16X3, refine_src="auto",
                 want_vectors=False, device="cuda", L0=None, fourier="auto", fp32_solve=False):
        if not isinstance(instances, (list, tuple)):
            instances = [instances]
        self.plan = lhf.Plan(instances, prec=prec, gram=gram if prec == lhf.LHF_PREC_MIXED else lhf.LHF_GRAM_FP64,
                             L0=L0)
        sz = self.plan.sizes
        self.prec = prec
        self.sizes = sz
        dev = torch.device(device)
        G, B = int(sz.gen_elems), int(sz.nblocks)
        rdt = torch.float64 if prec == lhf.LHF_PREC_FP64 else torch.float32
        cdt = torch.complex128 if prec == lhf.LHF_PREC_FP64 else torch.complex64
        self.ws = self.plan.workspace(dev)
        self.H_gen = torch.empty(G, dtype=rdt, device=dev)
        self.S_gen = torch.empty(G, dtype=rdt, device=dev)
        self.H_bar = torch.empty(G, dtype=cdt, device=dev)
        self.S_bar = torch.empty(G, dtype=cdt, device=dev)
        self.grams64 = torch.empty(max(1, int(sz.grams_elems)), dtype=torch.float64, device=dev)
        self.w = torch.empty(int(sz.w_elems), dtype=torch.float64, device=dev)
        self.info = torch.empty(B, dtype=torch.int32, device=dev)
        self.want_vectors = want_vectors
        self.fp32_solve = bool(fp32_solve) and prec == lhf.LHF_PREC_MIXED
        self.V = None
        if want_vectors:
            # FP64 solves and refined mixed solves both return complex128 vectors
            self.V = torch.empty(G, dtype=torch.complex128, device=dev)
        self.H_gen64 = self.S_gen64 = self.H_bar64 = self.S_bar64 = None
        if prec == lhf.LHF_PREC_MIXED:
            if refine_src == "auto":
                refine_src = "direct"
            assert refine_src in ("direct", "dual", "bar64", "band")
            self.refine_src = refine_src
            self.H_gen64 = torch.empty(G, dtype=torch.float64, device=dev)
            self.S_gen64 = torch.empty(G, dtype=torch.float64, device=dev)
            if refine_src in ("bar64", "dual", "direct"):
                self.H_bar64 = torch.empty(G, dtype=torch.complex128, device=dev)
                self.S_bar64 = torch.empty(G, dtype=torch.complex128, device=dev)
        else:
            self.refine_src = None
        assert fourier in ("auto", "sep", "dft")
        if fourier != "auto":
            t = self.plan.lhf_plan_get_tuning()
            t.fourier_sep = 1 if fourier == "sep" else 0
            self.plan.lhf_plan_set_tuning(t)
            if fourier == "sep" and self.plan.lhf_plan_get_tuning().fourier_sep != 1:
                raise ValueError("this plan does not qualify for the separable Fourier blocks")

    def separable(self):
        """Whether a step forms the complex128 blocks separably (as lhf_step does)."""
        if self.prec == lhf.LHF_PREC_MIXED and self.refine_src != "direct":
            return False
        return self.plan.lhf_plan_get_tuning().fourier_sep == 1

    def step_args(self):
        """The lhf_step_args of this pipeline's buffers (kept alive by self)."""
        def ptr(t):
            return None if t is None else t.data_ptr()

        flags = lhf.LHF_HEEV_VECTORS if self.want_vectors else 0
        if self.prec == lhf.LHF_PREC_MIXED:
            flags |= lhf.LHF_HEEV_REFINE_FP64
        if self.fp32_solve:
            flags |= lhf.LHF_HEEV_FP32_SOLVE
        dual = self.prec == lhf.LHF_PREC_MIXED and self.refine_src in ("dual", "direct")
        direct = self.prec == lhf.LHF_PREC_MIXED and self.refine_src == "direct"
        return lhf.lhf_step_args(None if dual else ptr(self.H_gen), None if dual else ptr(self.S_gen),
                                 ptr(self.grams64), ptr(self.H_gen64), ptr(self.S_gen64),
                                 None if direct else ptr(self.H_bar), None if direct else ptr(self.S_bar),
                                 ptr(self.H_bar64),
                                 ptr(self.S_bar64), ptr(self.w), ptr(self.V), ptr(self.info), ptr(self.ws),
                                 self.ws.numel(), flags)

    def step_native(self):
        """One step through the single lhf_step call."""
        self.plan.lhf_step(self.step_args())

    def capture(self):
        """A hipGraph of one step over this pipeline's buffers (lhf.Graph)."""
        return self.plan.lhf_graph_create(self.step_args())

    def autotune(self, cache_path=None):
        return self.plan.lhf_plan_autotune(self.step_args(), cache_path)

    def stages(self):
        """The step's C-ABI calls in order, as (name, callable) pairs: "assemble",
        "fourier" (block DFT or separable formation; for the mixed "bar64"
        route a second, FP64, transform "fourier64") and "eigensolve"."""
        p = self.plan
        sep = self.separable()
        out = []
        if self.prec == lhf.LHF_PREC_FP64:
            if sep:
                out.append(("assemble", lambda: p.lhf_assemble_blocks(None, None, self.grams64, self.ws)))
                out.append(("fourier", lambda: p.lhf_fourier_blocks(self.grams64, self.H_bar, self.S_bar, self.ws)))
            else:
                out.append(("assemble", lambda: p.lhf_assemble_blocks(self.H_gen, self.S_gen, self.grams64, self.ws)))
                out.append(("fourier", lambda: p.lhf_block_fft(lhf.LHF_PREC_FP64, self.H_gen, self.S_gen, self.H_bar,
                                                               self.S_bar, self.ws)))
            flags = lhf.LHF_HEEV_VECTORS if self.want_vectors else 0
            out.append(("eigensolve", lambda: p.lhf_heev_batched(flags, self.H_bar, self.S_bar, self.w, self.info,
                                                                 self.ws, V=self.V)))
            return out
        if self.refine_src == "direct" and sep:
            out.append(("assemble", lambda: p.lhf_assemble_blocks(None, None, self.grams64, self.ws)))
            out.append(("fourier", lambda: p.lhf_fourier_blocks(self.grams64, self.H_bar64, self.S_bar64, self.ws)))
        elif self.refine_src == "direct":
            out.append(("assemble", lambda: p.lhf_assemble_blocks(None, None, self.grams64, self.ws,
                                                                  H_gen64=self.H_gen64, S_gen64=self.S_gen64)))
            out.append(("fourier", lambda: p.lhf_block_fft(lhf.LHF_PREC_FP64, self.H_gen64, self.S_gen64,
                                                           self.H_bar64, self.S_bar64, self.ws)))
        elif self.refine_src == "dual":
            out.append(("assemble", lambda: p.lhf_assemble_blocks(None, None, self.grams64, self.ws,
                                                                  H_gen64=self.H_gen64, S_gen64=self.S_gen64)))
            out.append(("fourier", lambda: p.lhf_block_fft_dual(self.H_gen64, self.S_gen64, self.H_bar64,
                                                                self.S_bar64, self.H_bar, self.S_bar, self.ws)))
        else:
            out.append(("assemble", lambda: p.lhf_assemble_blocks(self.H_gen, self.S_gen, self.grams64, self.ws,
                                                                  H_gen64=self.H_gen64, S_gen64=self.S_gen64)))
            out.append(("fourier", lambda: p.lhf_block_fft(lhf.LHF_PREC_MIXED, self.H_gen, self.S_gen, self.H_bar,
                                                           self.S_bar, self.ws)))
        if self.refine_src == "bar64":
            out.append(("fourier64", lambda: p.lhf_block_fft(lhf.LHF_PREC_FP64, self.H_gen64, self.S_gen64,
                                                              self.H_bar64, self.S_bar64, self.ws)))
        flags = lhf.LHF_HEEV_REFINE_FP64 | (lhf.LHF_HEEV_VECTORS if self.want_vectors else 0)
        if self.fp32_solve:
            flags |= lhf.LHF_HEEV_FP32_SOLVE
        direct = self.refine_src == "direct"
        out.append(("eigensolve", lambda: p.lhf_heev_batched(
            flags, None if direct else self.H_bar, None if direct else self.S_bar, self.w, self.info, self.ws,
            V=self.V, H_bar64=self.H_bar64, S_bar64=self.S_bar64, H_gen64=self.H_gen64, S_gen64=self.S_gen64)))
        return out

    def step(self):
        """One step through the stage calls (lhf_assemble_blocks, the Fourier
        blocks, lhf_heev_batched)."""
        for _, fn in self.stages():
            fn()

    def eigenvalues(self):
        """Per-lattice eigenvalue arrays [L1, L2, L3, m0] on the host."""
        w = self.w.cpu().numpy()
        out, off = [], 0
        for inst in self.plan.instances:
            cnt = inst.ncells * inst.m0
            out.append(w[off:off + cnt].reshape(*inst.L, inst.m0))
            off += cnt
        return out

    def stacks(self, which="H_gen"):
        t = getattr(self, which).cpu().numpy()
        out, off = [], 0
        for inst in self.plan.instances:
            cnt = inst.ncells * inst.m0 * inst.m0
            out.append(t[off:off + cnt].reshape(*inst.L, inst.m0, inst.m0))
            off += cnt
        return out
