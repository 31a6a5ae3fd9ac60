"""Seeded synthetic lattice instances (inputs only, no method arithmetic).

An instance describes one lattice system of the core-Hamiltonian problem
(paper Sec. 2.1 and 2.3): an L1 x L2 x L3 lattice of identical unit cells of
step ``a`` (bohr), each cell carrying m0 Gaussian basis functions (exponent,
centre relative to the cell centre, angular type) and M0 nuclei (charge,
position relative to the cell centre); the grid size n per dimension; the
boundary condition; and the two parameters (u0, step) of the exponential-
substitution sinc rule that approximates 1/r by R Gaussians (paper Sec. 2.2,
eq. ``sinc_general``; the paper does not print its nodes, so they are inputs).

The paper's own workloads are hydrogen-type chains with an unstated basis;
these seeded lattices stand in for them.  Random draws use
``numpy.random.Generator(PCG64(seed))`` in a fixed, documented order:
  1. shell exponents, log-uniform in [lo, hi], one per shell;
  2. shell centre jitter, uniform in [-j, j]^3, one per shell;
  3. the nuclear charge (integer, uniform), when a range is given;
  4. (Dirichlet chains with defects) defect cells, their charges and their
     exponent scale factors.
s shells give one function, p shells three (px, py, pz) sharing exponent and
centre.  Units: bohr, hartree.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Angular types of one basis function: power 1 of the coordinate in the
# indicated dimension, power 0 in the others.
ANG_S, ANG_PX, ANG_PY, ANG_PZ = 0, 1, 2, 3

CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


@dataclasses.dataclass
class Instance:
    name: str
    L: Tuple[int, int, int]
    n: Tuple[int, int, int]
    a: float
    pad: Tuple[float, float, float]
    bc: str                       # "periodic" or "dirichlet"
    alpha: np.ndarray             # [m0] exponents (bohr^-2)
    centre: np.ndarray            # [m0, 3] centres relative to the cell centre
    ang: np.ndarray               # [m0] angular type (ANG_*)
    Z: np.ndarray                 # [M0] nuclear charges
    nuc: np.ndarray               # [M0, 3] nuclear positions relative to the cell centre
    R: int                        # number of sinc terms
    sinc_u0: float                # first node is exp(u0)
    sinc_step: float              # node spacing in u = log t
    seed: int = 0
    # Dirichlet chains with defect cells (empty for pristine lattices)
    def_cells: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    def_Z: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))
    def_scale: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))

    @property
    def m0(self) -> int:
        return int(self.alpha.shape[0])

    @property
    def M0(self) -> int:
        return int(self.Z.shape[0])

    @property
    def ncells(self) -> int:
        return int(self.L[0] * self.L[1] * self.L[2])

    def summary(self) -> str:
        return (f"{self.name}: L={self.L} n={self.n} m0={self.m0} R={self.R} "
                f"bc={self.bc} Z={self.Z.tolist()} seed={self.seed}")


def _sinc_params(L, n, a, pad, bc, R, eps=1e-4):
    """Pick (u0, step) of the sinc rule for distances in [rho_min, rho_max].

    rho_min is half the smallest grid spacing, rho_max the diagonal of the
    region the lattice window covers.  The lower end of the u range is set so
    that the truncated left tail of the integral is ~eps relative at rho_max,
    the upper end so that exp(-rho_min^2 t^2) < 1e-15 there.  This only picks
    inputs; its accuracy (model error) is reported by the oracle tests.
    """
    spans, hs = [], []
    for ell in range(3):
        periodic = bc == "periodic" and L[ell] >= 2
        if periodic:
            hs.append(a * L[ell] / n[ell])
            spans.append(a * (L[ell] + 1))
        else:
            w = a * L[ell] + 2.0 * pad[ell]
            hs.append(w / (n[ell] + 1))
            spans.append(w)
    rho_min = 0.5 * min(hs)
    rho_max = math.sqrt(sum(s * s for s in spans))
    u_lo = math.log(eps * math.sqrt(math.pi) / (2.0 * rho_max))
    u_hi = math.log(6.0 / rho_min)
    step = (u_hi - u_lo) / (R - 1)
    return u_lo, step


def make_instance(*, name: str, L: Sequence[int], n: Sequence[int], a: float = 5.0,
                  pad: Sequence[float] = (6.0, 6.0, 6.0), bc: str = "periodic",
                  n_s: int = 4, n_p: int = 0, exp_range=(0.2, 8.0),
                  Z=1, R: int = 20, seed: int = 0, jitter: float = 0.3,
                  ndefect: int = 0, defect_seed: Optional[int] = None) -> Instance:
    """Draw one instance.  ``Z`` is an int (fixed) or a (lo, hi) inclusive range."""
    L = tuple(int(x) for x in L)
    n = tuple(int(x) for x in n)
    pad = tuple(float(x) for x in pad)
    assert bc in ("periodic", "dirichlet")
    rng = np.random.Generator(np.random.PCG64(seed))
    nsh = n_s + n_p
    lo, hi = exp_range
    sh_exp = np.exp(rng.uniform(math.log(lo), math.log(hi), nsh))
    sh_jit = rng.uniform(-jitter, jitter, (nsh, 3))
    if isinstance(Z, (tuple, list)):
        zval = float(rng.integers(Z[0], Z[1] + 1))
    else:
        zval = float(Z)
    alpha, centre, ang = [], [], []
    for s in range(nsh):
        if s < n_s:
            alpha.append(sh_exp[s]); centre.append(sh_jit[s]); ang.append(ANG_S)
        else:
            for t in (ANG_PX, ANG_PY, ANG_PZ):
                alpha.append(sh_exp[s]); centre.append(sh_jit[s]); ang.append(t)
    u0, step = _sinc_params(L, n, a, pad, bc, R)
    inst = Instance(name=name, L=L, n=n, a=float(a), pad=pad, bc=bc,
                    alpha=np.asarray(alpha, np.float64),
                    centre=np.asarray(centre, np.float64).reshape(-1, 3),
                    ang=np.asarray(ang, np.int8),
                    Z=np.asarray([zval], np.float64), nuc=np.zeros((1, 3)),
                    R=int(R), sinc_u0=u0, sinc_step=step, seed=seed)
    if ndefect > 0:
        drng = np.random.Generator(np.random.PCG64(defect_seed if defect_seed is not None else seed + 1))
        ncell = L[0] * L[1] * L[2]
        cells = np.sort(drng.permutation(ncell)[:ndefect])
        choices = [z for z in range(1, 7) if z != int(zval)]
        dz = np.asarray([choices[i] for i in drng.integers(0, len(choices), ndefect)], np.float64)
        dscale = np.exp(drng.uniform(math.log(0.5), math.log(2.0), ndefect))
        inst.def_cells, inst.def_Z, inst.def_scale = cells.astype(np.int64), dz, dscale
    return inst


def make_config(name: str, **over) -> Instance:
    """The single-lattice workloads.

    c1  periodic 8x1x1 chain, m0=4 s, n=128^3, R=20, Z=1      (dense-check case)
    c2  periodic 256x1x1 tube, m0=16 (4 s + 4 p shells), n=2048x256x256, R=30
    c3  periodic 32x32x32, m0=8 s, n=512^3, R=24
    c5  Dirichlet 512x1x1 chain, m0=16, n=4096x256x256, R=30, 26 defect cells
    """
    if name == "c1":
        kw = dict(name="c1", L=(8, 1, 1), n=(128, 128, 128), n_s=4, n_p=0,
                  exp_range=(0.2, 8.0), Z=1, R=20, seed=1)
    elif name == "c2":
        kw = dict(name="c2", L=(256, 1, 1), n=(2048, 256, 256), n_s=4, n_p=4,
                  exp_range=(0.1, 10.0), Z=(1, 6), R=30, seed=2)
    elif name == "c3":
        kw = dict(name="c3", L=(32, 32, 32), n=(512, 512, 512), n_s=8, n_p=0,
                  exp_range=(0.2, 8.0), Z=(1, 3), R=24, seed=3)
    elif name == "c5":
        nc = 8
        kw = dict(name="c5", L=(512, 1, 1), n=(4096, 256, 256), bc="dirichlet",
                  pad=(5.0 / (2 * nc), 6.0, 6.0), n_s=4, n_p=4,
                  exp_range=(0.1, 10.0), Z=(1, 6), R=30, seed=5,
                  ndefect=26, defect_seed=5000)
    else:
        raise ValueError(f"unknown single-lattice config {name!r}")
    kw.update(over)
    return make_instance(**kw)


def config_c4_lattices(count: int = 64, base_seed: int = 4000) -> List[Instance]:
    """The batched mix: ``count`` independent periodic lattices.

    Per lattice i (seed base_seed + i, drawn first from a separate stream):
    L1 ~ U{16..512}, L2, L3 ~ U{1, 2, 4}, m0 ~ U{4, 8, 16, 32};
    n = 16 L for periodic dimensions, 128 for one-cell (tube) dimensions;
    R = 24; m0 <= 8: all s, exponents log-U[0.2, 8], Z ~ U{1..3};
    m0 >= 16: m0/4 s + m0/4 p shells, exponents log-U[0.1, 10], Z ~ U{1..6}.
    """
    out = []
    for i in range(count):
        seed = base_seed + i
        srng = np.random.Generator(np.random.PCG64(seed + 100000))
        L1 = int(srng.integers(16, 513))
        L2 = int(srng.choice([1, 2, 4]))
        L3 = int(srng.choice([1, 2, 4]))
        m0 = int(srng.choice([4, 8, 16, 32]))
        L = (L1, L2, L3)
        n = tuple(16 * x if x >= 2 else 128 for x in L)
        if m0 <= 8:
            kw = dict(n_s=m0, n_p=0, exp_range=(0.2, 8.0), Z=(1, 3))
        else:
            kw = dict(n_s=m0 // 4, n_p=m0 // 4, exp_range=(0.1, 10.0), Z=(1, 6))
        out.append(make_instance(name=f"c4_{i:02d}", L=L, n=n, R=24, seed=seed, **kw))
    return out


def tiny_instance(L=(4, 1, 1), n=(32, 24, 24), n_s=2, n_p=0, seed=11, R=8,
                  exp_range=(0.3, 3.0), Z=(1, 3), bc="periodic", a=5.0,
                  pad=(4.0, 4.0, 4.0), jitter=0.3, **kw) -> Instance:
    """A small lattice for oracle pins and GPU parity cases."""
    return make_instance(name=f"tiny_L{'x'.join(map(str, L))}_n{'x'.join(map(str, n))}_s{seed}",
                         L=L, n=n, n_s=n_s, n_p=n_p, seed=seed, R=R, exp_range=exp_range,
                         Z=Z, bc=bc, a=a, pad=pad, jitter=jitter, **kw)
