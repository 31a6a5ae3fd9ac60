"""Grids, basis factors, 1D FEM matrices, sinc rule and potential factors.

TEST INFRASTRUCTURE (part of the CPU oracle; see the package docstring).

Paper passages followed:
  * Sec. 2.1 (eqs. HFcore, ElectrostPot, Core_Ham): H = -1/2 Laplacian - v_c,
    v_c = sum_nu Z_nu / |x - a_nu|, Galerkin pair (H, S).
  * Sec. 2.2 (eqs. galten, sinc_general): collocation of the Newton kernel on
    piecewise-constant cells, 1/z ~ sum_q w_q exp(-t_q^2 z^2).
  * Sec. 2.3 (eqs. EwaldSumE, EwaldTensorGl): lattice sums of the kernel.
  * Sec. 3.3 (eq. EwaldSumP): periodic case, potential summed at the central
    cell and replicated to every cell.
  * Sec. 2.4: 1D FEM stiffness (1/h) tridiag(-1, 2, -1) and mass
    (h/6) tridiag(1, 4, 1) on hat functions; nodal interpolation of the
    Gaussians; 3D operators as Kronecker sums.

Readings where the paper is silent or ambiguous:
  R1 one node set per dimension; the potential's piecewise-constant cells are
     the dual cells [x_i - h/2, x_i + h/2] of the FEM nodes.
  R2 periodic dimension (periodic boundary and L >= 2): nodes x_i = i h,
     i = 0..n-1, h = L a / n, n a multiple of L; cell k is [k a, (k+1) a) with
     centre (k + 1/2) a.  Box dimension: width W = L a + 2 pad, nodes
     x_i = -W/2 + i h, i = 1..n, h = W / (n + 1), zero Dirichlet values
     outside; cell k has centre -L a / 2 + (k + 1/2) a.
  R3 basis functions are normalised 1D primitives N (x-c)^l exp(-alpha (x-c)^2)
     per dimension, l in {0, 1}; on periodic dimensions they are periodised
     (summed over all translates by the supercell length).
  R4 lattice window (periodic or multi-cell dimensions): the images of a
     nucleus summed for the central cell are the L cells centred on it; odd L:
     k in [-(L-1)/2, (L-1)/2]; even L: k in [-L/2, L/2] with weight 1/2 on the
     two end images.  The sum is evaluated on the central cell's nodes and
     replicated to every cell.  One-cell dimensions use the cell's own nucleus.
  R5 sinc rule: t = exp(u), trapezoid in u: t_q = exp(u0 + q step),
     w_q = (2 / sqrt(pi)) step t_q, q = 0..R-1.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
from scipy.special import erf, erfc


# ----------------------------------------------------------------------------- grids

@dataclasses.dataclass
class Grid1D:
    periodic: bool
    L: int
    n: int
    a: float
    h: float
    x: np.ndarray            # [n] node coordinates
    centres: np.ndarray      # [L] cell centres
    period: float            # supercell length (periodic dims), 0 otherwise


def grid_1d(inst, ell: int) -> Grid1D:
    """Node set of dimension ``ell`` (reading R2)."""
    L, n, a = inst.L[ell], inst.n[ell], inst.a
    periodic = inst.bc == "periodic" and L >= 2
    if periodic:
        if n % L != 0:
            raise ValueError("periodic dimension needs n to be a multiple of L")
        h = L * a / n
        x = np.arange(n, dtype=np.float64) * h
        centres = (np.arange(L) + 0.5) * a
        return Grid1D(True, L, n, a, h, x, centres, L * a)
    W = L * a + 2.0 * inst.pad[ell]
    h = W / (n + 1)
    x = -0.5 * W + np.arange(1, n + 1, dtype=np.float64) * h
    centres = -0.5 * L * a + (np.arange(L) + 0.5) * a
    return Grid1D(False, L, n, a, h, x, centres, 0.0)


def grids(inst):
    return [grid_1d(inst, ell) for ell in range(3)]


# ----------------------------------------------------------------------------- basis

def gto_norm(alpha, l):
    """Normalisation of N (x-c)^l exp(-alpha (x-c)^2) on the real line (R3)."""
    base = (2.0 * alpha / math.pi) ** 0.25
    return base if l == 0 else base * 2.0 * math.sqrt(alpha)


def gto_1d(x, alpha, l, c):
    """One normalised 1D Gaussian primitive at points x."""
    d = x - c
    v = gto_norm(alpha, l) * np.exp(-alpha * d * d)
    return v * d if l == 1 else v


def image_range(g: Grid1D, alpha: float) -> int:
    """Number of periodic images each side needed before exp underflows."""
    if not g.periodic:
        return 0
    reach = math.sqrt(800.0 / alpha)
    return int(math.ceil(reach / g.period)) + 1


def angular_power(ang: int, ell: int) -> int:
    return 1 if ang == ell + 1 else 0


def nodal_factor(inst, g: Grid1D, ell: int, mu: int, cell: int) -> np.ndarray:
    """Nodal values of the dimension-ell factor of basis function mu of cell
    ``cell`` (periodised on periodic dimensions), Sec. 2.4 interpolant."""
    alpha = float(inst.alpha[mu])
    l = angular_power(int(inst.ang[mu]), ell)
    c = g.centres[cell] + inst.centre[mu, ell]
    if not g.periodic:
        return gto_1d(g.x, alpha, l, c)
    S = image_range(g, alpha)
    out = np.zeros(g.n)
    for s in range(-S, S + 1):
        out += gto_1d(g.x, alpha, l, c + s * g.period)
    return out


# ----------------------------------------------------------------------------- FEM

def fem_1d(g: Grid1D):
    """1D stiffness A = (1/h) tridiag(-1, 2, -1) and mass S = (h/6) tridiag(1, 4, 1)
    on the hat functions of the node set (Sec. 2.4); cyclic on periodic dims,
    truncated (zero Dirichlet values) on box dims."""
    n, h = g.n, g.h
    main = np.ones(n)
    off = np.ones(n - 1)
    A = sp.diags([-off, 2 * main, -off], [-1, 0, 1], format="lil")
    S = sp.diags([off, 4 * main, off], [-1, 0, 1], format="lil")
    if g.periodic:
        A[0, n - 1] = -1.0
        A[n - 1, 0] = -1.0
        S[0, n - 1] = 1.0
        S[n - 1, 0] = 1.0
    return (A.tocsr() / h), (S.tocsr() * (h / 6.0))


# ----------------------------------------------------------------------------- sinc rule

def sinc_rule(inst):
    """Nodes t_q and weights w_q with 1/r ~ sum_q w_q exp(-t_q^2 r^2) (R5)."""
    q = np.arange(inst.R, dtype=np.float64)
    t = np.exp(inst.sinc_u0 + q * inst.sinc_step)
    w = (2.0 / math.sqrt(math.pi)) * inst.sinc_step * t
    return t, w


# ----------------------------------------------------------------------------- potential

def cell_integral_gauss(x, h, t, A):
    """phi(x) = integral over [x - h/2, x + h/2] of exp(-t^2 (y - A)^2) dy.

    Collocation of one Gaussian term of the kernel on the piecewise-constant
    cell of node x (eq. galten, one dimension).  With u = t h and v = t (x - A):
      * u <= 0.1 and u |v| <= 0.1: the midpoint expansion
          phi = h exp(-v^2) sum_k u^(2k) H_2k(v) / (4^k (2k+1)!),  k = 0..4
        (H_n physicists' Hermite polynomials; the next term is below 1e-17
        relative), because the erf difference cancels when the cell is much
        narrower than the Gaussian;
      * otherwise sqrt(pi) / (2 t) times the difference of erf, or of erfc on
        the far side of A so that the difference does not cancel."""
    x = np.asarray(x, dtype=np.float64)
    u = t * h
    v = t * (x - A)
    out = np.empty_like(v)
    ser = (u <= 0.1) & (u * np.abs(v) <= 0.1)
    if np.any(ser):
        v2 = v[ser] ** 2
        u2 = u * u
        H2 = 4 * v2 - 2
        H4 = (16 * v2 - 48) * v2 + 12
        H6 = ((64 * v2 - 480) * v2 + 720) * v2 - 120
        H8 = (((256 * v2 - 3584) * v2 + 13440) * v2 - 13440) * v2 + 1680
        series = 1 + u2 * (H2 / 24 + u2 * (H4 / 1920 + u2 * (H6 / 322560 + u2 * H8 / 92897280)))
        out[ser] = h * np.exp(-v2) * series
    rest = ~ser
    lo = t * (x[rest] - 0.5 * h - A)
    hi = t * (x[rest] + 0.5 * h - A)
    val = np.empty_like(lo)
    right = lo > 0
    left = hi < 0
    mid = ~(right | left)
    val[right] = erfc(lo[right]) - erfc(hi[right])
    val[left] = erfc(-hi[left]) - erfc(-lo[left])
    val[mid] = erf(hi[mid]) - erf(lo[mid])
    out[rest] = val * (math.sqrt(math.pi) / (2.0 * t))
    return out


def window(L: int):
    """Image offsets and weights of the lattice window (R4)."""
    if L <= 1:
        return np.zeros(1, np.int64), np.ones(1)
    if L % 2 == 1:
        k = np.arange(-(L - 1) // 2, (L - 1) // 2 + 1)
        return k, np.ones(len(k))
    k = np.arange(-L // 2, L // 2 + 1)
    w = np.ones(len(k))
    w[0] = w[-1] = 0.5
    return k, w


def central_offsets(g: Grid1D):
    """Positions of the nodes relative to the centre of the cell that holds
    them, and that cell's index, for every node."""
    if g.periodic:
        cell = np.floor(g.x / g.a).astype(np.int64)
    else:
        cell = np.floor((g.x + 0.5 * g.L * g.a) / g.a).astype(np.int64)
    cell = np.clip(cell, 0, g.L - 1)
    return g.x - g.centres[cell], cell


def potential_factor(inst, g: Grid1D, ell: int, nu: int, t: float) -> np.ndarray:
    """Dimension-ell factor of the lattice-summed collocated potential of
    nucleus nu for one sinc node t, on every node (eqs. EwaldTensorGl and
    EwaldSumP, readings R4)."""
    A = float(inst.nuc[nu, ell])
    if g.L == 1:
        return cell_integral_gauss(g.x, g.h, t, g.centres[0] + A)
    y, _ = central_offsets(g)
    ks, wk = window(g.L)
    out = np.zeros(g.n)
    for k, w in zip(ks, wk):
        out += w * cell_integral_gauss(y, g.h, t, A + k * g.a)
    return out
