"""Pin of the oracle's lattice window (reading R4; Sec. 3.3, eq. EwaldSumP).

Reading R4: on a periodic dimension the potential of a nucleus is summed, at
the nodes of the central cell, over the images in the L cells centred on that
cell, and the sum is replicated to every cell.  Odd L: the (L - 1) / 2 cells
on either side.  Even L: L / 2 - 1 cells on either side at full weight, plus
the two cells at distance L / 2, each at half weight.

The check here builds that image set by a different route from the oracle's
``window`` function: it takes the cells nearest the central cell one distance
shell at a time until L cells of weight are used up, and the shell that does
not fit whole shares what is left equally among its cells.  Every image term
is evaluated as an erf difference at 60 significant digits.  The sinc nodes
are slowly decaying (t = 0.05 and 0.1 bohr^-1), so the two end images carry
between 1e-2 and 1 of the central image's weight.  A one-sided even-L window,
full end weights, or an odd-L off-by-one range therefore fails, and the last
test plants each of these in the oracle to show it.
"""

import math

import numpy as np
import pytest

from oracle import model
from synth import make_instance


def nearest_cells_window(L):
    """(offsets, weights): the L cells nearest the central one, ties at the
    last distance sharing the remaining weight equally."""
    if L <= 1:
        return [0], [1.0]
    left = float(L)
    out_k, out_w = [], []
    for dist in range(0, L + 1):
        shell = [0] if dist == 0 else [-dist, dist]
        take = min(1.0, left / len(shell))
        if take <= 0.0:
            break
        for k in shell:
            out_k.append(k)
            out_w.append(take)
        left -= take * len(shell)
    return out_k, out_w


def cell_integral_mp(x, h, t, A, mpmath):
    X, H, T, AA = (mpmath.mpf(v) for v in (x, h, t, A))
    return mpmath.sqrt(mpmath.pi) / (2 * T) * (mpmath.erf(T * (X + H / 2 - AA)) - mpmath.erf(T * (X - H / 2 - AA)))


def _chain(L, nc, nuc_x, t):
    inst = make_instance(name="win", L=(L, 1, 1), n=(L * nc, 6, 6), a=5.0, bc="periodic",
                         pad=(6.0, 3.0, 3.0), n_s=1, n_p=0, R=2, seed=3)
    inst.nuc[0, 0] = nuc_x
    inst.sinc_u0 = math.log(t)
    inst.sinc_step = 1.0
    return inst


@pytest.mark.parametrize("L", list(range(1, 10)))
def test_window_weights_match_nearest_cells(L):
    ks, wk = model.window(L)
    got = sorted(zip(ks.tolist(), wk.tolist()))
    ref = sorted(zip(*nearest_cells_window(L)))
    assert got == ref, (L, got, ref)
    assert abs(sum(wk) - L) < 1e-15 or (L == 1 and abs(sum(wk) - 1.0) < 1e-15)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("t", [0.05, 0.1])
@pytest.mark.parametrize("nuc_x", [0.0, 0.7])
def test_potential_factor_window_vs_brute_force(L, t, nuc_x):
    """potential_factor at every node equals the image sum over the nearest-L
    window, each image's cell integral taken at 60 digits, to 1e-13."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    nc = 10
    inst = _chain(L, nc, nuc_x, t)
    g = model.grid_1d(inst, 0)
    got = model.potential_factor(inst, g, 0, 0, t)
    ks, ws = nearest_cells_window(L)
    a, h = inst.a, g.h
    end = max(abs(k) for k in ks)
    ref = np.empty(g.n)
    end_share = 0.0
    for i, x in enumerate(g.x):
        c = int(math.floor(x / a + 1e-12))
        y = x - (c + 0.5) * a          # offset from the centre of the node's own cell
        terms = [w * cell_integral_mp(y, h, t, nuc_x + k * a, mpmath) for k, w in zip(ks, ws)]
        total = sum(terms)
        ref[i] = float(total)
        if L > 1:
            end_share = max(end_share, float(sum(tm for tm, k in zip(terms, ks) if abs(k) == end) / total))
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), np.abs(got - ref).max()
    if L > 1:
        # the end images weigh enough that a wrong end weight cannot hide
        assert end_share > 1e-3, end_share


@pytest.mark.parametrize("L", [4, 5, 6])
def test_potential_factor_mirror_symmetric_for_centred_nucleus(L):
    """A nucleus at the cell centre sees a window symmetric about it: node
    offsets y and -y of the central cell get the same value."""
    nc = 10
    inst = _chain(L, nc, 0.0, 0.07)
    g = model.grid_1d(inst, 0)
    P = model.potential_factor(inst, g, 0, 0, 0.07)
    cell0 = P[:nc]                       # offsets -a/2 + i h, i = 0..nc-1
    for i in range(1, nc):
        assert abs(cell0[i] - cell0[nc - i]) <= 1e-14 * abs(cell0[i]), (i, cell0[i], cell0[nc - i])
    # replicated: every cell carries the central cell's values
    for c in range(1, L):
        assert np.array_equal(P[c * nc:(c + 1) * nc], cell0)


def _one_sided(L):
    if L <= 1:
        return np.zeros(1, np.int64), np.ones(1)
    k = np.arange(-(L // 2), L - L // 2)
    return k, np.ones(len(k))


def _full_ends(L):
    k, _ = _ORIG_WINDOW(L)
    return k, np.ones(len(k))


def _odd_off_by_one(L):
    k, w = _ORIG_WINDOW(L)
    if L % 2 == 1 and L > 1:
        k = k + 1
    return k, w


_ORIG_WINDOW = model.window


@pytest.mark.parametrize("bad,L", [(_one_sided, 4), (_one_sided, 6), (_full_ends, 4), (_full_ends, 6),
                                   (_odd_off_by_one, 3), (_odd_off_by_one, 5)],
                         ids=["one-sided-4", "one-sided-6", "full-ends-4", "full-ends-6", "odd-shift-3", "odd-shift-5"])
def test_planted_window_mistakes_are_caught(monkeypatch, bad, L):
    """The brute-force check above fails for each plausible misreading of R4
    planted in the oracle."""
    monkeypatch.setattr(model, "window", bad)
    with pytest.raises(AssertionError):
        test_potential_factor_window_vs_brute_force(L, 0.05, 0.7)
    with pytest.raises(AssertionError):
        test_window_weights_match_nearest_cells(L)
