"""The dense Rayleigh-Ritz eigensolver of the block LOBPCG (lhf_dense_syev)
through the C ABI, on matrices with known spectra.

Each matrix is Q diag(lam) Q^T with a random orthogonal Q, so its
eigenvalues are lam exactly, by construction.  The spectra carry exact
degeneracies, clusters split by 1e-9 and 1e-6, a dense band (eigenvalues
2e-4 apart, as the Ritz values of a chain's lowest band), a diagonal matrix
(every coupling of the tridiagonal form zero) and a matrix with two decoupled
blocks and an 8-fold eigenvalue across the boundary of two chunks of the
inverse iteration (40 vectors), at sizes from 1 to the maximum, with k from 1
to m.

Tolerances (from the arithmetic): eigenvalues within 1e-12 of |A| (bisection
to a few ulps, Householder backward error ~ m eps |A|); residuals
|A z - lambda z| within 1e-11 |A|; the vectors orthonormal to 1e-9 (vectors of
eigenvalues closer than 1e-8 |A| are orthogonalised; the others are
orthogonal to about eps |A| / gap).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1702_00339_amd import lhf  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lhf.load()
    torch.cuda.set_device(0)


def _spectrum(kind, m, rng):
    if kind == "random":
        return np.sort(rng.uniform(-3.0, 5.0, m))
    if kind == "degenerate":
        base = np.repeat([-2.0, -1.0, 0.5], [4, 3, 5])[:m]
        return np.sort(np.concatenate([base, rng.uniform(1.0, 5.0, m - len(base))]))
    if kind == "clusters":
        base = np.concatenate([-1.0 + 1e-9 * np.arange(6), -0.5 + 1e-6 * np.arange(5)])[:m]
        return np.sort(np.concatenate([base, rng.uniform(0.0, 5.0, m - len(base))]))
    if kind == "straddle":
        base = np.concatenate([rng.uniform(-4.0, -1.0, 36), np.full(8, 0.25)])[:m]
        return np.sort(np.concatenate([base, rng.uniform(1.0, 5.0, m - len(base))]))
    if kind == "band":
        nb = min(m, 40)
        base = -15.0 + 2e-4 * np.arange(nb) + 1e-5 * rng.standard_normal(nb)
        return np.sort(np.concatenate([base, rng.uniform(-5.0, 40.0, m - nb)]))
    raise ValueError(kind)


def _matrix(kind, m, rng):
    if kind == "diagonal":
        lam = rng.uniform(-3.0, 3.0, m)
        return np.diag(lam), np.sort(lam)
    if kind == "blocks":
        h = m // 2
        A = np.zeros((m, m))
        for lo, hi in ((0, h), (h, m)):
            Q, _ = np.linalg.qr(rng.standard_normal((hi - lo, hi - lo)))
            A[lo:hi, lo:hi] = (Q * rng.uniform(-2.0, 2.0, hi - lo)) @ Q.T
        A = 0.5 * (A + A.T)
        return A, np.linalg.eigvalsh(A)
    lam = _spectrum(kind, m, rng)
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), lam


CASES = [("random", 108, 36), ("degenerate", 108, 36), ("clusters", 72, 36), ("band", 108, 36),
         ("diagonal", 108, 36), ("blocks", 96, 48), ("random", 112, 112), ("degenerate", 40, 40),
         ("random", 1, 1), ("random", 2, 2), ("random", 3, 1), ("random", 9, 5), ("band", 33, 33),
         ("straddle", 100, 60), ("random", 112, 41)]


@pytest.mark.parametrize("kind,m,k", CASES, ids=lambda v: str(v))
def test_known_spectra(kind, m, k):
    rng = np.random.default_rng(m * 31 + k + len(kind))
    A, lam = _matrix(kind, m, rng)
    lda, ldv = m + 3, k + 2
    Ad = torch.zeros((m, lda), dtype=torch.float64, device="cuda")
    Ad[:, :m] = torch.from_numpy(A)
    w = torch.empty(k, dtype=torch.float64, device="cuda")
    V = torch.full((m, ldv), float("nan"), dtype=torch.float64, device="cuda")
    lhf.lhf_dense_syev(m, k, Ad, lda, w, V, ldv)
    torch.cuda.synchronize()
    got = w.cpu().numpy()
    Z = V[:, :k].cpu().numpy()
    nrm = max(np.abs(lam).max(), 1e-300)
    assert np.abs(got - lam[:k]).max() <= 1e-12 * nrm, np.abs(got - lam[:k]).max()
    assert np.all(np.diff(got) >= 0)
    assert np.abs(A @ Z - Z * got).max() <= 1e-11 * nrm
    assert np.abs(Z.T @ Z - np.eye(k)).max() <= 1e-9
    assert torch.isnan(V[:, k:]).all()   # columns beyond k untouched


def test_rejects_bad_sizes():
    A = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    w = torch.empty(4, dtype=torch.float64, device="cuda")
    V = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    for m, k, lda, ldv in ((4, 5, 4, 4), (0, 0, 4, 4), (113, 1, 113, 4), (4, 2, 3, 4), (4, 4, 4, 3)):
        with pytest.raises(lhf.LhfError):
            lhf.lhf_dense_syev(m, k, A, lda, w, V, ldv)
