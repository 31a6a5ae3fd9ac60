"""Sturm counts of the FP64 bisection eigensolver, on the host.

The kernel's row recurrences (csrc/sturm.h) are compiled host-only by hipcc
and run here.  Split tridiagonal matrices (a zero subdiagonal entry, as
Householder reduction produces for a block-diagonal Hermitian matrix) with
shifts at eigenvalues of a leading block are where the plain product form
loses every later sign change; the kernel takes the restarting row for such
matrices and the plain one otherwise.  Away from eigenvalues a count must
equal the number of eigenvalues below the shift; at an eigenvalue either the
count below or the count at or below keeps bisection correct (the interval
still brackets it), anything else does not.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def sturm_bin(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("sturm") / "sturm_check")
    r = subprocess.run([HIPCC, "--offload-host-only", "-x", "hip", "-O2", "-std=c++17",
                        os.path.join(HERE, "sturm_check.cpp"), "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def run_counts(binary, cases):
    """cases: list of (d, e2, xs); per case an array [len(xs), 2] of the
    (restarting, plain) counts."""
    lines = [str(len(cases))]
    for d, e2, xs in cases:
        lines.append(str(len(d)))
        lines.append(" ".join(repr(float(v)) for v in d))
        lines.append(" ".join(repr(float(v)) for v in e2))
        lines.append(str(len(xs)))
        lines.append(" ".join(repr(float(v)) for v in xs))
    r = subprocess.run([binary], input="\n".join(lines) + "\n", capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    vals = np.array([int(v) for v in r.stdout.split()]).reshape(-1, 2)
    out, at = [], 0
    for _, _, xs in cases:
        out.append(vals[at:at + len(xs)])
        at += len(xs)
    return out


def _admissible(eig, x, got):
    return (eig < x).sum() <= got <= (eig <= x).sum()


def test_split_at_leading_pivot(sturm_bin):
    # d = (1.5, 1, 3), e = 0: at x = 1.5 the first minor is zero; the
    # eigenvalue 1 lies below, 1.5 at the shift
    d, e2 = [1.5, 1.0, 3.0], [0.0, 0.0, 0.0]
    xs = [1.5, 1.0, 3.0, 1.25, 2.0, 3.5, 0.5]
    (c,) = run_counts(sturm_bin, [(d, e2, xs)])
    eig = np.array(d)
    for x, got in zip(xs, c[:, 0]):
        assert _admissible(eig, x, got), (x, got)
    assert c[3:, 0].tolist() == [1, 2, 3, 0]


def _blocks_case(rng, nblocks):
    """Direct sum of 1x1 blocks (d) and 2x2 blocks [[a, b], [b, a]] (eigenvalues
    a -+ b), all in halves, so every eigenvalue and every minor at those
    shifts is exact in binary."""
    d, e2, eig = [], [], []
    for _ in range(nblocks):
        first = len(d)
        if rng.random() < 0.5:
            v = rng.integers(-8, 9) / 2
            d.append(v); e2.append(0.0); eig.append(v)
        else:
            a = rng.integers(-8, 9) / 2
            b = rng.integers(1, 5) / 2
            d += [a, a]; e2 += [0.0, b * b]; eig += [a - b, a + b]
        assert e2[first] == 0.0
    return np.array(d), np.array(e2), np.array(eig)


def test_split_blocks_at_block_eigenvalues(sturm_bin):
    rng = np.random.default_rng(11)
    cases, eigs = [], []
    for _ in range(60):
        d, e2, eig = _blocks_case(rng, int(rng.integers(2, 12)))
        xs = np.concatenate([np.unique(eig), np.unique(eig) + 0.25, [eig.min() - 1, eig.max() + 1]])
        cases.append((d, e2, xs))
        eigs.append(eig)
    missed = 0
    for (d, e2, xs), eig, got in zip(cases, eigs, run_counts(sturm_bin, cases)):
        for x, (g, plain) in zip(xs, got):
            assert _admissible(eig, x, g), (d, e2, x, g)
            missed += not _admissible(eig, x, plain)
    assert missed > 0   # the cases do reach the split-at-a-zero-minor situation


def test_unsplit_random_vs_lapack(sturm_bin):
    rng = np.random.default_rng(12)
    cases, eigs = [], []
    for n in (2, 3, 5, 8, 16, 24, 32):
        d = rng.uniform(-0.5, 0.5, n)
        e = rng.uniform(0.01, 0.3, n - 1)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        eig = np.linalg.eigvalsh(T)
        xs = np.concatenate([rng.uniform(-1.2, 1.2, 40), (eig[:-1] + eig[1:]) / 2])
        xs = xs[np.min(np.abs(xs[:, None] - eig[None, :]), axis=1) > 1e-9]
        cases.append((d, np.concatenate([[0.0], e * e]), xs))
        eigs.append(eig)
    for (d, e2, xs), eig, got in zip(cases, eigs, run_counts(sturm_bin, cases)):
        want = np.array([(eig < x).sum() for x in xs])
        assert np.array_equal(got[:, 0], want)
        assert np.array_equal(got[:, 1], want)   # without splits the plain row agrees
