"""Host logic of the spectrum solver: the complex Hessenberg eigensolver
(csrc/hessenberg.h), compiled with g++ into a small checker and compared with
numpy's general eigensolver; eigenvector residuals must be at rounding level."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "hessenberg_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "hessenberg_check.cpp"),
                    "-o", exe], check=True)
    return exe


def _run(exe, H):
    n = H.shape[0]
    txt = f"{n}\n" + "\n".join("%.17g %.17g" % (z.real, z.imag) for z in H.ravel())
    out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    vals = [tuple(map(float, l.split())) for l in out.strip().splitlines()]
    ev = np.array([complex(*v) for v in vals[:n]])
    res = np.array([v[0] for v in vals[n:]])
    return ev, res


def _match(a, b):
    """Largest distance of a greedy one-to-one matching of two eigenvalue sets."""
    b = list(b)
    worst = 0.0
    for z in a:
        k = int(np.argmin([abs(z - w) for w in b]))
        worst = max(worst, abs(z - b.pop(k)))
    return worst


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (40, 3), (120, 4)])
def test_random_hessenberg_matches_numpy(checker, n, seed):
    rng = np.random.default_rng(seed)
    H = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    ev, res = _run(checker, H)
    ref = np.linalg.eigvals(H)
    scale = max(1.0, np.abs(ref).max())
    assert _match(ev, ref) <= 1e-10 * scale
    assert res.max() <= 1e-9 * scale


def test_structured_cases(checker):
    """Real matrix with conjugate pairs, a Jordan-like block, a diagonal matrix
    and a zero subdiagonal (already split)."""
    rng = np.random.default_rng(7)
    H = np.triu(rng.standard_normal((12, 12)), -1).astype(complex)
    ev, _ = _run(checker, H)
    assert _match(ev, np.linalg.eigvals(H)) <= 1e-10 * np.abs(ev).max()
    D = np.diag(np.arange(1, 6) + 0.5j)
    ev, res = _run(checker, D)
    assert _match(ev, np.diag(D)) == 0.0 and res.max() < 1e-14
    S = np.triu(rng.standard_normal((6, 6)) + 0j, -1)
    S[3, 2] = 0.0
    ev, _ = _run(checker, S)
    assert _match(ev, np.linalg.eigvals(S)) <= 1e-11 * np.abs(ev).max()


@pytest.fixture(scope="module")
def schur():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "schur_check")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "schur_check.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.mark.parametrize("n,seed,structured", [(1, 0, False), (5, 1, False), (30, 2, False),
                                               (40, 3, True)])
def test_schur_decomposition_and_reordering(schur, n, seed, structured):
    """A = Q T Q^H with Q unitary and T upper triangular, before and after
    moving every other diagonal entry to the front; the eigenvalues are numpy's.
    structured: the Krylov-Schur shape (triangular block, one full row, then
    Hessenberg)."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if structured:
        k = n // 3
        A = np.triu(A, -1)
        A[:k, :k] = np.triu(A[:k, :k])
        A[k, :k] = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    flags = [i % 2 for i in range(n)]
    txt = (f"{n}\n" + "\n".join("%.17g %.17g" % (z.real, z.imag) for z in A.ravel())
           + "\n" + " ".join(map(str, flags)))
    out = subprocess.run([schur], input=txt, capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()
    scale = max(1.0, np.abs(A).max())
    for line in (out[0], out[n + 1]):
        e1, e2, e3 = map(float, line.split())
        assert e1 <= 1e-12 * n * scale and e2 <= 1e-12 * n and e3 == 0.0
    d0 = np.array([complex(*map(float, l.split())) for l in out[1:n + 1]])
    d1 = np.array([complex(*map(float, l.split())) for l in out[n + 2:]])
    assert _match(d0, np.linalg.eigvals(A)) <= 1e-10 * scale
    # the flagged entries lead, in their original order; the rest follow
    want = d0[np.array(flags, dtype=bool)]
    rest = d0[~np.array(flags, dtype=bool)]
    assert np.abs(d1[:len(want)] - want).max(initial=0.0) <= 1e-10 * scale
    assert _match(d1[len(want):], rest) <= 1e-10 * scale
