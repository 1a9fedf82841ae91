"""The library's Sturm count (the eigenvalue count below x of the Lanczos
tridiagonal T_M, used for theta_0 and theta_1 of the ground-state test),
compiled for the host and checked against counts fixed independently: exact
inertia arguments where a pivot vanishes, numpy eigenvalues elsewhere, and
the invariance of the count under scaling T and x by a power of two (which
exercises the rescaling of the three-term sequence)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "sturm_host.hip")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def sturm(tmp_path_factory):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("sturm") / "sturm_host")
    r = subprocess.run([cc, "--offload-host-only", "-O2", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", SRC, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr

    def run(cases):
        lines = []
        for a, b2, x in cases:
            lines.append(f"{len(a)} {float(x).hex()}")
            lines.append(" ".join(float(v).hex() for v in a))
            lines.append(" ".join(float(v).hex() for v in b2) if len(a) > 1 else "")
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True)
        assert out.returncode == 0, out.stderr
        return [int(s) for s in out.stdout.split()]
    return run


def test_vanishing_pivot_after_tiny_leading_entry(sturm):
    # T = [[e, d, 0], [d, 1, 1], [0, 1, 1]], e = d^2 = 2^-80, x = 0: the
    # leading 2x2 block is singular, so p_1 = 0 exactly while |p_0| = 2^-80.
    # Count: the trailing block [[1, 1], [1, 1]] has eigenvalues 0 and 2, so by
    # interlacing l1 <= 0 <= l2 <= 2 <= l3; det T = -e < 0 with l3 > 0 gives
    # l1 l2 < 0: exactly one eigenvalue below 0.
    e, d = 2.0 ** -80, 2.0 ** -40
    assert sturm([([e, 1.0, 1.0], [d * d, 1.0], 0.0)]) == [1]


def test_vanishing_pivot_then_more_rows(sturm):
    # T = [[e, d, 0, 0], [d, B]] with B = [[1, 1, 0], [1, -3, 1], [0, 1, 2]]:
    # inertia(T) = inertia(B) + inertia(e - d^2 (B^-1)_00) (Haynsworth), and
    # (B^-1)_00 = 7/9, so the Schur complement is 2^-80 (2/9) > 0: the count
    # below 0 is the number of negative eigenvalues of B.
    e, d = 2.0 ** -80, 2.0 ** -40
    B = np.array([[1.0, 1, 0], [1, -3, 1], [0, 1, 2]])
    nneg = int((np.linalg.eigvalsh(B) < 0).sum())
    assert abs(np.linalg.inv(B)[0, 0] - 7 / 9) < 1e-15
    got = sturm([([e, 1.0, -3.0, 2.0], [d * d, 1.0, 1.0], 0.0)])
    assert got == [nneg]


def test_random_tridiagonals_against_eigenvalues(sturm):
    rng = np.random.default_rng(7)
    cases, want = [], []
    for _ in range(300):
        M = int(rng.integers(1, 60))
        a = rng.normal(size=M) * rng.choice([1e-3, 1.0, 30.0])
        b = rng.normal(size=M - 1) * rng.choice([1e-3, 1.0, 30.0])
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        lam = np.linalg.eigvalsh(T)
        span = max(1.0, np.abs(lam).max())
        x = float(rng.uniform(lam.min() - 0.1 * span, lam.max() + 0.1 * span))
        if np.abs(lam - x).min() < 1e-8 * span:
            continue
        cases.append((a, b * b, x))
        want.append(int((lam < x).sum()))
    assert sturm(cases) == want


@pytest.mark.parametrize("k", [-400, -250, 250, 400])
def test_count_invariant_under_power_of_two_scaling(sturm, k):
    rng = np.random.default_rng(1000 + k)
    cases, scaled = [], []
    for _ in range(100):
        M = int(rng.integers(2, 80))
        a, b = rng.normal(size=M), rng.normal(size=M - 1)
        x = float(rng.normal())
        s = 2.0 ** k
        cases.append((a, b * b, x))
        scaled.append((a * s, (b * s) ** 2, x * s))
    assert sturm(cases) == sturm(scaled)
