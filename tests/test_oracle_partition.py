"""Pins of the oracle's statement of the paper's partitioned solve (Sec.
"Linear Solver": local Thomas solves per subdomain, the P x P Schur
complement system, local corrections): for every subdomain count P it must
give the same solution as one cyclic Thomas + Sherman-Morrison solve and as a
dense solve of the written-out periodic matrix, also on ragged partitions and
on the paper's own (very ill-conditioned) pressure-increment coefficients;
and its Schur complement must be periodic tridiagonal, as the paper states."""
import numpy as np
import pytest

import oracle
from oracle import partition as pt

COUNTS = (1, 2, 3, 4, 8, 16, 32, 64)


def dense(c, a, b):
    N = len(a)
    A = np.diag(a) + np.diag(c[1:], -1) + np.diag(b[:-1], 1)
    A[0, -1] += c[0]
    A[-1, 0] += b[-1]
    return A


def system(N, seed):
    """Random diagonally dominant periodic rows with distinct coefficients
    per row (so a transposed or shifted coefficient index shows)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, N)
    b = rng.uniform(-1, 1, N)
    a = 2.5 + rng.uniform(0, 1, N)
    return c, a, b, rng.standard_normal(N)


@pytest.mark.parametrize("N", [128, 131, 200])
@pytest.mark.parametrize("P", COUNTS)
def test_partitioned_equals_cyclic_and_dense(N, P):
    c, a, b, f = system(N, 7 * N + P)
    x = pt.partitioned_cyclic_solve(c, a, b, f, P)
    ref = oracle.cyclic_solve(c, a, b, f)          # (sub, diag, super) order
    assert np.abs(x - ref).max() <= 1e-13 * np.abs(ref).max()
    den = np.linalg.solve(dense(c, a, b), f)
    assert np.abs(x - den).max() <= 1e-13 * np.abs(den).max()
    # and the residual of the periodic rows themselves
    r = c * np.roll(x, 1) + a * x + b * np.roll(x, -1) - f
    assert np.abs(r).max() <= 1e-13 * np.abs(f).max()


@pytest.mark.parametrize("P", COUNTS)
def test_partitioned_on_the_paper_coefficients(P):
    """The 256^3 psi sweep (1 - D_xx): diag 1 + 2/h^2, off -1/h^2, condition
    number 1 + 4/h^2 = 262145; and a momentum sweep (nu = mu dt/2, mu = 0.01,
    dt = 5e-4).  Agreement within the conditioning bound."""
    N = 256
    h = 1.0 / N
    rng = np.random.default_rng(P)
    f = rng.standard_normal(N)
    for nu in (1.0, 0.01 * 5e-4 / 2):
        off = -nu / h ** 2
        a = np.full(N, 1 - 2 * off)
        c = np.full(N, off)
        b = np.full(N, off)
        x = pt.partitioned_cyclic_solve(c, a, b, f, P)
        ref = oracle.cyclic_solve(c, a, b, f)
        cond = 1 + 4 * nu / h ** 2
        assert np.abs(x - ref).max() <= 50 * cond * 2.0 ** -52 * np.abs(ref).max()


@pytest.mark.parametrize("P", [3, 4, 8, 16, 64])
def test_schur_complement_is_periodic_tridiagonal(P):
    c, a, b, _ = system(200, 3 + P)
    S = pt.schur_matrix(c, a, b, P)
    for p in range(P):
        for q in range(P):
            if (q - p) % P not in (0, 1, P - 1):
                assert S[p, q] == 0.0
        assert S[p, (p + 1) % P] != 0.0 and S[p, (p - 1) % P] != 0.0


def test_subdomains_need_an_interior():
    c, a, b, f = system(10, 1)
    with pytest.raises(ValueError):
        pt.partitioned_cyclic_solve(c, a, b, f, 6)          # subdomains of 1-2 unknowns
