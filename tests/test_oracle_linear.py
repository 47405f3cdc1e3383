"""Pins of the oracle's periodic tridiagonal solver (eq:TriDiagX, Sec. "Linear
Solver") against references that are not the oracle: dense LU of the assembled
matrix, the circulant eigenvalues (Fourier modes), an FFT solve of whole
fields, and the closed-form solution of the paper's directional-split
comparison problem (Sec. "Comparison with Poisson Solvers")."""
import numpy as np
import pytest

import oracle


def dense_cyclic(a, b, c):
    n = len(b)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, (i - 1) % n] += a[i]
        A[i, i] += b[i]
        A[i, (i + 1) % n] += c[i]
    return A


@pytest.mark.parametrize("n", list(range(3, 17)))
def test_cyclic_solve_matches_dense_lu(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(4):
        a, c = rng.standard_normal(n), rng.standard_normal(n)
        b = rng.standard_normal(n) + np.sign(rng.standard_normal(n)) * (
            np.abs(a) + np.abs(c) + (0.5 if trial < 2 else 0.05))
        d = rng.standard_normal(n)
        x = oracle.cyclic_solve(a, b, c, d)
        ref = np.linalg.solve(dense_cyclic(a, b, c), d)
        assert np.allclose(x, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("N,nu", [(16, 2.5e-6), (64, 0.05e-3), (16, None)])
def test_cyclic_solve_paper_coefficients(N, nu):
    """Momentum (1 - nu D_xx) and pressure-increment (1 - D_xx) matrices."""
    h = 1.0 / N
    if nu is None:
        diag, off = 1 + 2 / h ** 2, -1 / h ** 2
    else:
        diag, off = 1 + 2 * nu / h ** 2, -nu / h ** 2
    rng = np.random.default_rng(7)
    d = rng.standard_normal(N)
    a = np.full(N, off)
    b = np.full(N, diag)
    x = oracle.cyclic_solve(a, b, a, d)
    A = dense_cyclic(a, b, a)
    ref = np.linalg.solve(A, d)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - ref) <= 10 * cond * 1e-16 * np.linalg.norm(ref)
    assert np.linalg.norm(A @ x - d) <= 1e-13 * np.linalg.norm(A) * np.linalg.norm(x)


@pytest.mark.parametrize("N", [8, 33, 256])
def test_fourier_mode_is_eigenvector(N):
    """The circulant (off, diag, off) maps cos(2 pi k i/N + t) to
    (diag + 2 off cos(2 pi k / N)) times itself."""
    h = 1.0 / N
    diag, off = 1 + 2 / h ** 2, -1 / h ** 2
    i = np.arange(N)
    for k in (1, 3, N // 2):
        b = np.cos(2 * np.pi * k * i / N + 0.4)
        lam = diag + 2 * off * np.cos(2 * np.pi * k / N)
        x = oracle.line_solve(b[None, :], 0, diag, off)[0]
        # forward error bound of a backward-stable solve: cond(A) eps, with
        # cond(1 - D_xx) = 1 + 4 N^2 on the unit line
        tol = 50 * (1 + 4 * N * N) * 2.2e-16
        assert np.abs(x - b / lam).max() <= tol * np.abs(b / lam).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_line_solve_axis_matches_fft(axis):
    """Batched line solve along each axis of a 3-D field equals the FFT
    (circulant diagonalisation) solve along that axis."""
    rng = np.random.default_rng(11 + axis)
    f = rng.standard_normal((6, 10, 12))  # (n2, n1, n0)
    diag, off = 3.1, -1.2
    x = oracle.line_solve(f, axis, diag, off)
    ax = 2 - axis
    N = f.shape[ax]
    k = np.arange(N)
    lam = diag + 2 * off * np.cos(2 * np.pi * k / N)
    shape = [1, 1, 1]
    shape[ax] = N
    ref = np.real(np.fft.ifft(np.fft.fft(f, axis=ax) / lam.reshape(shape), axis=ax))
    assert np.allclose(x, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim,N", [(2, 64), (2, 128), (3, 32)])
def test_directional_split_closed_form(dim, N):
    """(1 - D_xx)(1 - D_yy)[(1 - D_zz)] psi = sin 2 pi x cos 2 pi y [cos 2 pi z]
    at the cell centres: a single Fourier mode, so the discrete solution is
    f / prod_a (1 + (4/h^2) sin^2(pi h))."""
    h = 1.0 / N
    c = (np.arange(N) + 0.5) * h
    if dim == 2:
        Y, X = np.meshgrid(c, c, indexing="ij")
        f = (np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y))[None]
    else:
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        f = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) * np.cos(2 * np.pi * Z)
    psi = f
    for ax in range(dim):
        psi = oracle.line_solve(psi, ax, 1 + 2 / h ** 2, -1 / h ** 2)
    lam = 1 + (4 / h ** 2) * np.sin(np.pi * h) ** 2
    exact = f / lam ** dim
    assert np.abs(psi - exact).max() <= 1e-12 * np.abs(exact).max()
