"""Pins of the oracle's delta kernel (eq:discretedelta) against the properties
it was built to have (Peskin's moment conditions) and its one-square-root
closed form."""
import numpy as np
import pytest

import oracle


def test_phi_values():
    assert oracle.phi(0.0) == pytest.approx(0.5, abs=1e-16)
    assert oracle.phi(1.0) == pytest.approx(0.25, abs=1e-16)
    assert oracle.phi(-1.0) == pytest.approx(0.25, abs=1e-16)
    assert oracle.phi(2.0) == 0.0
    assert oracle.phi(2.5) == 0.0
    assert oracle.phi(1.5) == pytest.approx((2 - np.sqrt(2)) / 8, abs=1e-16)
    # continuity at the branch points
    for r in (1.0, 2.0):
        assert abs(oracle.phi(r - 1e-12) - oracle.phi(r + 1e-12)) < 1e-10


def test_phi_moment_conditions():
    rng = np.random.default_rng(3)
    for r in rng.uniform(-3, 3, size=200):
        j = np.arange(np.floor(r) - 3, np.floor(r) + 4)
        w = oracle.phi(r - j)
        assert abs(w.sum() - 1.0) < 1e-15
        assert abs(((r - j) * w).sum()) < 1e-15
        assert abs((w ** 2).sum() - 3.0 / 8.0) < 1e-15
        even = w[(j % 2) == 0].sum()
        assert abs(even - 0.5) < 1e-15


def test_phi_one_sqrt_form():
    """On [1, 2) phi(r) = 1/2 - phi(2 - r) with 2 - r in (0, 1]: the outer
    branch follows from the inner one."""
    inner = lambda r: (3 - 2 * r + np.sqrt(1 + 4 * r - 4 * r * r)) / 8
    for r in np.linspace(1.0, 1.999, 57):
        assert abs(oracle.phi(r) - (0.5 - inner(2 - r))) < 1e-15
        assert abs(oracle.phi(-r) - oracle.phi(r)) == 0.0
    for r in np.linspace(0.0, 0.999, 57):
        assert abs(oracle.phi(r) - inner(r)) < 1e-16
