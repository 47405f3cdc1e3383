"""GPU parity of Steps 1a, 2a and 2b through the C ABI against the oracle:
interpolation, link force and spreading on seeded points (including
unwrapped positions and points on grid lines), 2-D and 3-D, FP64 and FP32
storage; plus the adjoint identity on the GPU."""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_3976_amd import inputs

pytestmark = pytest.mark.gpu


def _setup(dim, N, precision, npts=300, seed=0):
    from paper_1305_3976_amd import ibgm
    rng = np.random.default_rng(seed)
    n = (N, N + 3, N + 5 if dim == 3 else 1)  # ragged, non-square
    shp = (n[2], n[1], n[0])
    if dim == 2:
        S = inputs.ellipse(npts, 0.3, 0.2, 1.3)
    else:
        S = inputs.ellipsoid_shell(npts)
    X = S.X + rng.uniform(-1, 1, size=S.X.shape) * 0.01
    X[:, :5] += rng.integers(-2, 3, size=(dim, 5))  # unwrapped copies
    X[:, 5] = 0.5  # on grid lines
    u = [rng.standard_normal(shp) for _ in range(dim)]
    cfg = ibgm.Config(dim, n, 1.0 / N, precision=precision)
    sim = ibgm.Simulation(cfg, u, S)
    P = oracle.make_params(dim, n, 1.0 / N)
    return ibgm, sim, P, S, X, u


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("prec", [0, 1])
def test_interp_spread_force_match_oracle(dim, prec):
    ibgm, sim, P, S, X, u = _setup(dim, 24 if dim == 3 else 40, prec)
    gd = sim.cfg.grid_dtype
    tol = 1e-13 if prec == 0 else 3e-6
    ud = [torch.tensor(c, dtype=gd, device="cuda") for c in u]
    uo = [c.astype(np.float32).astype(np.float64) if prec else c for c in u]
    Xd = torch.tensor(X, device="cuda")
    U = sim.interp(Xd, ud).cpu().numpy()
    Uo = oracle.interp(P, uo, X)
    assert np.abs(U - Uo).max() <= tol * np.abs(Uo).max()

    F = sim.force(Xd).cpu().numpy()
    box = [sim.cfg.n[c] * sim.cfg.h for c in range(dim)]
    Fo = oracle.link_force(X, S.links, period=box)
    assert np.abs(F - Fo).max() <= 1e-13 * np.abs(Fo).max()

    wd = torch.tensor(S.w, device="cuda")
    f = sim.spread(Xd, torch.tensor(Fo, device="cuda"), wd)
    fo = oracle.spread(P, X, Fo, S.w)
    for c in range(dim):
        got = f[c].double().cpu().numpy()
        assert np.abs(got - fo[c]).max() <= (1e-13 if prec == 0 else 3e-6) * np.abs(fo[c]).max()
    # adjoint identity <S F, u>_h = <F, J u>_w, evaluated on the device results
    lhs = sum((f[c].double().cpu().numpy() * ud[c].double().cpu().numpy()).sum()
              for c in range(dim)) * P.h ** dim
    rhs = float((S.w * Fo * U).sum())
    assert abs(lhs - rhs) <= (1e-12 if prec == 0 else 1e-5) * max(1.0, abs(rhs))
    sim.close()


def test_spread_accumulate_and_empty():
    ibgm, sim, P, S, X, u = _setup(2, 32, 0)
    Xd = torch.tensor(X, device="cuda")
    Fd = torch.tensor(oracle.link_force(X, S.links), device="cuda")
    wd = torch.tensor(S.w, device="cuda")
    f1 = sim.spread(Xd, Fd, wd)
    f2 = sim.spread(Xd, Fd, wd, out=[t.clone() for t in f1], accumulate=True)
    for c in range(2):
        assert torch.allclose(f2[c], 2 * f1[c], rtol=1e-14, atol=1e-14 * f1[c].abs().max().item())
    f3 = sim.spread(Xd[:, :0].contiguous(), Fd[:, :0].contiguous(), wd[:0].contiguous())
    assert all(t.abs().max().item() == 0 for t in f3)
    sim.close()
