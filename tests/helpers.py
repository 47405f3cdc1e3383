"""Shared test helpers: build oracle and GPU simulations from one seeded
workload and compare fields with the paper's discrete l2 norms."""
import importlib

import numpy as np

import oracle


class LazyModule:
    """A module imported on first attribute access.  GPU test modules bind
    the HIP library through this, so that collecting them (on a machine
    where the library is not built, with -m "not gpu") imports nothing;
    on a GPU run the first use imports it and fails loudly if it is
    missing."""

    def __init__(self, name):
        self._name = name
        self._mod = None

    def __getattr__(self, attr):
        # dunder lookups (pickling, introspection by pytest) must not import;
        # the module's own private names (e.g. closure._p) are forwarded
        if attr.startswith("__"):
            raise AttributeError(attr)
        if self._mod is None:
            self._mod = importlib.import_module(self._name)
        return getattr(self._mod, attr)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def oracle_sim(w, rotate=True, no_advection=False, walls_y=False, body_force=(0.0, 0.0, 0.0),
               wall_velocity=(0.0, 0.0, 0.0)):
    P = oracle.make_params(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi,
                           rotate=rotate, no_advection=no_advection, walls_y=walls_y,
                           body_force=body_force, wall_velocity=wall_velocity)
    S = w.structure
    return oracle.Sim(P, [np.asarray(c, dtype=np.float64) for c in w.u0], S.X, S.links, S.w,
                      tether=S.tether)


def gpu_sim(w, precision, rotate=True, no_advection=False, walls_y=False,
            body_force=(0.0, 0.0, 0.0), deterministic=False, wall_velocity=(0.0, 0.0, 0.0)):
    from paper_1305_3976_amd import ibgm
    cfg = ibgm.Config(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi,
                      precision=precision, rotate_split=rotate, no_advection=no_advection,
                      walls_y=walls_y, body_force=body_force,
                      deterministic_spread=deterministic, wall_velocity=wall_velocity)
    return ibgm.Simulation(cfg, w.u0, w.structure)


def field_errors(gpu_state, orc, dim):
    errs = {}
    for c in range(dim):
        errs["u%d" % c] = rel_l2(gpu_state["u"][c], orc.u[c])
    errs["p"] = rel_l2(gpu_state["p"], orc.p)
    errs["psi"] = rel_l2(gpu_state["psi"], orc.psi)
    errs["X"] = rel_l2(gpu_state["X"], orc.X)
    return errs


def psi_vs_p(psi, psi_ref, p_ref):
    """psi error measured against the scale of p (psi is p's per-step
    increment, often orders of magnitude smaller)."""
    scale = max(np.linalg.norm(psi_ref), np.linalg.norm(p_ref), 1e-30)
    return float(np.linalg.norm(np.asarray(psi) - np.asarray(psi_ref)) / scale)


def field_maxabs(gpu_state, orc, dim):
    """max |a - b| / max |b| per field: the point-wise companion of rel_l2,
    which dilutes a fault in one cell by the square root of the cell count."""
    def one(a, b):
        a = np.asarray(a, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    errs = {}
    for c in range(dim):
        errs["u%d" % c] = one(gpu_state["u"][c], orc.u[c])
    errs["p"] = one(gpu_state["p"], orc.p)
    errs["X"] = one(gpu_state["X"], orc.X)
    scale = max(np.abs(np.asarray(orc.psi)).max(), np.abs(np.asarray(orc.p)).max(), 1e-30)
    errs["psi_vs_p"] = float(np.abs(np.asarray(gpu_state["psi"]) - np.asarray(orc.psi)).max() / scale)
    return errs
