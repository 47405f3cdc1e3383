"""Batched ensembles of independent 2-D IB-GM problems of uneven size.

Problems of equal grid size N form one size class; a class is one library
context whose 2-D grid has n = (N, N, m): m layers that never exchange data
(each with its own time step and line-solve factors, and its points tagged
with their layer).  A class of more than `split_cells` cells is dealt out to
several contexts of near-equal layer counts, so that with one graph branch
per context no single branch carries most of the work.  All contexts share
one stream; after the first step (which uses the start-up rules of the
method) the steps of every context are replayed from one captured hipGraph
(ib_graph_create / ib_graph_launch), optionally with one independent graph
branch per context.  The line-solve tile shapes of each context can be
picked by the library's autotuner (ib_tune).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import ibgm


@dataclass
class _Batch:
    X: np.ndarray
    links: tuple
    w: np.ndarray
    layer: np.ndarray


class Ensemble:
    """members: objects with n (grid cells per side, the box is the unit
    square), dt, and structure (X (2, np), links (a, b, kappa, l0), w).
    split_cells: 0 keeps one context per size class; otherwise a class of
    more cells is split over ceil(cells / split_cells) contexts."""

    def __init__(self, members, rho: float = 1.0, mu: float = 0.01, chi: float = 0.6,
                 precision: int = ibgm.IB_PREC_MIXED, device="cuda", stream=None,
                 split_cells: int = 0):
        self.members = list(members)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        sizes = sorted({int(m.n) for m in self.members})
        groups = []
        for n in sizes:
            cls = [m for m in self.members if int(m.n) == n]
            parts = 1
            if split_cells > 0:
                parts = min(len(cls), -(-len(cls) * n * n // int(split_cells)))
            for q in range(parts):  # members q, q + parts, ... (near-equal counts)
                groups.append((n, cls[q::parts]))
        self.sims, self.classes, self.where = [], [], {}
        for n, group in groups:
            Xs, a, b, k, l0, w, lay = [], [], [], [], [], [], []
            off = 0
            for layer, m in enumerate(group):
                st = m.structure
                npts = st.X.shape[1]
                Xs.append(np.asarray(st.X, dtype=np.float64))
                la, lb, lk, ll = st.links
                a.append(np.asarray(la, dtype=np.int64) + off)
                b.append(np.asarray(lb, dtype=np.int64) + off)
                k.append(np.asarray(lk, dtype=np.float64))
                l0.append(np.asarray(ll, dtype=np.float64))
                w.append(np.asarray(st.w, dtype=np.float64))
                lay.append(np.full(npts, layer, dtype=np.int32))
                self.where[id(m)] = (len(self.sims), layer, off, npts)
                off += npts
            batch = _Batch(np.concatenate(Xs, axis=1),
                           (np.concatenate(a).astype(np.int32), np.concatenate(b).astype(np.int32),
                            np.concatenate(k), np.concatenate(l0)),
                           np.concatenate(w), np.concatenate(lay))
            ldt = [float(m.dt) for m in group]
            cfg = ibgm.Config(2, (n, n, len(group)), 1.0 / n, rho=rho, mu=mu, dt=ldt[0], chi=chi,
                              precision=precision, layer_dt=ldt)
            u0 = [np.zeros(cfg.shape) for _ in range(2)]
            self.sims.append(ibgm.Simulation(cfg, u0, batch, device=self.device,
                                             stream=self.stream))
            self.classes.append((n, group))
        self.graph = None
        self.cells = sum(int(m.n) ** 2 for m in self.members)

    # -- stepping --------------------------------------------------------
    def tune(self, reps: int = 3):
        return [s.tune(reps) for s in self.sims]

    def step(self, nsteps: int = 1):
        """Eager: enqueue nsteps steps of every class, class after class."""
        for _ in range(nsteps):
            for s in self.sims:
                s.step(1)
        return self

    def capture(self, steps_per_launch: int = 2, branches: bool = False):
        """Capture steps_per_launch steps of every class into one hipGraph
        (every class must have taken its first step)."""
        if self.graph is not None:
            self.graph.close()
        self.graph = ibgm.Graph(self.sims, steps_per_launch, branches=branches,
                                stream=self.stream)
        return self.graph

    def launch(self, nlaunches: int = 1):
        if self.graph is None:
            raise ibgm.IBError(ibgm.IB_E_STATE, "no captured graph: call capture() first")
        self.graph.launch(nlaunches)

    def run(self, nsteps: int, steps_per_launch: int = 2, branches: bool = False):
        """Advance every member by nsteps: the first step eagerly (start-up
        rules), then graph launches, then any remainder eagerly."""
        done = 0
        if self.sims[0].sync() == 0 and nsteps > 0:
            self.step(1)
            done = 1
        full = (nsteps - done) // steps_per_launch
        if full > 0:
            if self.graph is None or self.graph.steps_per_launch != steps_per_launch:
                self.capture(steps_per_launch, branches)
            self.launch(full)
            done += full * steps_per_launch
        self.step(nsteps - done)
        return self

    def sync(self):
        return [s.sync() for s in self.sims]

    # -- results ---------------------------------------------------------
    def member_state(self, m):
        """u, p, psi, X of one member (numpy, its own shapes)."""
        ci, layer, off, npts = self.where[id(m)]
        st = self.sims[ci].state()
        return {"u": [st["u"][c][layer] for c in range(2)], "p": st["p"][layer],
                "psi": st["psi"][layer], "X": st["X"][:, off:off + npts]}

    def close(self):
        if self.graph is not None:
            self.graph.close()
            self.graph = None
        for s in self.sims:
            s.close()
