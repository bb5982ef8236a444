"""Gap pass / no-pass classification on the batched sweep.

The paper's filter experiment (Sec. 3) steps the gap between obstacles and
asks whether a cell passes.  Here every channel of a batch holds one post
pair across the flow with its own gap; the tracker follows each cell's
vertex centroid (unwrapped, so periodic laps count) and records every
crossing of the plane through the post centres, with the cross-stream
offset at the crossing: within the span of the post centres it is a pass
through the gap, outside it the cell went around the posts.  A channel
passes when one of its cells went through its gap; the smallest passing gap
of a sweep is the simulated counterpart of the paper's minimum gap (in
lattice units: the physical calibration is not available).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import scenario as S


def centroids(X: np.ndarray, vert_off: np.ndarray) -> np.ndarray:
    """Vertex centroid of each cell, [ncells, 3], from positions [nverts, 3]."""
    n = len(vert_off) - 1
    return np.array([X[vert_off[c]:vert_off[c + 1]].mean(0) for c in range(n)]).reshape(n, 3)


class GapTracker:
    """Crossings of each cell's centroid through the post plane of its channel."""

    def __init__(self, scenarios: Sequence[S.Scenario], vert_off: np.ndarray, chan: Optional[np.ndarray] = None):
        self.scs = list(scenarios)
        self.vert_off = np.asarray(vert_off)
        n = len(self.vert_off) - 1
        self.chan = np.zeros(n, np.int64) if chan is None else np.asarray(chan, np.int64)
        self.prev: Optional[np.ndarray] = None
        self.prev_step = 0
        self.events: List[Dict] = []

    def _geometry(self, k: int):
        s = self.scs[k]
        (xa, ya), (xb, yb) = s.meta["post_centres"][:2]
        return s, xa, 0.5 * (ya + yb), 0.5 * abs(yb - ya)

    def update(self, X: np.ndarray, step: int) -> None:
        c = centroids(X, self.vert_off)
        if self.prev is not None:
            for i in range(len(c)):
                s, xp, ymid, half = self._geometry(self.chan[i])
                x0, x1 = self.prev[i, 0] - xp, c[i, 0] - xp
                k0, k1 = np.floor(x0 / s.nx), np.floor(x1 / s.nx)
                for lap in range(int(k0) + 1, int(k1) + 1):  # downstream crossings of x = xp (mod nx)
                    t = (lap * s.nx - x0) / (x1 - x0)
                    y = self.prev[i, 1] + t * (c[i, 1] - self.prev[i, 1])
                    dy = (y - ymid + s.ny / 2) % s.ny - s.ny / 2
                    self.events.append(dict(cell=i, channel=int(self.chan[i]), step=self.prev_step + t * (step - self.prev_step),
                                            dy=float(dy), through=bool(abs(dy) < half)))
        self.prev = c
        self.prev_step = step

    def summary(self) -> List[Dict]:
        out = []
        for k, s in enumerate(self.scs):
            ev = [e for e in self.events if e["channel"] == k]
            out.append(dict(channel=k, gap=s.meta.get("gap"), through=sum(e["through"] for e in ev),
                            around=sum(not e["through"] for e in ev), passed=any(e["through"] for e in ev)))
        return out

    def min_passing_gap(self) -> Optional[float]:
        g = [r["gap"] for r in self.summary() if r["passed"]]
        return min(g) if g else None


def run_sweep(lbm, scenarios: Sequence[S.Scenario], nsteps: int, check_every: int = 50, prec: str = "f32dev",
              contact: bool = True, **contact_kw) -> GapTracker:
    """Step the channels as one batch (graph-captured groups of check_every
    steps) with the contact forces of the collisions, tracking the cells."""
    lat = lbm.Lattice.batch(scenarios, prec=prec)
    cells, chan = S.batch_cells(scenarios)
    mesh = lbm.Mesh(lat, cells, chan, contact=S.contact_params_batch(scenarios, **contact_kw) if contact else None)
    tr = GapTracker(scenarios, cells.vert_off, chan)
    tr.update(mesh.positions(), 0)
    spg = check_every if check_every % 2 == 0 else 0
    done = 0
    while done < nsteps:
        n = min(check_every, nsteps - done)
        lat.run(n, mesh, steps_per_graph=spg if n == check_every else 0)
        done += n
        tr.update(mesh.positions(), done)
    lat.close()
    return tr
