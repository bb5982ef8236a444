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

from . import _lib
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


class LadderTracker:
    """Outcome of each channel of a gap ladder (scenario.gap_ladder): its
    cell has passed once every vertex is downstream of the posts' surface
    (x > meta["exit_x"]); it has stalled once, after ``t_min`` steps, its
    vertex centroid advanced less than ``stall_dist`` over the last
    ``stall_window`` steps while still in front of that surface.  Positions
    are unwrapped (anchor + offset), so a cell that passed cannot come back
    into the opening through the periodic x boundary.  A channel whose
    membrane positions stop being finite is recorded as "non-finite"; the
    tracker keeps following the others (the channels of a batch are
    independent)."""

    def __init__(self, scenarios: Sequence[S.Scenario], vert_off: np.ndarray, chan: np.ndarray,
                 stall_window: int = 2000, stall_dist: float = 0.05, t_min: int = 2000):
        self.scs = list(scenarios)
        self.vert_off = np.asarray(vert_off)
        self.chan = np.asarray(chan, np.int64)
        self.stall_window, self.stall_dist, self.t_min = stall_window, stall_dist, t_min
        self.hist: List[tuple] = []  # (step, centroid x per channel)
        self.outcome: List[Optional[str]] = [None] * len(self.scs)
        self.at: List[Optional[int]] = [None] * len(self.scs)

    def update(self, X: np.ndarray, step: int) -> None:
        n = len(self.scs)
        cx = np.zeros(n)
        xmin = np.full(n, np.inf)
        for c in range(len(self.vert_off) - 1):
            k = int(self.chan[c])
            v = X[self.vert_off[c]:self.vert_off[c + 1]]
            if not np.isfinite(v).all():
                cx[k] = np.nan
                continue
            cx[k] = v[:, 0].mean()
            xmin[k] = min(xmin[k], v[:, 0].min())
        self.hist.append((step, cx))
        past = [h for h in self.hist if h[0] <= step - self.stall_window]
        for k, s in enumerate(self.scs):
            if self.outcome[k] is not None:
                continue
            if not np.isfinite(cx[k]):
                self.outcome[k], self.at[k] = "non-finite", step
            elif xmin[k] > s.meta["exit_x"]:
                self.outcome[k], self.at[k] = "passed", step
            elif step >= self.t_min and past and cx[k] - past[-1][1][k] < self.stall_dist:
                self.outcome[k], self.at[k] = "stalled", step

    def done(self) -> bool:
        return all(o is not None for o in self.outcome)

    def results(self) -> List[Dict]:
        last = self.hist[-1][1] if self.hist else np.zeros(len(self.scs))
        return [dict(channel=k, cell=s.meta["cell"], gap=s.meta["gap"], outcome=self.outcome[k] or "undecided",
                     step=self.at[k], centroid_x=float(last[k])) for k, s in enumerate(self.scs)]


def ladder_summary(results: Sequence[Dict]) -> Dict[str, Dict]:
    """Per cell type: gaps in increasing order with their outcomes, whether
    the decided outcomes are monotone in the gap (every passing gap above
    every stalling one), the smallest passing gap (None if none passed;
    with a non-monotone curve it is the smallest gap above every stall), and
    the gaps whose run went non-finite."""
    out: Dict[str, Dict] = {}
    for cell in sorted({r["cell"] for r in results}):
        rs = sorted((r for r in results if r["cell"] == cell), key=lambda r: r["gap"])
        gaps = [r["gap"] for r in rs]
        oc = [r["outcome"] for r in rs]
        passed = [g for g, o in zip(gaps, oc) if o == "passed"]
        nonfinite = [g for g, o in zip(gaps, oc) if o == "non-finite"]
        stalled = [g for g, o in zip(gaps, oc) if o == "stalled"]
        monotone = not passed or not stalled or min(passed) > max(stalled)
        above = [g for g in passed if not stalled or g > max(stalled)]
        out[cell] = dict(gaps=gaps, outcome=oc, steps=[r["step"] for r in rs], monotone=bool(monotone),
                         min_passing_gap=(min(above) if above else None),
                         max_stalling_gap=(max(stalled) if stalled else None),
                         undecided=sum(o == "undecided" for o in oc), non_finite=nonfinite)
    return out


def run_ladder(lbm, scenarios: Sequence[S.Scenario], max_steps: int, check_every: int = 250,
               prec: str = "f32dev", contact: bool = True, log=None, **track_kw) -> LadderTracker:
    """Step the ladder channels as one batch (graph-captured groups of
    check_every steps, contact forces of the collisions on) until every
    channel is decided or max_steps have run.  When the library reports
    non-finite populations the run stops there: the channels whose membranes
    went non-finite are marked, the rest keep their outcome so far
    (tracker.stopped says why)."""
    lat = lbm.Lattice.batch(scenarios, prec=prec)
    cells, chan = S.batch_cells(scenarios)
    mesh = lbm.Mesh(lat, cells, chan, contact=S.contact_params_batch(scenarios) if contact else None)
    tr = LadderTracker(scenarios, cells.vert_off, chan, **track_kw)
    tr.update(mesh.positions(), 0)
    spg = check_every if check_every % 2 == 0 else 0
    done = 0
    tr.stopped = None
    try:
        while done < max_steps and not tr.done():
            n = min(check_every, max_steps - done)
            try:
                lat.run(n, mesh, steps_per_graph=spg if n == check_every else 0)
            except _lib.LbmError as e:
                if e.code != _lib.LBM_ENONFINITE:
                    raise
                tr.update(mesh.positions(), done)
                tr.stopped = f"non-finite populations reported before step {done}"
                break
            done += n
            tr.update(mesh.positions(), done)
            if log is not None:
                log(done, tr)
    finally:
        lat.close()
    tr.steps_run = done
    return tr
