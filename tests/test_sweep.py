"""CPU checks of the gap pass / no-pass tracker on synthetic centroid
trajectories (known crossings of the post plane)."""
import numpy as np

from paper_1110_0995_amd import scenario as S
from paper_1110_0995_amd import sweep


def _tracker(gap=8):
    s = S.gap_pair(gap=gap)  # 64 x 32 x 24, posts at x = 32, y = 16 -+ (4 + gap/2)
    return s, sweep.GapTracker([s], s.cells.vert_off)


def _at(s, c):
    """Positions of the one cell translated so its centroid is c."""
    X = s.cells.positions()
    return X - X.mean(0) + np.asarray(c, np.float64)


def test_through_the_gap():
    s, tr = _tracker(gap=8)
    tr.update(_at(s, (30.0, 16.5, 11.5)), 0)
    tr.update(_at(s, (34.0, 17.5, 11.5)), 100)
    (e,) = tr.events
    assert e["through"] and e["step"] == 50.0 and abs(e["dy"] - 1.0) < 1e-12
    assert tr.summary()[0]["passed"] and tr.min_passing_gap() == 8


def test_around_the_posts_and_periodic_laps():
    s, tr = _tracker(gap=8)
    # beyond the post centres (|dy| >= 8) through the periodic y boundary, three laps of x
    tr.update(_at(s, (20.0, 31.0, 11.5)), 0)
    tr.update(_at(s, (20.0 + 3 * 64, 33.0, 11.5)), 300)
    assert len(tr.events) == 3 and not any(e["through"] for e in tr.events)
    assert [round(e["step"]) for e in tr.events] == [19, 119, 219]
    assert tr.summary()[0]["around"] == 3 and tr.min_passing_gap() is None


def test_no_crossing_upstream_or_backwards():
    s, tr = _tracker()
    tr.update(_at(s, (10.0, 16.0, 11.5)), 0)
    tr.update(_at(s, (31.9, 16.0, 11.5)), 50)
    tr.update(_at(s, (20.0, 16.0, 11.5)), 100)  # backwards across nothing
    tr.update(_at(s, (40.0, 16.0, 11.5)), 150)
    tr.update(_at(s, (30.0, 16.0, 11.5)), 200)  # backwards across the plane: not a pass
    assert len(tr.events) == 1 and tr.events[0]["through"]


# --- the gap ladder (one cell per channel, gaps stepped by 1) -------------

def _reachable(fluid2d, start):
    """Fluid (y, x) cells reachable from start in the (y, x) plane, with 4-
    neighbour moves, periodic in y, not across the x ends (so upstream and
    downstream of the posts meet only through the posts' row)."""
    ny, nx = fluid2d.shape
    seen = np.zeros_like(fluid2d, bool)
    stack = [start]
    while stack:
        y, x = stack.pop()
        if seen[y, x] or not fluid2d[y, x]:
            continue
        seen[y, x] = True
        stack += [((y + 1) % ny, x), ((y - 1) % ny, x)] + [(y, x2) for x2 in (x - 1, x + 1) if 0 <= x2 < nx]
    return seen


def test_ladder_slit_has_one_opening_of_the_gap():
    """At the posts' centre line the fluid nodes are exactly gap nodes
    (y0 .. y0 + gap - 1, so the halfway surfaces are gap apart); cutting
    them leaves the upstream and downstream halves of the (x, y) plane
    disconnected; every post lies within the row."""
    for cell in ("tumour", "red"):
        for g in (1, 2, 5, 12, 16):
            (s,) = S.gap_ladder(cell, [g])
            plane = s.solid[s.nz // 2] == 0  # [ny, nx], posts span z
            xc = s.nx // 2
            col = np.where(plane[:, xc])[0]
            assert len(col) == g and col[-1] - col[0] == g - 1, (cell, g, col)
            assert abs(col.mean() - s.meta["midline"]) < 1e-12
            assert all(abs(x - s.nx / 2) < 1e-12 for x, _ in s.meta["post_centres"])
            cut = plane.copy()
            cut[col, xc] = False
            assert not _reachable(cut, (0, 2))[:, xc + 1:].any()
            # with the opening the two sides connect
            assert _reachable(plane, (0, 2))[0, s.nx - 1]


def test_ladder_cells_clear_and_centred():
    for cell, diameter in (("tumour", S.DIAMETER_CTC), ("red", S.DIAMETER_RBC)):
        scs = S.gap_ladder(cell, range(1, 17))
        for s in scs:
            X = s.cells.positions()
            assert s.cells.ncells == 1
            face = s.nx / 2 - s.meta["post_radius"] - 0.5
            assert abs(X[:, 0].max() - (face - 1.5)) < 1e-5  # front 1.5 upstream of the posts' surface
            assert abs(0.5 * (X[:, 1].max() + X[:, 1].min()) - s.meta["midline"]) < 1e-5
            assert abs((X[:, 1].max() - X[:, 1].min()) - diameter) < 1e-4  # diameter across the gap
            assert X[:, 2].min() > 1.5 and X[:, 2].max() < s.nz - 2.5  # clear of the z walls
        cells, chan = S.batch_cells(scs)  # one batch per ladder (shared law and mass)
        assert list(chan) == list(range(len(scs)))


def _ladder_tracker(**kw):
    scs = S.gap_ladder("tumour", [4, 8]) + S.gap_ladder("red", [2])
    cells, chan = S.batch_cells(scs)
    return scs, cells, sweep.LadderTracker(scs, cells.vert_off, chan, **kw)


def _shift(X, cells, k, dx):
    Y = X.copy()
    Y[cells.vert_off[k]:cells.vert_off[k + 1], 0] += dx
    return Y


def test_ladder_tracker_pass_stall_nonfinite():
    scs, cells, tr = _ladder_tracker(stall_window=1000, stall_dist=0.05, t_min=2000)
    X0 = cells.positions()
    exit_x = scs[0].meta["exit_x"]
    xmin1 = X0[cells.vert_off[1]:cells.vert_off[2], 0].min()
    tr.update(X0, 0)
    # channel 0 creeps 0.01 per 500 steps (stalls once t >= t_min); channel 1
    # moves steadily and then its last vertex leaves the posts; channel 2 blows up
    for t in range(500, 4001, 500):
        X = _shift(X0, cells, 0, 0.01 * t / 500)
        X = _shift(X, cells, 1, (exit_x - xmin1 + 0.01) * t / 3000 if t <= 3000 else exit_x - xmin1 + 0.5)
        if t >= 1500:
            X[cells.vert_off[2] + 7, 1] = np.nan
        tr.update(X, t)
    r = tr.results()
    assert [x["outcome"] for x in r] == ["stalled", "passed", "non-finite"]
    assert [x["step"] for x in r] == [2000, 3000, 1500]
    assert tr.done()


def test_ladder_tracker_no_stall_before_t_min_or_while_moving():
    scs, cells, tr = _ladder_tracker(stall_window=1000, stall_dist=0.05, t_min=2000)
    X0 = cells.positions()
    tr.update(X0, 0)
    for t in range(500, 6001, 500):  # every cell advances 0.04 per 500 steps = 0.08 per window
        tr.update(X0 + np.array([0.04 * t / 500, 0.0, 0.0]), t)
    assert [x["outcome"] for x in tr.results()] == ["undecided"] * 3 and not tr.done()


def test_ladder_summary_monotone_and_min_gap():
    res = [dict(cell="tumour", gap=g, outcome=o, step=100 * g) for g, o in
           [(5, "passed"), (3, "stalled"), (4, "stalled"), (6, "passed"), (2, "stalled")]]
    res += [dict(cell="red", gap=g, outcome=o, step=10) for g, o in
            [(1, "stalled"), (2, "passed"), (3, "stalled"), (4, "passed"), (5, "undecided")]]
    d = sweep.ladder_summary(res)
    t = d["tumour"]
    assert t["gaps"] == [2, 3, 4, 5, 6] and t["monotone"] and t["min_passing_gap"] == 5
    assert t["max_stalling_gap"] == 4 and t["undecided"] == 0
    r = d["red"]
    assert not r["monotone"] and r["min_passing_gap"] == 4 and r["undecided"] == 1
