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
