"""GPU test of the minimum-gap experiment (Sec. 3; Table 1 cells): gap
ladders of one tumour cell or one red cell per channel, stepped as one batch
with the contact forces in FP32 deviation storage until every channel is
decided.

  - over the first 1500 steps the centroid of a tumour cell (gap 10) and of
    a red cell (gap 3) follow the FP64 oracle, each channel run alone there;
  - gaps well below and well above the threshold are classified as stalled
    and passed for both cell types, and the red cell passes a gap at which
    the tumour cell stalls."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu

NCHECK, EVERY = 1500, 250


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


def _oracle_centroids(orc, s, nsteps, every):
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells, contact=S.contact_params(s))
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = L.rest()
    out = [X.mean(0)]
    for _ in range(nsteps // every):
        f = orc.run(L, M, f, X, V, nsteps=every)
        out.append(X.mean(0))
    return np.array(out)


def test_ladder_follows_oracle(orc, lbm):
    scs = S.gap_ladder("tumour", [10]) + S.gap_ladder("red", [3])
    lat = lbm.Lattice.batch(scs, prec="f32dev")
    cells, chan = S.batch_cells(scs)
    mesh = lbm.Mesh(lat, cells, chan, contact=S.contact_params_batch(scs))
    traj = []
    for t in range(0, NCHECK + 1, EVERY):
        if t:
            lat.run(EVERY, mesh, steps_per_graph=EVERY)
        X = mesh.positions()
        traj.append([X[cells.vert_off[k]:cells.vert_off[k + 1]].mean(0) for k in range(len(scs))])
    lat.close()
    traj = np.array(traj)
    assert np.isfinite(traj).all()
    for k, s in enumerate(scs):
        ref = _oracle_centroids(orc, s, NCHECK, EVERY)
        assert ref[-1, 0] - ref[0, 0] > 2.0  # the cell has moved on towards the opening
        assert np.abs(traj[:, k] - ref).max() < 2e-3, s.name


def test_ladder_classifies_both_cell_types(lbm):
    from paper_1110_0995_amd import sweep
    scs = S.gap_ladder("tumour", [3, 4, 10]) + S.gap_ladder("red", [1, 4])
    tr = sweep.run_ladder(lbm, scs, 20000, check_every=250)
    d = sweep.ladder_summary(tr.results())
    assert d["tumour"]["outcome"] == ["stalled", "stalled", "passed"], d
    assert d["red"]["outcome"] == ["stalled", "passed"], d
    assert d["tumour"]["monotone"] and d["red"]["monotone"]
    assert d["red"]["min_passing_gap"] < d["tumour"]["min_passing_gap"]
    assert tr.done() and tr.steps_run < 20000
