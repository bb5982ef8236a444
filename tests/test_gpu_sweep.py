"""GPU test of the gap sweep with contact forces: a batch of two channels
(gap 12 and gap 2 between a post pair, one cell of radius 3 upstream,
centred on the gap) stepped 1200 times in FP32 deviation storage.

  - the cells' centroid trajectories equal the FP64 oracle's (each channel
    run alone in the oracle with its walls and posts), sampled every 50 steps;
  - the tracker classifies the wide gap as passed and the narrow one as not
    passed through the gap."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu

GAPS = (12, 2)
NSTEPS, EVERY = 1200, 50


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


def _oracle_centroids(orc, s):
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells, contact=S.contact_params(s))
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = L.rest()
    out = [X.mean(0)]
    for _ in range(NSTEPS // EVERY):
        f = orc.run(L, M, f, X, V, nsteps=EVERY)
        out.append(X.mean(0))
    return np.array(out)


def test_gap_sweep_pass_no_pass(orc, lbm):
    from paper_1110_0995_amd import sweep
    scs = [S.gap_pair(gap=g, cell_centre=(20.0, None, None), gx=1e-4) for g in GAPS]
    lat = lbm.Lattice.batch(scs, prec="f32dev")
    cells, chan = S.batch_cells(scs)
    mesh = lbm.Mesh(lat, cells, chan, contact=S.contact_params_batch(scs))
    tr = sweep.GapTracker(scs, cells.vert_off, chan)
    X = mesh.positions()
    tr.update(X, 0)
    traj = [np.array([X[cells.vert_off[k]:cells.vert_off[k + 1]].mean(0) for k in range(len(scs))])]
    for t in range(EVERY, NSTEPS + 1, EVERY):
        lat.run(EVERY, mesh, steps_per_graph=EVERY)
        X = mesh.positions()
        tr.update(X, t)
        traj.append(np.array([X[cells.vert_off[k]:cells.vert_off[k + 1]].mean(0) for k in range(len(scs))]))
    traj = np.array(traj)  # [checks, channel, 3]
    assert np.isfinite(traj).all()
    for k, s in enumerate(scs):
        ref = _oracle_centroids(orc, s)
        # FP32 storage against FP64 over 1200 steps: the centroid drifts by
        # ~1e-4 of its ~20 LU travel at most
        assert np.abs(traj[:, k] - ref).max() < 2e-3, f"gap {s.meta['gap']}"
    summ = {r["gap"]: r for r in tr.summary()}
    assert summ[12]["passed"] and summ[12]["through"] == 1
    assert not summ[2]["passed"]
    # the narrow gap held the cell back: it travelled less far
    assert traj[-1, 1, 0] < traj[-1, 0, 0]
