"""GPU tests of the batched form: several independent channels in one
context (one launch per kernel for the whole batch), stepped eagerly or from
a captured HIP graph.

  - a channel inside a batch gives bitwise the populations and membrane
    positions it gives alone (the channels share no node, no cell and no
    arithmetic), at small sizes and on sampled channels of the 64-channel
    gap sweep in the launch shape the benchmark times;
  - every replay of a captured graph equals the eager loop bitwise, with
    eager work and synchronisations between the replays, across a change of
    state-buffer parity and of launch shape, also when the captured steps run
    the membrane kernels on the context's second stream;
  - each channel of an FP64 batch matches the FP64 oracle run on that
    channel alone;
  - the launch shape (tiles per workgroup, tile-list workgroups) does not
    change results."""
import ctypes as C

import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


def _small_batch(seed=7, nch=4):
    scs = S.gap_sweep(nch, lengths=(40, 64, 100), ny=32, nz=16, gap_range=(4, 8), post_radius=4, ncells=2,
                      cell_radius=3.0, level=2, tau=0.8, gx=1e-4, seed=seed)
    for s in scs:  # softer membranes keep the short runs far from any instability
        s.cells.moduli[:] = (0.02, 0.005, 0.01, 0.1, 0.5)
    return scs


def _batch(lbm, scs, prec="f32dev"):
    lat = lbm.Lattice.batch(scs, prec=prec)
    cells, chan = S.batch_cells(scs)
    mesh = lbm.Mesh(lat, cells, chan)
    return lat, mesh, cells, chan


def _alone(lbm, s, prec="f32dev"):
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    return lat, lbm.Mesh(lat, s.cells)


def _vert_range(cells, chan, k):
    idx = np.nonzero(chan == k)[0]
    return int(cells.vert_off[idx[0]]), int(cells.vert_off[idx[-1] + 1])


def _state(lat, mesh):
    import torch
    torch.cuda.synchronize()
    return lat.current().cpu().numpy().copy(), mesh.x.cpu().numpy().copy(), mesh.v.cpu().numpy().copy()


def test_batch_channels_equal_alone_bitwise(lbm):
    scs = _small_batch()
    assert len({s.nx for s in scs}) > 1, "the batch should mix channel lengths"
    lat, mesh, cells, chan = _batch(lbm, scs)
    lat.run(30, mesh)
    fb, xb, vb = _state(lat, mesh)
    # the membrane kernels beside the velocity pass: the same bits
    lo, mo, _, _ = _batch(lbm, scs)
    lo.set_ibm_overlap(1)
    lo.run(30, mo)
    fo, xo, vo = _state(lo, mo)
    assert np.array_equal(fo, fb) and np.array_equal(xo, xb) and np.array_equal(vo, vb)
    lo.close()
    for k, s in enumerate(scs):
        la, ma = _alone(lbm, s)
        la.run(30, ma)
        fa, xa, va = _state(la, ma)
        sl = lat.channel(k)
        assert np.array_equal(fb[:, sl], fa), f"channel {k} populations differ"
        v0, v1 = _vert_range(cells, chan, k)
        assert np.array_equal(xb[:, v0:v1], xa), f"channel {k} positions differ"
        assert np.array_equal(vb[:, v0:v1], va), f"channel {k} velocities differ"
        la.close()
    assert np.isfinite(fb).all()


def test_graph_replays_equal_eager(lbm):
    scs = _small_batch(seed=8)
    A, MA, _, _ = _batch(lbm, scs)
    B, MB, _, _ = _batch(lbm, scs)
    B.set_ibm_overlap(1)  # the captured steps fork and join the second stream
    S_ = 4
    for r in range(4):
        A.run(S_, MA)
        B.run(S_, MB, steps_per_graph=S_)
        B.sums()  # eager work and a synchronisation between replays
        fa, xa, va = _state(A, MA)
        fb, xb, vb = _state(B, MB)
        assert np.array_equal(fa, fb) and np.array_equal(xa, xb) and np.array_equal(va, vb), f"replay {r}"
    # flip the state-buffer parity: the graph is captured again
    A.step(1)
    B.step(1)
    A.run(2 * S_ + 3, MA)
    B.run(2 * S_ + 3, MB, steps_per_graph=S_)  # two replays and three eager steps
    assert np.array_equal(_state(A, MA)[0], _state(B, MB)[0])
    # a new launch shape drops the graph; results do not move
    B.set_launch(2, 5)
    A.run(S_, MA)
    B.run(S_, MB, steps_per_graph=S_)
    fa, xa, _ = _state(A, MA)
    fb, xb, _ = _state(B, MB)
    assert np.array_equal(fa, fb) and np.array_equal(xa, xb)
    assert A.steps_taken() == B.steps_taken() == 4 * S_ + 1 + 2 * S_ + 3 + S_
    # a fluid-only graph
    A.run(6)
    B.run(6, steps_per_graph=2)
    assert np.array_equal(_state(A, MA)[0], _state(B, MB)[0])


@pytest.mark.parametrize("waves,blocks", [(1, 0), (2, 1), (8, 3), (4, 64)])
def test_launch_shape_does_not_change_results(lbm, waves, blocks):
    scs = _small_batch(seed=9, nch=3)
    A, MA, _, _ = _batch(lbm, scs)
    B, MB, _, _ = _batch(lbm, scs)
    B.set_launch(waves, blocks)
    A.run(12, MA)
    B.run(12, MB)
    fa, xa, _ = _state(A, MA)
    fb, xb, _ = _state(B, MB)
    assert np.array_equal(fa, fb) and np.array_equal(xa, xb)


def test_batch_f64_matches_oracle(orc, lbm):
    scs = _small_batch(seed=10, nch=3)
    lat, mesh, cells, chan = _batch(lbm, scs, prec="f64")
    nsteps = 12
    lat.run(nsteps, mesh, steps_per_graph=4)
    fg = lat.populations_f64().cpu().numpy()
    xg = mesh.positions()
    for k, s in enumerate(scs):
        L = orc.Lattice.from_scenario(s)
        M = orc.Mesh(s.cells)
        X = s.cells.positions()
        M.rest_shape(X)
        V = np.zeros_like(X)
        f = L.rest()
        for _ in range(nsteps):
            f = orc.step(L, M, f, X, V)
        fl = s.solid.reshape(-1) == 0
        sl = lat.channel(k)
        # FP64 roundoff only: populations are O(1/3), so 3e-14 is a few
        # hundred ulp after 12 coupled steps in which the GPU fuses
        # multiply-adds and sums the membrane forces in another order; a
        # wrong term would show at the size of the forces (>= 1e-8).
        assert np.abs(fg[:, sl][:, fl] - f[:, fl]).max() < 3e-14, f"channel {k}"
        v0, v1 = _vert_range(cells, chan, k)
        assert np.abs(xg[v0:v1] - X).max() < 1e-12, f"channel {k}"


def test_batch_mesh_needs_channels(lbm):
    from paper_1110_0995_amd import _lib
    scs = _small_batch(seed=11, nch=2)
    lat = lbm.Lattice.batch(scs)
    cells, chan = S.batch_cells(scs)
    with pytest.raises(_lib.LbmError, match="cell_chan"):
        lbm.Mesh(lat, cells)
    bad = chan.copy()
    bad[-1] = 2
    with pytest.raises(_lib.LbmError, match="names channel 2"):
        lbm.Mesh(lat, cells, bad)
    m = lbm.Mesh(lat, cells, chan)
    m.s.xi = 0.0
    assert lat.lib.lbm_run(lat.ctx, C.byref(m.s), 2, 2) == _lib.LBM_EINVAL
    m.s.xi = cells.xi
    assert lat.lib.lbm_run(lat.ctx, C.byref(m.s), 2, 3) == _lib.LBM_EINVAL  # odd group length
    assert lat.lib.lbm_set_launch(lat.ctx, 3, 0) == _lib.LBM_EINVAL


def test_gap_sweep_full_size_sampled_channels(lbm):
    """The 64-channel sweep at full size, in the benchmark's launch shape
    (graph groups of 10 steps): sampled channels equal the same channel run
    alone, bitwise, after 20 coupled steps."""
    scs = S.gap_sweep()
    lat, mesh, cells, chan = _batch(lbm, scs)
    lat.run(20, mesh, steps_per_graph=10)
    fb, xb, _ = _state(lat, mesh)
    assert np.isfinite(fb).all()
    for k in (0, 17, 63):
        la, ma = _alone(lbm, scs[k])
        la.run(20, ma)
        fa, xa, _ = _state(la, ma)
        assert np.array_equal(fb[:, lat.channel(k)], fa), f"channel {k}"
        v0, v1 = _vert_range(cells, chan, k)
        assert np.array_equal(xb[:, v0:v1], xa), f"channel {k}"
        la.close()


def test_autotune_restores_state_and_caches(lbm, tmp_path):
    from paper_1110_0995_amd import autotune
    scs = _small_batch(seed=12, nch=3)
    A, MA, _, _ = _batch(lbm, scs)
    B, MB, _, _ = _batch(lbm, scs)
    A.run(6, MA)
    B.run(6, MB)
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(B, MB, steps=4, cache=cache)
    assert best["collide_waves_per_block"] in autotune.WAVES
    assert best["list_blocks"] in autotune.LIST_BLOCKS
    assert best["steps_per_graph"] in autotune.GRAPH_STEPS
    fa, xa, va = _state(A, MA)
    fb, xb, vb = _state(B, MB)
    assert np.array_equal(fa, fb) and np.array_equal(xa, xb) and np.array_equal(va, vb)
    g = best["steps_per_graph"]
    A.run(g, MA)
    B.run(g, MB, steps_per_graph=g)
    assert np.array_equal(_state(A, MA)[0], _state(B, MB)[0])
    assert autotune.tune(B, MB, cache=cache) == best  # second call reads the cache
