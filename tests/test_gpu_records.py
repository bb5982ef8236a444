"""GPU tests of the next-step records: the collide-stream pass copies the
populations it streams into the next step's stencil nodes, and the next
coupling takes the fluid velocity there (Sec. 2.2 step 1) from the copies
instead of gathering the 19 population planes of the lattice.

Records on and off must give the same bits (the velocity is computed from
the same stored values with the same operations), and the records must
really be used (lbm_node_records_used), except where a stencil node is not
among them, in which case that step gathers.  Cases: FP32 deviations and FP64
with posts (bounced links feed records too), x rows of one and of several
64-node tiles (the x wrap of the shifted populations), several channels of
different lengths, two membranes per step, points moved by the caller
between steps (the uncovered nodes must be detected), graph-captured runs,
and an FP64 run against the oracle."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu

MOD = (0.02, 0.005, 0.01, 0.1, 0.5)


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


def _scenario(nx=128, ny=40, nz=24, ncells=3, seed=5, gx=1e-4):
    s = S.posts_and_cells(nx, ny, nz, posts_x=2, posts_y=1, post_radius=4, gap=6, ncells=ncells,
                          cell_radius=3.0, level=2, tau=0.8, gx=gx, seed=seed, moduli=MOD)
    return s


def _state(lat, meshes):
    import torch
    torch.cuda.synchronize()
    out = [lat.current().cpu().numpy().copy()]
    for m in meshes:
        out += [m.x.cpu().numpy().copy(), m.v.cpu().numpy().copy(), m.f_el.cpu().numpy().copy()]
    return out


def _run_pair(lbm, s, prec, body, nsteps, meshes_fn=None):
    """The same sequence with records off and on; returns both final states
    and the per-step (used, missed) flags of the run with records."""
    res, flags = {}, []
    for mode in (0, 1):
        lat = lbm.Lattice.from_scenario(s, prec=prec)
        lat.set_node_records(mode)
        meshes = meshes_fn(lat) if meshes_fn else [lbm.Mesh(lat, s.cells)]
        for k in range(nsteps):
            body(lat, meshes, k)
            if mode == 1:
                flags.append(lat.node_records_used())
            lat.step(1)
        res[mode] = _state(lat, meshes)
        lat.close()
    return res, flags


def _couple_all(lat, meshes, k):
    for m in meshes:
        lat.couple(m)


@pytest.mark.parametrize("prec", ["f32dev", "f64"])
@pytest.mark.parametrize("nx", [64, 128])
def test_records_equal_gather_bitwise(lbm, prec, nx):
    s = _scenario(nx=nx)
    res, flags = _run_pair(lbm, s, prec, _couple_all, 12)
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    assert flags[0] == (False, False)  # the first step has no records yet
    assert all(f == (True, False) for f in flags[1:]), flags


def test_records_mask_high_words_bitwise(lbm):
    """A 128-long channel whose cells' stencils cover x = 30..35 (bits 31 and 32
    of a tile's node mask: the mask's two 32-bit halves must each widen as
    unsigned) and a post across the two tile columns."""
    s = S.gap_sweep(4, lengths=(64, 128), ny=32, nz=16, gap_range=(4, 8), post_radius=4, ncells=2,
                    cell_radius=3.0, level=2, tau=0.8, gx=1e-4, seed=3)[0]
    s.cells.moduli[:] = MOD
    assert s.nx == 128
    for prec in ("f32dev", "f64"):
        res, flags = _run_pair(lbm, s, prec, _couple_all, 6)
        for a, b in zip(res[0], res[1]):
            assert np.array_equal(a, b), prec
        assert all(f == (True, False) for f in flags[1:]), flags


def test_records_batch_of_channels_bitwise(lbm):
    scs = S.gap_sweep(4, lengths=(64, 128), ny=32, nz=16, gap_range=(4, 8), post_radius=4, ncells=2,
                      cell_radius=3.0, level=2, tau=0.8, gx=1e-4, seed=3)
    for s in scs:
        s.cells.moduli[:] = MOD
    assert len({s.nx for s in scs}) == 2
    cells, chan = S.batch_cells(scs)
    out, flags = {}, []
    for mode in (0, 1):
        lat = lbm.Lattice.batch(scs)
        lat.set_node_records(mode)
        mesh = lbm.Mesh(lat, cells, chan)
        for k in range(10):
            lat.couple(mesh)
            if mode:
                flags.append(lat.node_records_used())
            lat.step(1)
        lat.run(8, mesh, steps_per_graph=4)
        out[mode] = _state(lat, [mesh])
        lat.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    assert all(f == (True, False) for f in flags[1:]), flags


def test_records_two_meshes_per_step_bitwise(lbm):
    nx, ny, nz = 64, 24, 20
    cen = np.array([[12.2, 11.7, 9.6], [14.9, 12.3, 10.1], [40.5, 10.2, 9.0]])
    a = S.make_cells(cen[:2], 3.0, 2, moduli=MOD)
    b = S.make_cells(cen[2:], 3.0, 2, moduli=MOD)
    s = S.Scenario("two", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10,
                   cells=S.make_cells(cen, 3.0, 2, moduli=MOD))
    res, flags = _run_pair(lbm, s, "f64", _couple_all, 10,
                           meshes_fn=lambda lat: [lbm.Mesh(lat, a), lbm.Mesh(lat, b)])
    for u, w in zip(res[0], res[1]):
        assert np.array_equal(u, w)
    assert all(f == (True, False) for f in flags[1:]), flags


def test_records_points_moved_by_caller(lbm):
    """Between steps the caller shifts one cell by a lattice spacing: its new
    stencil is not among the recorded nodes, the marking finds that, the step
    gathers, and the results stay those of the gather every step."""
    s = _scenario(nx=64, seed=9)
    nv0 = int(s.cells.vert_off[1])

    def body(lat, meshes, k):
        m = meshes[0]
        if k == 5:
            x = m.x.clone()
            x[0, :nv0] += 1.0
            m.x.copy_(x)
        lat.couple(m)

    res, flags = _run_pair(lbm, s, "f32dev", body, 9)
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    assert flags[5] == (True, True)
    assert all(f == (True, False) for i, f in enumerate(flags[1:], 1) if i != 5), flags


def test_records_in_graph_runs_bitwise(lbm):
    """lbm_run with captured graph groups (the first step of a run without
    records runs eagerly, so every captured step finds them) against the
    eager loop with records off."""
    s = _scenario(nx=128, seed=7)
    out = {}
    for mode in (0, 1):
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        lat.set_node_records(mode)
        mesh = lbm.Mesh(lat, s.cells)
        if mode:
            lat.run(9, mesh, steps_per_graph=4)
            lat.run(8, mesh, steps_per_graph=4)
            lat.run(3, mesh)
        else:
            lat.run(20, mesh)
        out[mode] = _state(lat, [mesh])
        lat.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_records_f64_matches_oracle(orc, lbm):
    s = _scenario(nx=128, seed=12)
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    lat.set_node_records(1)
    mesh = lbm.Mesh(lat, s.cells)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells)
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = L.rest()
    used = []
    for _ in range(10):
        lat.couple(mesh)
        used.append(lat.node_records_used()[0])
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    assert all(used[1:])
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12


def test_records_unavailable_for_partial_tiles(lbm):
    """nx not a multiple of 64: the gather is used every step."""
    s = _scenario(nx=40)
    lat = lbm.Lattice.from_scenario(s)
    lat.set_node_records(1)
    mesh = lbm.Mesh(lat, s.cells)
    for _ in range(3):
        lat.couple(mesh)
        assert lat.node_records_used() == (False, False)
        lat.step(1)
