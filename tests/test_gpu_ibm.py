"""GPU parity of the coupled LBM + immersed-boundary step against the FP64
oracle, through the C ABI: FP64 to rounding on small cases, FP32 deviation
storage within 1e-5 relative velocity error after 1000 steps (the
full-size workloads over long horizons are in test_gpu_long_parity.py)."""
import time

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


def rel_l2(a, b, mask=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _pair(orc, lbm, s, prec, deform=0.0, seed=0, vel=0.0):
    """GPU lattice+mesh and oracle lattice+mesh on the same seeded inputs.
    Both take their rest shape from the generated (undeformed) mesh; a
    seeded deformation and velocity are then applied to both."""
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    mesh = lbm.Mesh(lat, s.cells)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells)
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    if deform or vel:
        rng = np.random.default_rng(seed)
        off = (s.cells.offset.astype(np.float64) + deform * rng.standard_normal(X.shape)).astype(np.float32)
        mesh.set_offsets(off)
        X = s.cells.anchor[s.cells.vertex_cell()] + off.astype(np.float64)
        Vn = (vel * rng.standard_normal(X.shape)).astype(np.float32)
        mesh.v.copy_(__import__("torch").as_tensor(Vn.T.copy()).to(mesh.v.device, mesh.v.dtype))
        V = Vn.astype(np.float64)
    return lat, mesh, L, M, X, V


def _small(nx=40, ny=32, nz=24, ncells=2, level=2, radius=3.0, posts=True, gx=1e-4, seed=11, tau=0.8):
    s = S.posts_and_cells(nx, ny, nz, posts_x=1 if posts else 0, posts_y=1 if posts else 0, post_radius=4,
                          gap=6, ncells=ncells, cell_radius=radius, level=level, tau=tau, gx=gx, seed=seed,
                          moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    return s


def test_coupled_f64_matches_oracle(orc, lbm):
    s = _small()
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.05, seed=1, vel=1e-3)
    f = L.rest()
    for _ in range(25):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    fg = lat.populations_f64().cpu().numpy()
    assert np.abs(fg[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13
    # the elastic force of the last step, against the oracle's at the previous positions
    assert np.isfinite(mesh.f_el.cpu().numpy()).all()


def test_coupled_f64_elastic_forces(orc, lbm):
    s = _small(posts=False, ncells=3)
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.1, seed=2)
    Fo = M.forces(X)
    lat.couple(mesh)
    Fg = mesh.f_el.double().cpu().numpy().T
    assert np.abs(Fg - Fo).max() < 1e-13 * max(1.0, np.abs(Fo).max())
    assert np.abs(Fo).max() > 1e-4


@pytest.mark.parametrize("prec", ["f32dev", "f32"])
def test_coupled_f32_elastic_forces(orc, lbm, prec):
    s = _small(posts=False, ncells=3, level=3, radius=4.0)
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, prec, deform=0.05, seed=3)
    Fo = M.forces(X)
    lat.couple(mesh)
    Fg = mesh.f_el.double().cpu().numpy().T
    err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    print(f"elastic force {prec}: max error / max force {err:.3e}")
    assert err < 2e-4


def test_rest_state_with_cells_exact(lbm):
    """Undeformed cells in a fluid at rest: FP32 deviation storage stays at
    h = 0 bit-exactly and the points do not move."""
    s = S.posts_and_cells(64, 48, 32, posts_x=1, posts_y=1, ncells=3, gx=0.0, seed=4)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells)
    x0 = mesh.x.clone()
    lat.run(100, mesh)
    assert (lat.current() == 0).all()
    assert (mesh.x == x0).all() and (mesh.v == 0).all()


def test_momentum_periodic_box_with_cells(lbm):
    """Fully periodic, no solids, g = 0: fluid momentum plus point momentum
    is conserved (spread force sums equal the point force sums)."""
    nx, ny, nz = 48, 40, 36
    s = S.Scenario("box", nx, ny, nz, 0.8, (0.0, 0.0, 0.0), np.zeros((nz, ny, nx), np.uint8), 100,
                   cells=S.make_cells(np.array([[20.3, 18.7, 17.9], [33.1, 9.4, 25.2]]), 4.0, 2,
                                      moduli=(0.02, 0.005, 0.01, 0.1, 0.5)))
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells)
    rng = np.random.default_rng(5)
    mesh.set_offsets(s.cells.offset + 0.1 * rng.standard_normal(s.cells.offset.shape))
    import torch
    mesh.v.copy_(torch.as_tensor(1e-3 * rng.standard_normal((3, s.cells.nverts)), dtype=mesh.v.dtype))
    mk = mesh.point_mass()[:, None]
    p0 = lat.sums()[1:] + (mk * mesh.velocities()).sum(0)
    scale = (mk * np.abs(mesh.velocities())).sum()
    lat.run(100, mesh)
    p1 = lat.sums()[1:] + (mk * mesh.velocities()).sum(0)
    assert np.abs(p1 - p0).max() < 1e-12 * scale


def test_f32dev_1000_steps_small_posts_cells(orc, lbm):
    """Posts and cells, FP32 deviation storage, 1000 coupled steps: velocity
    relative L2 error against the FP64 oracle <= 1e-5."""
    s = _small(64, 48, 32, ncells=3, level=3, radius=4.0, gx=1e-5, seed=12)
    s.cells.moduli[:] = S.MODULI_CTC
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f32dev")
    f = L.rest()
    t = time.time()
    orc.run(L, M, f, X, V, nsteps=1000)
    lat.run(1000, mesh)
    fl = s.solid.reshape(-1) == 0
    _, uo = orc.fluid_velocity(L, f)
    _, ug = lat.fields()
    err = rel_l2(ug.double().cpu().numpy(), uo, fl)
    perr = np.abs(mesh.positions() - X).max()
    print(f"small posts+cells f32dev 1000 steps: u rel L2 {err:.3e}, max position error {perr:.3e} "
          f"(oracle {time.time() - t:.1f}s)")
    assert err < 1e-5
    assert perr < 1e-4


def test_two_meshes_in_one_step(orc, lbm):
    """Two membrane populations coupled before the same collide-stream pass
    (tiles shared by both) equal one merged population in the oracle."""
    s = _small(48, 40, 28, ncells=4, level=2, radius=3.0, posts=False, seed=21)
    c = s.cells
    half = lambda lo, hi: S.make_cells(c.anchor[lo:hi] + 0.0, 3.0, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    # rebuild the same cells as two populations with the same offsets
    a, b = half(0, 2), half(2, 4)
    a.offset[:] = c.offset[: a.nverts]
    b.offset[:] = c.offset[a.nverts:]
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    ma, mb = lbm.Mesh(lat, a), lbm.Mesh(lat, b)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(c)
    X = c.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = L.rest()
    for _ in range(15):
        lat.couple(ma)
        lat.couple(mb)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(np.concatenate([ma.positions(), mb.positions()]) - X).max() < 1e-12


def test_dense_cell_f64(orc, lbm):
    """A 642-vertex cell of radius 1.5: many points share each stencil base
    node, so the per-base-node sums run over long sorted runs."""
    nx, ny, nz = 24, 20, 18
    # small moduli: explicit elastic forces on 0.2-long edges need them to stay stable
    cells = S.make_cells(np.array([[11.3, 9.6, 8.7]]), 1.5, 3, moduli=(0.001, 0.0002, 0.0005, 0.005, 0.02))
    s = S.Scenario("dense", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10, cells=cells)
    b = np.floor(cells.positions()).astype(int)
    assert np.unique(b[:, 0] + nx * (b[:, 1] + ny * b[:, 2]), return_counts=True)[1].max() > 8
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.02, seed=8)
    f = L.rest()
    for _ in range(6):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12


def test_cell_across_periodic_faces_f64(orc, lbm):
    """A cell centred on the corner where the periodic x and y faces meet:
    its stencils wrap across both faces (the spread sums it in a box
    unwrapped around one of its points).  Coupled FP64 steps equal the
    oracle's."""
    nx, ny, nz = 36, 32, 24
    cells = S.make_cells(np.array([[0.3, 31.6, 11.4]]), 4.0, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    X = cells.positions()
    assert (X[:, 0] < 0).any() and (X[:, 0] > 0).any() and (X[:, 1] > ny - 1).any()
    s = S.Scenario("corner", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 6, cells=cells)
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.05, seed=14, vel=1e-3)
    f = L.rest()
    for _ in range(6):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13


def test_large_cell_spread_fallback_f64(orc, lbm):
    """A cell of radius 14: the box of its stencil base nodes holds more than
    16384 nodes, so the spread takes it point by point through the atomic
    fallback.  The coupled FP64 steps still match the oracle."""
    nx, ny, nz = 44, 40, 40
    cells = S.make_cells(np.array([[21.4, 19.7, 19.3]]), 14.0, 3, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    b = np.floor(cells.positions()).astype(int)
    assert np.prod(b.max(0) - b.min(0) + 2) > 16384
    s = S.Scenario("large", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 4, cells=cells)
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.05, seed=12, vel=1e-3)
    f = L.rest()
    for _ in range(4):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13


def test_overlapping_cells_share_base_nodes_f64(orc, lbm):
    """Two cells of one population overlap, so some stencil nodes (and base
    nodes) hold points of both: the second cell to claim such a node spreads
    through the fallback path.  Results must still match the oracle."""
    nx, ny, nz = 32, 24, 20
    cells = S.make_cells(np.array([[12.2, 11.7, 9.6], [14.9, 12.3, 10.1]]), 3.0, 2,
                         moduli=(0.01, 0.002, 0.005, 0.05, 0.2))
    s = S.Scenario("overlap", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10, cells=cells)
    b = np.floor(cells.positions()).astype(int)
    key = b[:, 0] + nx * (b[:, 1] + ny * b[:, 2])
    cell = cells.vertex_cell()
    assert len(set(key[cell == 0]) & set(key[cell == 1])) > 0
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.02, seed=9)
    f = L.rest()
    for _ in range(6):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12


def test_two_meshes_sharing_stencil_nodes_f64(orc, lbm):
    """The overlapping pair of cells split into two membrane populations,
    each coupled before the same collide-stream pass: nodes under both
    stencils receive the force of both (the second coupling adds to the
    first, including at base nodes the second population claims anew)."""
    nx, ny, nz = 32, 24, 20
    cen = np.array([[12.2, 11.7, 9.6], [14.9, 12.3, 10.1]])
    mod = (0.01, 0.002, 0.005, 0.05, 0.2)
    both = S.make_cells(cen, 3.0, 2, moduli=mod)
    a, b = S.make_cells(cen[:1], 3.0, 2, moduli=mod), S.make_cells(cen[1:], 3.0, 2, moduli=mod)
    s = S.Scenario("overlap2", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10, cells=both)
    # the two stencils share nodes
    stencil = lambda X: {tuple(int(v) for v in np.floor(p) + d) for p in X for d in np.ndindex(2, 2, 2)}
    assert len(stencil(a.positions()) & stencil(b.positions())) > 0
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    ma, mb = lbm.Mesh(lat, a), lbm.Mesh(lat, b)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(both)
    X = both.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = L.rest()
    for _ in range(6):
        lat.couple(ma)
        lat.couple(mb)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(np.concatenate([ma.positions(), mb.positions()]) - X).max() < 1e-12


def test_coupled_step_is_bit_reproducible(lbm):
    """Two identical runs give identical populations, positions and forces:
    membrane forces are gathered per vertex in a fixed order and the spread
    sums each base node's points in sorted order."""
    s = _small(48, 40, 28, ncells=3, level=3, radius=4.0, seed=13)
    out = []
    for _ in range(2):
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm.Mesh(lat, s.cells)
        lat.run(30, mesh)
        out.append((lat.current().cpu().numpy().copy(), mesh.x.cpu().numpy().copy(), mesh.f_el.cpu().numpy().copy()))
        lat.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_overlapped_schedule_f64(orc, lbm):
    """The membrane kernels on the context's second stream beside the
    velocity pass (forced on for a small mesh) give the same bits as the
    in-order schedule, eager and in captured graphs, with one membrane per
    step and with two, and match the oracle."""
    s = _small(ncells=2, seed=31)
    law = S.contact_params(s)
    out = {}
    off = (s.cells.offset.astype(np.float64)
           + 0.05 * np.random.default_rng(2).standard_normal(s.cells.offset.shape)).astype(np.float32)
    for mode in (0, 1):
        lat = lbm.Lattice.from_scenario(s, prec="f64")
        lat.set_ibm_overlap(mode)
        mesh = lbm.Mesh(lat, s.cells, contact=law)
        mesh.set_offsets(off)
        for _ in range(5):
            lat.couple(mesh)
            lat.step(1)
        lat.run(8, mesh, steps_per_graph=4)
        out[mode] = (lat.populations_f64().cpu().numpy(), mesh.positions(), mesh.velocities())
        lat.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
    lat, mesh, L, M, X, V = _pair(orc, lbm, s, "f64", deform=0.05, seed=1, vel=1e-3)
    lat.set_ibm_overlap(1)
    f = L.rest()
    for _ in range(10):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    lat.close()
    # two membranes per step: the second marks on its own and adds its force
    nx, ny, nz = 32, 24, 20
    cen = np.array([[12.2, 11.7, 9.6], [14.9, 12.3, 10.1]])
    mod = (0.01, 0.002, 0.005, 0.05, 0.2)
    a, b = S.make_cells(cen[:1], 3.0, 2, moduli=mod), S.make_cells(cen[1:], 3.0, 2, moduli=mod)
    s2 = S.Scenario("overlap2", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10,
                    cells=S.make_cells(cen, 3.0, 2, moduli=mod))
    res = {}
    for mode in (0, 1):
        lat = lbm.Lattice.from_scenario(s2, prec="f64")
        lat.set_ibm_overlap(mode)
        ma, mb = lbm.Mesh(lat, a), lbm.Mesh(lat, b)
        for _ in range(6):
            lat.couple(ma)
            lat.couple(mb)
            lat.step(1)
        res[mode] = (lat.populations_f64().cpu().numpy(), ma.positions(), mb.positions())
        lat.close()
    for u, w in zip(res[0], res[1]):
        assert np.array_equal(u, w)


def test_couple_requires_rest_shape(lbm):
    from paper_1110_0995_amd import _lib
    s = _small(posts=False, ncells=1)
    lat = lbm.Lattice.from_scenario(s, prec="f32")
    mesh = lbm.Mesh(lat, s.cells)
    mesh.s.checked = 0
    with pytest.raises(_lib.LbmError) as e:
        lat.couple(mesh)
    assert e.value.code == _lib.LBM_ESTATE


def test_graphs_after_a_pending_couple_f64(lbm):
    """ibm_couple(A) followed by a graph-replayed lbm_run(B) or a graphed
    lbm_run_record(B): the first step adds B's spread force to A's at the
    stencil nodes both share, exactly as the eager couple(A), couple(B),
    step does, also when a graph for B alone was captured before."""
    nx, ny, nz = 32, 24, 20
    cen = np.array([[12.2, 11.7, 9.6], [14.9, 12.3, 10.1]])
    mod = (0.01, 0.002, 0.005, 0.05, 0.2)
    a, b = S.make_cells(cen[:1], 3.0, 2, moduli=mod), S.make_cells(cen[1:], 3.0, 2, moduli=mod)
    s = S.Scenario("pending", nx, ny, nz, 0.8, (1e-4, 0, 0), S.channel_mask(nx, ny, nz), 10,
                   cells=S.make_cells(cen, 3.0, 2, moduli=mod))

    def go(graph):
        lat = lbm.Lattice.from_scenario(s, prec="f64")
        ma, mb = lbm.Mesh(lat, a), lbm.Mesh(lat, b)

        def run_b(n):
            if graph:
                lat.run(n, mb, steps_per_graph=2)
            else:
                for _ in range(n):
                    lat.couple(mb)
                    lat.step(1)

        run_b(4)            # captures B's graph with nothing pending
        lat.couple(ma)
        run_b(5)            # A pending before the first step
        lat.couple(ma)
        run_b(4)
        run_b(4)            # nothing pending again
        rec = lat.record_buffers(2, mb)
        for pending in (False, True):
            if pending:
                lat.couple(ma)
            lat.run_record(2, mb, rec, use_graph=graph)
        out = (lat.populations_f64().cpu().numpy(), ma.positions(), mb.positions(), mb.velocities())
        lat.close()
        return out

    eager, graphed = go(False), go(True)
    for u, w in zip(eager, graphed):
        assert np.array_equal(u, w)
