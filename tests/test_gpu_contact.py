"""GPU parity of the contact forces (Sec. 2.4, collisions) against the FP64
oracle: cell-cell repulsion and wall repulsion inside a coupled step, across
a periodic boundary, in a batch, at full size on sampled cells, and a longer
FP32 run in which the cells stay apart."""
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


def _close_pair(gap=0.3, L=(48, 32, 24), radius=3.0, level=2, post=True, seed=3):
    """A small channel (walls z = 0, nz-1, one post) with two cells whose
    closest vertices are `gap` apart and the lower one near the bottom wall."""
    nx, ny, nz = L
    s = S.posts_and_cells(nx, ny, nz, posts_x=1 if post else 0, posts_y=1 if post else 0, post_radius=3, gap=6,
                          ncells=0, tau=0.8, gx=1e-4, seed=seed)
    unit, _ = S.icosphere(level)
    ext = radius * unit[:, 0].max()
    c0 = np.array([10.0, 8.0, radius + 1.1])
    c1 = c0 + np.array([2 * ext + gap, 0.0, 0.0])
    cells = S.make_cells(np.array([c0, c1]), radius, level, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    s.cells = cells
    return s


def _law(s, **kw):
    return S.contact_params(s, a=1e-4, **kw)


def _oracle_step(orc, s, contact, nsteps, X=None, V=None):
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells, contact=contact)
    X0 = s.cells.positions()
    M.rest_shape(X0)
    X = X0.copy() if X is None else X.copy()
    V = np.zeros_like(X0) if V is None else V.copy()
    f = L.rest()
    for _ in range(nsteps):
        f = orc.step(L, M, f, X, V)
    return L, M, f, X, V


def test_contact_step_matches_oracle_f64(orc, lbm):
    s = _close_pair()
    contact = _law(s)
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    nsteps = 6
    lat.run(nsteps, mesh)
    L, M, f, X, V = _oracle_step(orc, s, contact, nsteps)
    # the contact forces actually act in this configuration
    Fk = M.contact_forces(L, s.cells.positions())
    assert np.abs(Fk).max() > 1e-4
    fl = s.solid.reshape(-1) == 0
    fg = lat.populations_f64().cpu().numpy()
    assert np.abs(fg[:, fl] - f[:, fl]).max() < 1e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13
    # without contact the trajectory is measurably different
    L2, M2, f2, X2, V2 = _oracle_step(orc, s, None, nsteps)
    assert np.abs(X2 - X).max() > 1e-6


def test_cell_cell_force_in_membrane_force(orc, lbm):
    """After ibm_couple, f_el holds elastic + cell-cell contact forces of the
    positions at the start of the step (the walls act inside the point
    update); compare with the oracle's two terms at those positions."""
    import torch
    s = _close_pair(gap=0.2)
    contact = _law(s)
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    X = s.cells.positions()
    lat.couple(mesh)
    torch.cuda.synchronize()
    fg = mesh.f_el.cpu().numpy().T
    M = orc.Mesh(s.cells, contact=dict(contact, planes=np.zeros((0, 4)), cyl=np.zeros((0, 3))))
    M.rest_shape(X)
    L = orc.Lattice.from_scenario(s)
    ref = M.forces(X) + M.contact_forces(L, X)
    assert np.abs(M.contact_forces(L, X)).max() > 1e-3
    assert np.abs(fg - ref).max() <= 1e-12 * np.abs(ref).max()


def test_contact_across_periodic_boundary(orc, lbm):
    import torch
    s = _close_pair(post=False)
    unit, _ = S.icosphere(2)
    ext = 3.0 * unit[:, 0].max()
    c0 = np.array([ext + 0.15, 16.0, 12.0])
    c1 = np.array([s.nx - ext - 0.15, 16.0, 12.0])
    s.cells = S.make_cells(np.array([c0, c1]), 3.0, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    contact = _law(s, planes=np.zeros((0, 4)), cyl=np.zeros((0, 3)))
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    X = s.cells.positions()
    lat.couple(mesh)
    torch.cuda.synchronize()
    M = orc.Mesh(s.cells, contact=contact)
    M.rest_shape(X)
    L = orc.Lattice.from_scenario(s)
    Fk = M.contact_forces(L, X)
    assert np.abs(Fk).max() > 1e-3
    ref = M.forces(X) + Fk
    fg = mesh.f_el.cpu().numpy().T
    assert np.abs(fg - ref).max() <= 1e-12 * np.abs(ref).max()


def test_contact_in_batch_matches_channel_alone(lbm):
    """Two cells per channel: at most one cell pair per channel, so each point
    gets at most one contact add and the result is deterministic: bitwise."""
    import torch
    scs = S.gap_sweep(3, lengths=(40, 64), ny=32, nz=16, gap_range=(4, 8), post_radius=4, ncells=2,
                      cell_radius=3.0, level=2, tau=0.8, gx=1e-4, seed=21)
    for s in scs:
        s.cells.moduli[:] = (0.02, 0.005, 0.01, 0.1, 0.5)
    lat = lbm.Lattice.batch(scs)
    cells, chan = S.batch_cells(scs)
    mesh = lbm.Mesh(lat, cells, chan, contact=S.contact_params_batch(scs, a=1e-4, rcut=3.0))
    lat.run(20, mesh)
    torch.cuda.synchronize()
    fb = lat.current().cpu().numpy()
    xb = mesh.x.cpu().numpy()
    moved = 0
    for k, s in enumerate(scs):
        la = lbm.Lattice.from_scenario(s)
        ma = lbm.Mesh(la, s.cells, contact=S.contact_params(s, a=1e-4, rcut=3.0))
        la.run(20, ma)
        torch.cuda.synchronize()
        assert np.array_equal(fb[:, lat.channel(k)], la.current().cpu().numpy()), f"channel {k}"
        idx = np.nonzero(chan == k)[0]
        v0, v1 = int(cells.vert_off[idx[0]]), int(cells.vert_off[idx[-1] + 1])
        assert np.array_equal(xb[:, v0:v1], ma.x.cpu().numpy())
        # the walls are within range of some points (rcut 3 from z = 1/2)
        lo = (s.cells.positions()[:, 2] - 0.5).min()
        moved += lo < 3.0
        la.close()
    assert moved > 0


def test_full_size_sampled_contact(orc, lbm):
    """Posts-and-cells workload at full size (256x128x64, 20 cells of 642
    vertices), FP32 deviation storage: cell 1 is moved next to cell 0; after
    one coupled step the membrane force of both equals the oracle's elastic
    + contact force computed on those two cells alone."""
    import torch
    s = S.posts_and_cells()
    contact = S.contact_params(s, a=1e-4)
    X = s.cells.positions()
    vo = s.cells.vert_off
    # move cell 1 so that its closest vertex is 0.3 from cell 0's furthest along x
    a0, a1 = slice(vo[0], vo[1]), slice(vo[1], vo[2])
    shift = X[a0].mean(0) - X[a1].mean(0) + np.array([X[a0, 0].max() - X[a0].mean(0)[0] +
                                                     (X[a1].mean(0)[0] - X[a1, 0].min()) + 0.3, 0.0, 0.0])
    off = s.cells.offset.astype(np.float64).copy()
    off[a1] += shift
    Xn = s.cells.anchor[s.cells.vertex_cell()] + off
    rest = slice(vo[2], None)
    for part in (a0, a1):  # the moved pair is out of range of every other cell
        d = np.linalg.norm(Xn[part][:, None, :] - Xn[rest][None, :, :], axis=2).min()
        assert d > contact["rcut"] + contact["roff"]
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    mesh.set_offsets(off)
    lat.couple(mesh)
    torch.cuda.synchronize()
    fg = mesh.f_el.double().cpu().numpy().T
    Xn = s.cells.anchor[s.cells.vertex_cell()] + off
    sub = S.Cells(vert_off=vo[:3] - 0, tri_off=s.cells.tri_off[:3], edge_off=s.cells.edge_off[:3],
                  tri=s.cells.tri[:s.cells.tri_off[2]], hinge=s.cells.hinge[:s.cells.edge_off[2]],
                  anchor=s.cells.anchor[:2], offset=s.cells.offset[:vo[2]], moduli=s.cells.moduli[:2])
    M = orc.Mesh(sub, contact=dict(contact, planes=np.zeros((0, 4)), cyl=np.zeros((0, 3))))
    M.rest_shape(s.cells.positions()[:vo[2]])
    L = orc.Lattice.from_scenario(s)
    Fk = M.contact_forces(L, Xn[:vo[2]])
    assert np.abs(Fk).max() > 1e-4
    ref = M.forces(Xn[:vo[2]]) + Fk
    # FP32 storage of the forces: rounding 6e-8 of the largest
    assert np.abs(fg[:vo[2]] - ref).max() <= 1e-6 * np.abs(ref).max()


def test_cells_stay_apart_f32dev(lbm):
    """300 steps with the cells pushed together by the flow around the post:
    the points of different cells never come closer than dmin."""
    import torch
    s = _close_pair(gap=0.4)
    contact = _law(s)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    vo = s.cells.vert_off
    dmin = np.inf
    for _ in range(6):
        lat.run(50, mesh, steps_per_graph=50)
        torch.cuda.synchronize()
        X = mesh.positions()
        d = np.linalg.norm(X[vo[0]:vo[1], None, :] - X[None, vo[1]:vo[2], :], axis=2).min()
        dmin = min(dmin, d)
        assert np.isfinite(X).all()
    assert dmin > contact["dmin"]
