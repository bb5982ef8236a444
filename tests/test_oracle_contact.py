"""Pins of the oracle's contact forces (soft-sphere repulsion between cells and
from the walls; Sec. 2.4, collisions), CPU only.

Hand values of the law U(d) = a d^-n (a = 1, n = 2 unless said), the force
as the negative gradient of the energy (central differences), Newton's third
law for the cell-cell part, the cut-off, exclusion of pairs within one cell,
the periodic minimum image, hand values for planes, posts and fixed spheres,
the linear continuation below dmin, and momentum
conservation of a coupled step with contact forces on."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S


def _two_cells(orc, gap, axis=0, level=1, L=(40, 20, 20), contact=None, periodic=(1, 1, 1), radius=2.0):
    """Two icosphere cells whose closest vertices are `gap` apart along `axis`."""
    unit, _ = S.icosphere(level)
    c0 = np.array([10.0, 10.0, 10.0])
    # the vertex furthest along +axis of cell 0 and along -axis of cell 1
    ext = radius * unit[:, axis].max()
    c1 = c0.copy()
    c1[axis] += 2 * ext + gap
    cells = S.make_cells(np.array([c0, c1]), radius, level)
    # the generator stores float32 offsets: set the gap exactly in FP64
    X = cells.positions()
    nv0 = int(cells.vert_off[1])
    X[nv0:, axis] += X[:nv0, axis].max() + gap - X[nv0:, axis].min()
    cells.positions = lambda: X.copy()
    lat = orc.Lattice(*L, tau=0.8, periodic=periodic)
    M = orc.Mesh(cells, contact=contact)
    return lat, M, cells


def _law(**kw):
    d = dict(a=1.0, n=2.0, rcut=1.0, roff=0.0, dmin=0.05, cell_cell=1, planes=np.zeros((0, 4)), cyl=np.zeros((0, 3)))
    d.update(kw)
    return d


def test_pair_hand_value(orc):
    # closest vertices 0.5 apart along x: U = 1 * 0.5^-2 = 4 per such pair,
    # force magnitude 2 * 0.5^-3 = 16 along x, pushing the cells apart
    lat, M, cells = _two_cells(orc, 0.5, contact=_law())
    X = cells.positions()
    nv0 = cells.vert_off[1]
    i = np.argmax(X[:nv0, 0])
    j = nv0 + np.argmin(X[nv0:, 0])
    F = M.contact_forces(lat, X)
    assert F[i] == pytest.approx([-16.0, 0.0, 0.0], abs=1e-12)
    assert F[j] == pytest.approx([16.0, 0.0, 0.0], abs=1e-12)
    # every other pair is further than the cut-off for a level-1 sphere of radius 2
    others = np.ones(len(X), bool)
    others[[i, j]] = False
    assert np.abs(F[others]).max() == 0.0
    assert M.contact_energy(lat, X) == pytest.approx(4.0, rel=1e-14)


def test_cutoff_and_same_cell_exclusion(orc):
    lat, M, cells = _two_cells(orc, 1.0 + 1e-9, contact=_law())
    X = cells.positions()
    assert np.abs(M.contact_forces(lat, X)).max() == 0.0
    assert M.contact_energy(lat, X) == 0.0
    # one cell alone: its own vertices (edge ~1.2 apart, some pairs closer than
    # the cut-off after shrinking) never repel each other
    cells1 = S.make_cells(np.array([[10.0, 10.0, 10.0]]), 0.4, 1)
    M1 = orc.Mesh(cells1, contact=_law())
    assert np.abs(M1.contact_forces(lat, cells1.positions())).max() == 0.0


def test_force_is_minus_energy_gradient(orc):
    rng = np.random.default_rng(0)
    lat, M, cells = _two_cells(orc, 0.3, contact=_law(a=1e-3, n=1.5, rcut=1.2, roff=0.1, dmin=0.01,
                                                      planes=np.array([[0.0, 0.0, 1.0, 7.6]]),
                                                      cyl=np.array([[10.0, 7.3, 0.5]]),
                                                      spheres=np.array([[13.0, 10.4, 12.9, 0.6]])))
    X = cells.positions() + 0.05 * rng.standard_normal(cells.positions().shape)
    F = M.contact_forces(lat, X)
    assert np.abs(F).max() > 0
    # the sphere is within range of some vertices
    assert (np.linalg.norm(X - [13.0, 10.4, 12.9], axis=1) - 0.7 < 1.2).any()
    h = 1e-6
    for k in rng.choice(len(X), 12, replace=False).tolist() + list(np.nonzero(np.abs(F).sum(1))[0][:8]):
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, a] += h
            Xm[k, a] -= h
            fd = -(M.contact_energy(lat, Xp) - M.contact_energy(lat, Xm)) / (2 * h)
            assert F[k, a] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(F).max())


def test_cell_cell_forces_cancel(orc):
    rng = np.random.default_rng(1)
    lat, M, cells = _two_cells(orc, 0.2, level=2, contact=_law())
    X = cells.positions() + 0.1 * rng.standard_normal(cells.positions().shape)
    F = M.contact_forces(lat, X)
    assert np.abs(F).max() > 1.0
    assert np.abs(F.sum(0)).max() <= 1e-12 * np.abs(F).max()
    # central forces: zero net torque
    tq = np.cross(X, F).sum(0)
    assert np.abs(tq).max() <= 1e-11 * np.abs(F).max() * np.abs(X).max()


def test_periodic_minimum_image(orc):
    # the cells sit across the periodic x boundary: gap 0.5 through x = 0
    unit, _ = S.icosphere(1)
    r = 2.0
    ext = r * unit[:, 0].max()
    c0 = np.array([ext + 0.25, 10.0, 10.0])
    c1 = np.array([40.0 - ext - 0.25, 10.0, 10.0])
    cells = S.make_cells(np.array([c0, c1]), r, 1)
    M = orc.Mesh(cells, contact=_law())
    X = cells.positions()
    Fp = M.contact_forces(orc.Lattice(40, 20, 20, tau=0.8, periodic=(1, 1, 1)), X)
    Fw = M.contact_forces(orc.Lattice(40, 20, 20, tau=0.8, periodic=(0, 1, 1)), X)
    assert np.abs(Fw).max() == 0.0
    assert Fp[:, 0].max() == pytest.approx(16.0, rel=1e-12)  # cell 0 pushed to +x, away from the image
    assert Fp[:, 0].min() == pytest.approx(-16.0, rel=1e-12)


def test_walls_hand_values(orc):
    lat = orc.Lattice(40, 20, 20, tau=0.8, periodic=(1, 1, 0))
    cells = S.make_cells(np.array([[10.0, 10.0, 10.0]]), 2.0, 1)
    X = cells.positions()
    low = np.argmin(X[:, 2])
    # a plane 0.5 below the lowest vertex: U = 4, force +16 along its normal
    M = orc.Mesh(cells, contact=_law(planes=np.array([[0.0, 0.0, 1.0, X[low, 2] - 0.5]])))
    F = M.contact_forces(lat, X)
    assert F[low] == pytest.approx([0.0, 0.0, 16.0], abs=1e-12)
    # only vertices within the cut-off of the plane feel it, all along +z
    near = X[:, 2] - (X[low, 2] - 0.5) < 1.0
    assert np.all(F[near, 2] > 0) and np.abs(F[~near]).max() == 0.0 and np.abs(F[:, :2]).max() == 0.0
    # a z-cylinder whose surface is 0.25 from the vertex furthest along -y:
    # force 2 * 0.25^-3 = 128 along +y (away from the axis)
    south = np.argmin(X[:, 1])
    cyl = np.array([[X[south, 0], X[south, 1] - 0.25 - 1.5, 1.5]])
    M2 = orc.Mesh(cells, contact=_law(cyl=cyl))
    F2 = M2.contact_forces(lat, X)
    assert F2[south] == pytest.approx([0.0, 128.0, 0.0], abs=1e-9)
    # through the periodic y boundary: the same post shifted by ny acts the same
    M3 = orc.Mesh(cells, contact=_law(cyl=cyl + np.array([[0.0, 20.0, 0.0]])))
    assert np.abs(M3.contact_forces(lat, X) - F2).max() <= 1e-9


def test_sphere_hand_values(orc):
    """A fixed sphere (a bead of a frozen chain) whose surface is 0.4 from
    the vertex furthest along +x: force 2 * 0.4^-3 along the line from the
    centre; the same sphere seen through the periodic x boundary acts the
    same; with the axis not periodic its image is out of range."""
    cells = S.make_cells(np.array([[10.0, 10.0, 10.0]]), 2.0, 1)
    X = cells.positions()
    east = np.argmax(X[:, 0])
    R = 1.5
    u = np.array([1.0, 0.3, -0.2])
    u /= np.linalg.norm(u)
    c = X[east] + (R + 0.4) * u
    lat = orc.Lattice(40, 20, 20, tau=0.8, periodic=(1, 1, 0))
    F = orc.Mesh(cells, contact=_law(spheres=np.array([[*c, R]]))).contact_forces(lat, X)
    assert F[east] == pytest.approx(-2 * 0.4 ** -3 * u, rel=1e-12)
    near = np.linalg.norm(X - c, axis=1) - R < 1.0
    assert np.abs(F[~near]).max() == 0.0 and (np.abs(F[near]).sum(1) > 0).all()
    Fp = orc.Mesh(cells, contact=_law(spheres=np.array([[c[0] + 40.0, c[1], c[2], R]]))).contact_forces(lat, X)
    assert np.abs(Fp - F).max() <= 1e-9
    lat0 = orc.Lattice(40, 20, 20, tau=0.8, periodic=(0, 1, 0))
    F0 = orc.Mesh(cells, contact=_law(spheres=np.array([[c[0] + 40.0, c[1], c[2], R]]))).contact_forces(lat0, X)
    assert np.abs(F0).max() == 0.0


def test_linear_continuation_below_dmin(orc):
    # below dmin the energy continues with the slope at dmin: finite force, C1
    # energy (a short cut-off keeps every pair but the closest out of range)
    law = _law(dmin=0.1, rcut=0.3)
    for gap, force in ((0.05, 2 * 0.1 ** -3), (0.1 + 1e-12, 2 * 0.1 ** -3), (0.2, 2 * 0.2 ** -3)):
        lat, M, cells = _two_cells(orc, gap, contact=law)
        F = M.contact_forces(lat, cells.positions())
        assert np.abs(F[:, 0]).max() == pytest.approx(force, rel=1e-9)
    lat, M, cells = _two_cells(orc, 0.05, contact=law)
    # U(0.05) = U(0.1) + F(0.1) * 0.05 = 100 + 2000 * 0.05
    assert M.contact_energy(lat, cells.positions()) == pytest.approx(200.0, rel=1e-12)


def test_coupled_step_with_contact_conserves_momentum(orc):
    """Cell-cell contact forces are internal: in a periodic box without walls
    and with g = 0, fluid momentum + point momentum is conserved by a coupled
    step (the contact force enters the points' Newton equation)."""
    rng = np.random.default_rng(2)
    lat, M, cells = _two_cells(orc, 0.3, level=2, L=(24, 16, 16), contact=_law(a=1e-4), radius=2.5)
    M.rest_shape(cells.positions())
    X = cells.positions() + 0.02 * rng.standard_normal(cells.positions().shape)
    V = 1e-4 * rng.standard_normal(X.shape)
    f = lat.rest()
    m = M.point_mass()[:, None]
    P0 = orc.mass_momentum(lat, f)[1:] + (m * V).sum(0)
    Fk = M.contact_forces(lat, X)
    assert np.abs(Fk).max() > 1e-4
    for _ in range(3):
        f = orc.step(lat, M, f, X, V)
    P1 = orc.mass_momentum(lat, f)[1:] + (m * V).sum(0)
    assert np.abs(P1 - P0).max() <= 1e-13 * max(np.abs(m * V).sum(), 1e-10) + 1e-17
