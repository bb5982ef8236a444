"""Pins of the oracle's magnetic bead stage (the chain-forming stage of the
filter, Sec. 2.5: gradient force, dipole interaction, chains fixed in space),
CPU only.

  - the charge-sheet field: on the axis of a rectangle it equals sigma times
    the solid angle over 4 pi (closed form), far away it is the monopole
    field; off the axis field and gradient equal the corner closed form of a
    charged rectangle; the gradient is symmetric and traceless;
  - the dipole interaction equation: hand values for two aligned and two
    side-by-side moments, the negative gradient of the dipole energy, and
    Newton's third law;
  - the gradient force at fixed moment: zero in a uniform field, and the
    closed-form axial derivative on the axis of a sheet;
  - two beads in a uniform field settle along it at the separation where
    attraction and repulsion balance; many line up into chains;
  - freezing marks exactly the lattice nodes within a bead radius."""
import numpy as np
import pytest


def _axis_bz(sigma, A, B, d):
    """B_z at height d above the centre of a 2A x 2B sheet: sigma Omega / (4 pi)."""
    return sigma / np.pi * np.arctan(A * B / (d * np.sqrt(A * A + B * B + d * d)))


def test_sheet_field_closed_forms(orc):
    A, B = 20.0, 10.0
    G = orc.Magnet([[5.0, -A, A, -B, B, 2.0]], (0, 0, 0), 1.0, 1.0, 1.0, 1.0, quad=8)
    for d in (0.5, 1.0, 3.0, 10.0):
        up, down = G.field([[0, 0, 5.0 + d], [0, 0, 5.0 - d]])
        assert up[2] == pytest.approx(_axis_bz(2.0, A, B, d), rel=1e-9)
        assert down[2] == pytest.approx(-_axis_bz(2.0, A, B, d), rel=1e-9)
        assert np.abs(up[:2]).max() < 1e-12 and np.abs(down[:2]).max() < 1e-12
    # far field: a point charge sigma * area at the centre
    r = 30 * A
    for u in ([1, 0, 0], [0.6, 0.8, 0], [0, 0.6, 0.8]):
        u = np.array(u, float)
        Bf = G.field([[0, 0, 5.0] + r * u])[0]
        assert Bf == pytest.approx(2.0 * 4 * A * B / (4 * np.pi * r * r) * u, rel=2e-3, abs=1e-12)


def _rect_field(sheet, p):
    """Closed form of the field of a uniformly charged rectangle and of its
    gradient: sums over the four corners of log and arctangent terms (the
    antiderivatives of the Coulomb kernel over the rectangle)."""
    z, x0, x1, y0, y1, sig = sheet
    w = p[2] - z
    B, J = np.zeros(3), np.zeros((3, 3))
    for i, xc in enumerate((x0, x1)):
        for j, yc in enumerate((y0, y1)):
            s = (-1) ** (i + j)
            X, Y = xc - p[0], yc - p[1]
            R = np.sqrt(X * X + Y * Y + w * w)
            B += s * np.array([np.log(Y + R), np.log(X + R), np.arctan(X * Y / (w * R))])
            J[0, 0] -= s * X / (R * (Y + R))
            J[1, 1] -= s * Y / (R * (X + R))
            J[0, 1] -= s / R
            J[0, 2] += s * w / (R * (Y + R))
            J[1, 2] += s * w / (R * (X + R))
    J[1, 0], J[2, 0], J[2, 1] = J[0, 1], J[0, 2], J[1, 2]
    J[2, 2] = -J[0, 0] - J[1, 1]
    return sig / (4 * np.pi) * B, sig / (4 * np.pi) * J


def test_sheet_field_and_gradient_off_axis(orc):
    """Away from the axis: the quadrature equals the corner closed form for
    the field and its gradient, and the gradient equals central differences
    of the field (a check on the closed form's derivative terms too)."""
    sh = [3.0, -10.0, 30.0, -5.0, 25.0, 1.3]
    G = orc.Magnet([sh], (0, 0, 0), 1.0, 1.0, 1.0, 1.0)
    rng = np.random.default_rng(0)
    P = rng.uniform(-15, 35, (8, 3))
    P[:, 2] = np.where(np.abs(P[:, 2] - 3.0) < 1.0, 5.0, P[:, 2])
    Bo, Jo = G.field(P, jacobian=True)
    for p, bo, jo in zip(P, Bo, Jo):
        b, j = _rect_field(sh, p)
        assert np.abs(bo - b).max() <= 1e-13 * np.abs(b).max()
        assert np.abs(jo - j).max() <= 1e-12 * np.abs(j).max()
        h = 1e-4
        fd = np.array([(_rect_field(sh, p + h * e)[0] - _rect_field(sh, p - h * e)[0]) / (2 * h) for e in np.eye(3)]).T
        assert np.abs(j - fd).max() <= 1e-7 * np.abs(j).max()


def test_sheet_field_divergence_and_curl_free(orc):
    G = orc.Magnet([[0.0, -6, 6, -4, 4, 1.0], [8.0, -6, 6, -4, 4, -1.0]], (0.1, 0.0, 0.2), 1.0, 1.0, 1.0, 1.0)
    P = np.array([[1.0, 2.0, 3.0], [-4.5, 1.5, 1.0], [7.0, -5.0, 6.5]])
    _, J = G.field(P, jacobian=True)
    for j in J:
        scale = np.abs(j).max()
        assert abs(np.trace(j)) <= 1e-12 * scale
        assert np.abs(j - j.T).max() <= 1e-12 * scale


def test_dipole_interaction(orc):
    m, d = 1.7, 2.5
    mz = np.array([0.0, 0.0, m])
    # aligned along the moments: attraction -6 m^2 / (4 pi d^4) on bead 2
    F = orc.dipole_force(mz, mz, [0.0, 0.0, d])
    assert F == pytest.approx([0.0, 0.0, -6 * m * m / (4 * np.pi * d ** 4)], abs=1e-14)
    # side by side: repulsion 3 m^2 / (4 pi d^4)
    F = orc.dipole_force(mz, mz, [d, 0.0, 0.0])
    assert F == pytest.approx([3 * m * m / (4 * np.pi * d ** 4), 0.0, 0.0], abs=1e-14)
    rng = np.random.default_rng(0)
    for _ in range(5):
        m1, m2, r = rng.standard_normal(3), rng.standard_normal(3), 2 + rng.standard_normal(3)
        F = orc.dipole_force(m1, m2, r)
        h = 1e-6
        fd = np.array([-(orc.dipole_energy(m1, m2, r + h * e) - orc.dipole_energy(m1, m2, r - h * e)) / (2 * h)
                       for e in np.eye(3)])
        assert F == pytest.approx(fd, rel=1e-7, abs=1e-10)
        assert orc.dipole_force(m2, m1, -r) == pytest.approx(-F, rel=1e-13, abs=1e-16)


def test_gradient_force(orc):
    a, chi = 1.5, 4.0
    alpha = 4 * np.pi * a ** 3 * chi / (chi + 3)
    # uniform field: induced moment alpha B, no gradient force
    G = orc.Magnet([], (0.0, 0.0, 0.3), a, chi, 1.0, 1.0, rep=(0.0, 2.0, 0.1), dims=(64, 64, 64),
                   periodic=(0, 0, 0), walls_z=False)
    m, F = G.forces([[10.0, 10.0, 10.0]])
    assert m[0] == pytest.approx([0, 0, alpha * 0.3], rel=1e-14)
    assert np.abs(F).max() < 1e-15
    # on the axis of a sheet: F_z = m_z dB_z/dz from the closed form
    A, B, d, sig = 20.0, 10.0, 4.0, 1.0
    G = orc.Magnet([[0.0, -A, A, -B, B, sig]], (0, 0, 0), a, chi, 1.0, 1.0, rep=(0.0, 2.0, 0.1),
                   dims=(64, 64, 64), periodic=(0, 0, 0), walls_z=False, quad=8)
    m, F = G.forces([[0.0, 0.0, d]])
    bz = _axis_bz(sig, A, B, d)
    # d/dd of (sigma/pi) atan(f), f = AB / (d R), R = sqrt(A^2 + B^2 + d^2)
    R = np.sqrt(A * A + B * B + d * d)
    f = A * B / (d * R)
    dbz = sig / np.pi * (-A * B * (R * R + d * d) / (d * d * R ** 3)) / (1 + f * f)
    assert m[0, 2] == pytest.approx(alpha * bz, rel=1e-12)
    assert F[0, 2] == pytest.approx(alpha * bz * dbz, rel=1e-12)
    assert np.abs(F[0, :2]).max() < 1e-13 * abs(F[0, 2])


def test_bead_pair_settles_along_the_field(orc):
    """Two beads in a uniform field turn until their line of centres is
    parallel to it and stop where the dipole attraction 6 m^2 / (4 pi r^4)
    balances the soft-sphere repulsion n A g^-(n+1) (g = r - 2a), a root found
    here with a bracketing solver."""
    from scipy.optimize import brentq
    a, chi, bias, rep = 1.0, 4.0, 1.5, (0.1, 2.0, 1.0)
    m = 4 * np.pi * a ** 3 * chi / (chi + 3) * bias
    G = orc.Magnet([], (0.0, 0.0, bias), a, chi, 1.0, 0.1, rep=rep, dims=(32, 32, 32), periodic=(0, 0, 0),
                   walls_z=False)
    x = np.array([[10.0, 10.0, 10.0], [12.5, 10.5, 11.5]])
    c0 = x.mean(0)
    G.run(x, 20000)
    r = x[1] - x[0]
    g = brentq(lambda g: rep[1] * rep[0] * g ** (-rep[1] - 1) - 6 * m * m / (4 * np.pi * (2 * a + g) ** 4), 0.011, 1.0)
    assert np.linalg.norm(r) == pytest.approx(2 * a + g, rel=1e-9)
    assert np.abs(r[:2]).max() < 1e-9 and r[2] > 0
    # the pair forces are equal and opposite: the centre of mass stays put
    assert x.mean(0) == pytest.approx(c0, abs=1e-12)


def test_beads_form_chains_along_the_field(orc):
    rng = np.random.default_rng(3)
    n, a, L = 24, 1.0, 16
    G = orc.Magnet([], (0.0, 0.0, 1.5), a, 4.0, 1.0, 0.1, rep=(0.1, 2.0, 1.0), dims=(L, L, L),
                   periodic=(1, 1, 1), walls_z=False)
    # random positions at least 2.5 a apart (minimum image)
    x = []
    while len(x) < n:
        p = rng.uniform(0, L, 3)
        if all(np.linalg.norm((p - q + L / 2) % L - L / 2) > 2.5 * a for q in x):
            x.append(p)
    x = np.array(x)

    def alignment(x):
        d = x[:, None, :] - x[None, :, :]
        d = (d + L / 2) % L - L / 2
        r = np.linalg.norm(d, axis=2) + np.eye(n) * 1e9
        nn = d[np.arange(n), r.argmin(1)]
        return np.mean((nn[:, 2] / np.linalg.norm(nn, axis=1)) ** 2), r.min(1).mean()

    c0, r0 = alignment(x)
    G.run(x, 6000)
    c1, r1 = alignment(x)
    assert c0 < 0.5 and c1 > 0.95  # nearest neighbours now sit along the field
    assert 2 * a < r1 < 2.6 * a  # in contact, not overlapping


def test_freeze_marks_nodes_within_radius(orc):
    G = orc.Magnet([], (0, 0, 0), 2.5, 1.0, 1.0, 1.0, dims=(16, 16, 16), periodic=(1, 1, 1))
    solid = np.zeros(16 ** 3, np.uint8)
    G.freeze([[8.0, 8.0, 8.0]], solid)
    # integer points with x^2 + y^2 + z^2 <= 6.25: 1 + 6 + 12 + 8 + 6 + 24 + 24
    assert int(solid.sum()) == 81
    solid[:] = 0
    G.freeze([[0.0, 0.0, 0.0]], solid)  # wraps through every periodic face
    assert int(solid.sum()) == 81 and solid[15 + 16 * (0 + 16 * 0)] == 1


def test_wall_repulsion_and_mobility(orc):
    """No field: one overdamped step of a bead 0.3 above the bottom wall (and
    one 0.3 below the top wall) moves it by dt / (6 pi eta a) n A g^-(n+1)
    away from the wall."""
    a, eta, dt, rep = 1.2, 0.7, 0.05, (0.1, 2.0, 1.0)
    G = orc.Magnet([], (0.0, 0.0, 0.0), a, 4.0, eta, dt, rep=rep, dims=(16, 16, 40), periodic=(1, 1, 0),
                   walls_z=True)
    g = 0.3
    x = np.array([[5.0, 5.0, 0.5 + a + g], [9.0, 9.0, 40 - 1.5 - a - g]])
    x0 = x.copy()
    G.run(x, 1)
    step = dt / (6 * np.pi * eta * a) * rep[1] * rep[0] * g ** (-rep[1] - 1)
    assert x - x0 == pytest.approx(np.array([[0, 0, step], [0, 0, -step]]), rel=1e-13, abs=1e-16)
