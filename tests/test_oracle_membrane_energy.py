"""Closed-form pins of the oracle's membrane energy (Sec. 2.3.1 and 2.3.3, the
moduli K^S, K^B, K^A_l, K^A_g, K^V of Table 1 as energies):

    E_s  = sum_edges (k_s/2) (l - l0)^2 / l0     (or the neo-Hookean edge law)
    E_b  = sum_hinges (k_b/2) (theta - theta0)^2
    E_al = sum_tris (k_al/2) (A - A0)^2 / A0
    E_ag = (k_ag/2) (A_c - A0_c)^2 / A0_c
    E_v  = (k_v/2) (V_c - V0_c)^2 / V0_c

Two shapes whose deformed geometry is known by hand:
  * a regular icosahedron scaled by lam about its centre: every edge, face,
    the area and the volume scale by lam, lam^2, lam^2, lam^3 and no angle
    changes (E_b = 0);
  * the regular octahedron (square bipyramid, half-diagonal 1, apex height 1)
    with both apexes moved to height h: the face normals are (+-h, +-h, +-1)
    up to length, so the two hinge classes have cos(theta) = 1/(2h^2 + 1)
    (4 + 4 apex edges) and (2h^2 - 1)/(2h^2 + 1) (4 base edges), every face
    has area sqrt(2h^2 + 1)/2, and the volume is 4h/3.
One modulus is non-zero at a time, so a swapped modulus index, a dropped
factor 1/2 or a missing normaliser (l0, A0, A0_c, V0_c) changes the value.
The forces are tied to the same closed forms through dE/dlam and dE/dh."""
import math

import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

PHI = (1 + math.sqrt(5)) / 2


def _cell(verts, tris, moduli, law=0):
    tris = np.asarray(tris, np.int64)
    h = S.hinges(tris)
    n = len(verts)
    return S.Cells(vert_off=np.array([0, n], np.int32), tri_off=np.array([0, len(tris)], np.int32),
                   edge_off=np.array([0, len(h)], np.int32), tri=tris.astype(np.int32),
                   hinge=h.astype(np.int32), anchor=np.zeros((1, 3), np.int32),
                   offset=np.asarray(verts, np.float32), moduli=np.array([moduli], np.float64),
                   stretch_law=law)


def _outward(verts, tris):
    v = np.asarray(verts)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    return np.all(np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c - 3 * v.mean(0)) > 0)


# --- the scaled icosahedron -------------------------------------------------

def _icosahedron():
    v, t = S.icosphere(0)
    a = 4.0 / math.sqrt(10.0 + 2.0 * math.sqrt(5.0))  # edge of the unit-circumradius icosahedron
    # the input is the regular icosahedron (a check on the generator, not on the oracle)
    e = S.hinges(t)
    assert len(v) == 12 and len(t) == 20 and len(e) == 30
    assert np.abs(np.linalg.norm(v[e[:, 1]] - v[e[:, 0]], axis=1) - a).max() < 1e-14
    assert _outward(v, t)
    return v, t, a


def _ico_terms(lam, a, law=0):
    """(E_s, E_b, E_al, E_ag, E_v) per unit modulus, and dE/dlam, by hand."""
    At = math.sqrt(3.0) / 4.0 * a * a
    A0c = 20.0 * At
    V0 = 5.0 / 12.0 * (3.0 + math.sqrt(5.0)) * a ** 3
    if law == 0:
        es, des = 30 * 0.5 * (lam - 1) ** 2 * a, 30 * (lam - 1) * a
    else:
        es, des = 30 * a / 6 * (lam ** 2 + 2 / lam - 3), 30 * a / 6 * (2 * lam - 2 / lam ** 2)
    E = (es, 0.0, 20 * 0.5 * (lam ** 2 - 1) ** 2 * At, 0.5 * (lam ** 2 - 1) ** 2 * A0c,
         0.5 * (lam ** 3 - 1) ** 2 * V0)
    dE = (des, 0.0, 20 * 2 * lam * (lam ** 2 - 1) * At, 2 * lam * (lam ** 2 - 1) * A0c,
          3 * lam ** 2 * (lam ** 3 - 1) * V0)
    return E, dE


@pytest.mark.parametrize("lam", [1.1, 0.93, 1.37])
@pytest.mark.parametrize("term", range(5))
def test_scaled_icosahedron_energy_closed_form(orc, term, lam):
    v, t, a = _icosahedron()
    centre = np.array([3.25, -1.5, 7.0])
    mod = np.zeros(5)
    mod[term] = 0.7
    cells = _cell(v + centre, t, mod)
    M = orc.Mesh(cells)
    X0 = v + centre
    M.rest_shape(X0)
    X = centre + lam * v
    E, dE = _ico_terms(lam, a)
    want = 0.7 * E[term]
    got = M.energy(X)
    assert abs(got - want) <= 1e-12 * max(abs(want), 1e-300) + 1e-15
    # forces: X = centre + lam v, so dE/dlam = -sum_k F_k . v_k
    F = M.forces(X)
    dwant = 0.7 * dE[term]
    assert abs(-(F * v).sum() - dwant) <= 1e-12 * max(abs(dwant), 1.0)


@pytest.mark.parametrize("lam", [1.1, 0.93])
def test_scaled_icosahedron_neo_hookean_closed_form(orc, lam):
    v, t, a = _icosahedron()
    cells = _cell(v, t, (0.4, 0, 0, 0, 0), law=1)
    M = orc.Mesh(cells)
    M.rest_shape(v)
    E, dE = _ico_terms(lam, a, law=1)
    assert abs(M.energy(lam * v) - 0.4 * E[0]) <= 1e-12 * 0.4 * E[0]
    assert abs(-(M.forces(lam * v) * v).sum() - 0.4 * dE[0]) <= 1e-12 * abs(0.4 * dE[0])


# --- the stretched bipyramid --------------------------------------------------

OCT_V = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)], np.float64)
OCT_T = np.array([(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4),
                  (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)], np.int64)


def _bipyramid(h):
    v = OCT_V.copy()
    v[4, 2], v[5, 2] = h, -h
    return v


def _bip_terms(h, law=0):
    """(E_s, E_b, E_al, E_ag, E_v) per unit modulus of the bipyramid of apex
    height h against the regular octahedron (h = 1), by hand."""
    l, l0 = math.sqrt(1 + h * h), math.sqrt(2.0)
    if law == 0:
        es = 8 * 0.5 * (l - l0) ** 2 / l0
    else:
        lam = l / l0
        es = 8 * l0 / 6 * (lam ** 2 + 2 / lam - 3)
    th_apex = lambda q: math.acos(1.0 / (2 * q * q + 1))
    th_base = lambda q: math.acos((2 * q * q - 1) / (2 * q * q + 1))
    eb = 0.5 * (8 * (th_apex(h) - th_apex(1.0)) ** 2 + 4 * (th_base(h) - th_base(1.0)) ** 2)
    A, A0 = 0.5 * math.sqrt(2 * h * h + 1), 0.5 * math.sqrt(3.0)
    eal = 8 * 0.5 * (A - A0) ** 2 / A0
    eag = 0.5 * (8 * A - 8 * A0) ** 2 / (8 * A0)
    V, V0 = 4 * h / 3, 4.0 / 3.0
    ev = 0.5 * (V - V0) ** 2 / V0
    return (es, eb, eal, eag, ev)


def test_bipyramid_geometry_is_what_the_closed_forms_assume(orc):
    """The hinge classes, areas and volume of the hand derivation, read from
    the oracle's geometry routines on the same shape."""
    assert _outward(OCT_V, OCT_T)
    h = 1.3
    cells = _cell(OCT_V, OCT_T, (0, 0, 0, 0, 0))
    M = orc.Mesh(cells)
    X = _bipyramid(h)
    l, A, th = M.geometry(X)
    hin = M.hinge
    apex = np.isin(hin[:, 0], (4, 5)) | np.isin(hin[:, 1], (4, 5))
    assert apex.sum() == 8
    assert np.allclose(th[apex], math.acos(1 / (2 * h * h + 1)), rtol=0, atol=1e-14)
    assert np.allclose(th[~apex], math.acos((2 * h * h - 1) / (2 * h * h + 1)), rtol=0, atol=1e-14)
    assert np.allclose(A, 0.5 * math.sqrt(2 * h * h + 1), rtol=0, atol=1e-15)
    Ac, Vc = M.area_volume(X)
    assert abs(Vc[0] - 4 * h / 3) < 1e-15 and abs(Ac[0] - 4 * math.sqrt(2 * h * h + 1)) < 1e-14


@pytest.mark.parametrize("h", [1.3, 0.8])
@pytest.mark.parametrize("term", range(5))
def test_bipyramid_energy_closed_form(orc, term, h):
    mod = np.zeros(5)
    mod[term] = 1.9
    cells = _cell(OCT_V, OCT_T, mod)
    M = orc.Mesh(cells)
    M.rest_shape(OCT_V)
    assert M.energy(OCT_V) == 0.0
    want = 1.9 * _bip_terms(h)[term]
    assert want > 0
    assert abs(M.energy(_bipyramid(h)) - want) <= 1e-12 * want
    # only the apexes move with h: dE/dh = -(F_4z - F_5z); the derivative of
    # the closed form by a central difference of step 1e-5 (error ~1e-10 relative)
    F = M.forces(_bipyramid(h))
    d = 1e-5
    dwant = 1.9 * (_bip_terms(h + d)[term] - _bip_terms(h - d)[term]) / (2 * d)
    assert abs(-(F[4, 2] - F[5, 2]) - dwant) <= 1e-8 * abs(dwant)


@pytest.mark.parametrize("h", [1.3, 0.8])
def test_bipyramid_neo_hookean_closed_form(orc, h):
    cells = _cell(OCT_V, OCT_T, (0.6, 0, 0, 0, 0), law=1)
    M = orc.Mesh(cells)
    M.rest_shape(OCT_V)
    want = 0.6 * _bip_terms(h, law=1)[0]
    assert abs(M.energy(_bipyramid(h)) - want) <= 1e-12 * want


def test_all_moduli_together_add_their_terms(orc):
    """Table 1's tumour-cell moduli on the bipyramid: the energy is the
    moduli-weighted sum of the five closed-form terms (in the order
    K^S, K^B, K^A_l, K^A_g, K^V)."""
    mod = np.asarray(S.MODULI_CTC, np.float64)
    cells = _cell(OCT_V, OCT_T, mod)
    M = orc.Mesh(cells)
    M.rest_shape(OCT_V)
    for h in (1.3, 0.8):
        want = float(np.dot(mod, _bip_terms(h)))
        assert abs(M.energy(_bipyramid(h)) - want) <= 1e-12 * want
