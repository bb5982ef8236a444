"""GPU parity of the staged filter run (Sec. 2.5: chains formed, fixed in
space, then fluid and cells; Sec. 2.4 collisions with the fixed chains)
against the FP64 oracle:

  - frozen beads as contact spheres: coupled FP64 steps of a cell next to a
    chain, with a second chain across the periodic x boundary and beads
    spread over many cells of the sphere grid;
  - the whole pipeline on a small channel: bead stage, freezing (the masks
    bitwise), then a coupled FP32 run of cells upstream of the chains."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm, magnet, pipeline
    return lbm, magnet, pipeline


def _stage(x, dims, a=1.5):
    return S.BeadStage(x=np.asarray(x, np.float64), sheets=np.zeros((0, 6)), bias=(0.0, 0.0, 0.5), a=a, chi=4.0,
                       eta=0.1, dt=0.012, rep=(0.5, 2.0, 1.0), dims=dims, periodic=(1, 1, 0), walls_z=True)


def _oracle_stage(orc, st):
    return orc.Magnet(st.sheets, st.bias, st.a, st.chi, st.eta, st.dt, rep=st.rep, dims=st.dims,
                      periodic=st.periodic, walls_z=st.walls_z)


def _chains(dims, rng, keep_clear, extra=60):
    """A chain along z at (24, 16), one at x = 0.4 next to the periodic x
    face, and extra beads spread over the channel, apart from each other,
    from the chains and from the points keep_clear (the cells' centres)."""
    nx, ny, nz = dims
    zs = np.arange(2.5, nz - 3.0, 3.1)
    x = [[24.0, 16.0, z] for z in zs] + [[0.4, 8.0, z] for z in zs]
    L = np.array([nx, ny])
    while len(x) < 2 * len(zs) + extra:
        p = rng.uniform([0, 0, 2.5], [nx, ny, nz - 3.5])
        d = np.asarray(x) - p
        d[:, :2] -= L * np.floor(d[:, :2] / L + 0.5)
        c = np.asarray(keep_clear)[:, :2] - p[:2]
        c -= L * np.floor(c / L + 0.5)
        if np.linalg.norm(d, axis=1).min() > 4.5 and np.linalg.norm(c, axis=1).min() > 7.0:
            x.append(list(p))
    return np.array(x)


def test_sphere_contact_steps_f64(orc, gpu):
    import torch
    lbm, magnet, _ = gpu
    dims = (48, 32, 24)
    nx, ny, nz = dims
    rng = np.random.default_rng(11)
    a = 1.5
    unit, _ = S.icosphere(2)
    R = 3.0
    ext = R * unit[:, 0].max()
    # cells whose furthest vertex along +x is 0.3 from the surface of the
    # fourth bead of a chain: of the chain at x = 24, and of the chain at
    # x = 0.4 seen across the periodic x face
    cen1 = np.array([24.0 - (a + 0.5) - 0.3 - ext, 16.0, 0.0])
    cen2 = np.array([nx + 0.4 - (a + 0.5) - 0.3 - ext, 8.0, 0.0])
    xb = _chains(dims, rng, [cen1, cen2])
    cen1[2] = cen2[2] = xb[3, 2]
    st = _stage(xb, dims, a)
    # masks: the GPU's freeze for the GPU lattice, the oracle's for the oracle's
    solid = torch.as_tensor(S.channel_mask(nx, ny, nz).reshape(-1)).cuda()
    magnet.Beads(st).freeze(solid)
    solid_g = solid.cpu().numpy().reshape(nz, ny, nx)
    solid_o = _oracle_stage(orc, st).freeze(xb, S.channel_mask(nx, ny, nz).reshape(-1).copy()).reshape(nz, ny, nx)
    assert np.array_equal(solid_g, solid_o)
    cells = S.make_cells(cen1[None], R, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    s = S.Scenario("spheres", nx, ny, nz, 0.8, (1e-4, 0.0, 0.0), solid_g, 6, cells=cells)
    contact = S.contact_params(s, a=1e-4, spheres=S.bead_spheres(xb, st.a))
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, cells, contact=contact)
    lat.run(6, mesh)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(cells, contact=contact)
    X = cells.positions()
    M.rest_shape(X)
    # the spheres act in this configuration (the planes alone do not)
    Fs = M.contact_forces(L, X)
    Mp = orc.Mesh(cells, contact=dict(contact, spheres=np.zeros((0, 4))))
    assert np.abs(Fs - Mp.contact_forces(L, X)).max() > 1e-3
    V = np.zeros_like(X)
    f = L.rest()
    for _ in range(6):
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    fg = lat.populations_f64().cpu().numpy()
    assert np.abs(fg[:, fl] - f[:, fl]).max() < 3e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13
    # the same cell next to the image of the chain across x = 0
    cells2 = S.make_cells(cen2[None], R, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    F2 = orc.Mesh(cells2, contact=contact).contact_forces(L, cells2.positions())
    F2p = orc.Mesh(cells2, contact=dict(contact, spheres=np.zeros((0, 4)))).contact_forces(L, cells2.positions())
    assert np.abs(F2 - F2p).max() > 1e-3
    s2 = S.Scenario("spheres", nx, ny, nz, 0.8, (1e-4, 0.0, 0.0), solid_g, 6, cells=cells2)
    lat2 = lbm.Lattice.from_scenario(s2, prec="f64")
    mesh2 = lbm.Mesh(lat2, cells2, contact=contact)
    lat2.run(2, mesh2)
    M2 = orc.Mesh(cells2, contact=contact)
    X2 = cells2.positions()
    M2.rest_shape(X2)
    V2 = np.zeros_like(X2)
    f2 = L.rest()
    for _ in range(2):
        f2 = orc.step(L, M2, f2, X2, V2)
    assert np.abs(mesh2.velocities() - V2).max() < 1e-13
    assert np.abs(mesh2.positions() - X2).max() < 1e-12


def test_pipeline_small(orc, gpu):
    """Bead stage (40 beads in a band, bias field, 3000 steps), freezing,
    then two cells upstream in a 400-step FP32 run; every stage against the
    oracle's own run of the same stage."""
    lbm, _, pipeline = gpu
    dims = (96, 48, 32)
    st = S.bead_stage(*dims, n=40, seed=4, xband=(40.0, 64.0), sheets=False, bias=1.5)
    cells = S.make_cells(np.array([[16.0, 16.0, 15.5], [16.0, 34.0, 15.5]]), 3.0, 2, S.MODULI_CTC)
    cf = pipeline.chain_filter(st, 3000, cells, gx=1e-4, steps=400)
    G = _oracle_stage(orc, st)
    xo = G.run(st.x.copy(), 3000)
    assert np.abs(cf.beads - xo).max() < 1e-8
    assert np.abs(xo - st.x).max() > 1.0  # the beads moved into chains
    so = G.freeze(xo, S.channel_mask(*dims).reshape(-1).copy()).reshape(dims[2], dims[1], dims[0])
    assert np.array_equal(cf.scenario.solid, so)
    s = cf.scenario
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, cells, contact=cf.contact)
    lat.run(400, mesh, steps_per_graph=50)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(cells, contact=S.contact_params(s, spheres=S.bead_spheres(xo, st.a)))
    X = cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = orc.run(L, M, L.rest(), X, V, nsteps=400)
    _, uo = orc.fluid_velocity(L, f)
    _, ug = lat.fields()
    fl = s.solid.reshape(-1) == 0
    ug = ug.double().cpu().numpy()
    assert np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl]) < 1e-5
    assert np.abs(mesh.positions() - X).max() < 1e-4


def test_sphere_outside_the_lattice_f64(orc, gpu):
    """A contact sphere centred below z = 0 (outside the lattice along its
    non-periodic axis; the grid clamps it into the bottom cells) and one
    far above the top, with a cell resting just above the first: coupled
    FP64 steps equal the oracle's, and the sphere acts."""
    lbm, _, _ = gpu
    nx, ny, nz = 40, 32, 24
    unit, _ = S.icosphere(2)
    R = 3.0
    low = R * -unit[:, 2].min()
    cen = np.array([20.0, 16.0, 0.0])
    sph = np.array([[20.0, 16.0, -0.4, 2.0], [7.0, 9.0, nz + 5.0, 2.0]])
    cen[2] = sph[0, 2] + sph[0, 3] + 0.3 + low  # lowest vertex 0.3 above the sphere's top
    cells = S.make_cells(cen[None], R, 2, moduli=(0.02, 0.005, 0.01, 0.1, 0.5))
    s = S.Scenario("below", nx, ny, nz, 0.8, (1e-4, 0.0, 0.0), S.channel_mask(nx, ny, nz), 4, cells=cells,
                   periodic=(1, 1, 0))
    contact = S.contact_params(s, a=1e-4, planes=np.zeros((0, 4)), spheres=sph)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(cells, contact=contact)
    X = cells.positions()
    M.rest_shape(X)
    Fs = M.contact_forces(L, X)
    assert np.abs(Fs).max() > 1e-3
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, cells, contact=contact)
    lat.run(4, mesh)
    V = np.zeros_like(X)
    f = L.rest()
    for _ in range(4):
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 3e-14
    assert np.abs(mesh.velocities() - V).max() < 1e-13
    assert np.abs(mesh.positions() - X).max() < 1e-12
