"""GPU parity of the neo-Hookean stretching law and the biconcave red blood
cell (Sec. 2.3.1, Table 1 RBC column) against the FP64 oracle: elastic
forces and their Jacobian product, coupled FP64 steps, and a 600-step FP32
run of red cells and a tumour cell passing a post."""
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


def _rbc_scenario(nx=48, ny=32, nz=24, level=3, gx=5e-5):
    s = S.posts_and_cells(nx, ny, nz, posts_x=1, posts_y=1, post_radius=3, gap=8, ncells=0, tau=0.8, gx=gx)
    red = S.make_cells(np.array([[10.0, 8.0, 11.5], [10.0, 24.0, 11.5]]), 3.91, level, S.MODULI_RBC,
                       shape="rbc", stretch_law=1, mass=S.MASS_RBC)
    s.cells = red
    return s


def _to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype)


def test_neo_hookean_forces_and_jacobian(orc, lbm):
    import torch
    s = _rbc_scenario()
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells)
    M = orc.Mesh(s.cells)
    X0 = s.cells.positions()
    M.rest_shape(X0)
    rng = np.random.default_rng(4)
    X = X0 + 0.2 * rng.standard_normal(X0.shape)
    W = rng.standard_normal(X0.shape)
    off = X - s.cells.anchor[s.cells.vertex_cell()]
    f, jvp = mesh.force_jvp(_to_dev(off.T, torch.float64), _to_dev(W.T, torch.float64))
    Fo = M.forces(X)
    assert np.abs(f.cpu().numpy().T - Fo).max() <= 1e-12 * np.abs(Fo).max()
    h = 1e-6
    fd = (M.forces(X + h * W) - M.forces(X - h * W)) / (2 * h)
    assert np.abs(jvp.cpu().numpy().T - fd).max() <= 1e-6 * np.abs(fd).max()
    # the neo-Hookean law is in use: the linear law gives other forces
    Ml = orc.Mesh(s.cells, stretch_law=0)
    Ml.rest_shape(X0)
    assert np.abs(Ml.forces(X) - Fo).max() > 1e-3 * np.abs(Fo).max()


def test_rbc_coupled_f64_matches_oracle(orc, lbm):
    s = _rbc_scenario()
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    mesh = lbm.Mesh(lat, s.cells)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells)
    X = s.cells.positions()
    M.rest_shape(X)
    rng = np.random.default_rng(5)
    off = s.cells.offset.astype(np.float64) + 0.05 * rng.standard_normal(X.shape)
    mesh.set_offsets(off)
    X = s.cells.anchor[s.cells.vertex_cell()] + off
    V = np.zeros_like(X)
    f = L.rest()
    for _ in range(20):
        lat.couple(mesh)
        lat.step(1)
        f = orc.step(L, M, f, X, V)
    fl = s.solid.reshape(-1) == 0
    fg = lat.populations_f64().cpu().numpy()
    # FP64 rounding only (populations O(1/3), 20 steps with the stiff red-cell
    # moduli, FMA and another summation order on the GPU)
    assert np.abs(fg[:, fl] - f[:, fl]).max() < 3e-14
    assert np.abs(mesh.positions() - X).max() < 1e-12
    assert np.abs(mesh.velocities() - V).max() < 1e-13


def test_red_and_tumour_cells_f32dev(orc, lbm):
    """Two red cells (biconcave, RBC moduli) and a spherical tumour cell (CTC
    moduli), all neo-Hookean, pass a post with contact forces on: 600 FP32
    steps against the FP64 oracle."""
    import torch
    s = _rbc_scenario(gx=1e-4)
    ctc = S.make_cells(np.array([[36.0, 16.0, 11.5]]), 3.0, 2, S.MODULI_CTC, stretch_law=1, mass=S.MASS_RBC)
    s.cells = S.concat_cells([s.cells, ctc])
    contact = S.contact_params(s)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells, contact=contact)
    lat.run(600, mesh, steps_per_graph=50)
    torch.cuda.synchronize()
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells, contact=contact)
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = orc.run(L, M, L.rest(), X, V, nsteps=600)
    _, uo = orc.fluid_velocity(L, f)
    _, ug = lat.fields()
    fl = s.solid.reshape(-1) == 0
    ug = ug.double().cpu().numpy()
    err = np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl])
    assert err < 1e-5
    assert np.abs(mesh.positions() - X).max() < 1e-4
    # the cells moved and kept their volume (stiff volume modulus)
    assert np.abs(X.mean(0) - s.cells.positions().mean(0))[0] > 1.0


def test_red_cell_suspension_full_size(orc, lbm):
    """The benchmark's red-cell workload at full size (512x256x128, 1000
    randomly oriented red cells and 40 tumour cells, 642 vertices each,
    neo-Hookean): 3 FP32 coupled steps against the FP64 oracle (contact
    forces off: the oracle's all-pairs contact sum would take hours at this
    size; they are checked on sampled cells at full size elsewhere)."""
    s = S.red_cell_suspension()
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells)
    L = orc.Lattice.from_scenario(s)
    M = orc.Mesh(s.cells)
    X = s.cells.positions()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = orc.run(L, M, L.rest(), X, V, nsteps=3)
    lat.run(3, mesh)
    fl = s.solid.reshape(-1) == 0
    _, uo = orc.fluid_velocity(L, f)
    _, ug = lat.fields()
    ug = ug.double().cpu().numpy()
    err = np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl])
    print(f"red-cell suspension, 3 steps: u rel L2 {err:.3e}")
    assert err < 1e-5
    assert np.abs(mesh.positions() - X).max() < 1e-5
