"""GPU parity of the lattice path (collide-stream, bounce-back, forcing,
moments and FP64 sums) against the FP64 oracle, through the C ABI."""
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


def _gpu_u(lat):
    rho, u = lat.fields()
    return rho.double().cpu().numpy(), u.double().cpu().numpy()


def _random_state(orc, N, rng, amp=0.02):
    f = np.empty((19, N))
    for n in range(N):
        f[:, n] = orc.equilibrium(rng.uniform(0.97, 1.03), rng.uniform(-0.03, 0.03, 3)) * \
            (1 + amp * rng.uniform(-1, 1, 19))
    return f


def test_poiseuille_f64_1000_steps(orc, lbm):
    """64x16x16 FP64 channel, tau = 1, g = 1e-6, 1000 steps."""
    s = S.poiseuille()
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    lat.step(1000)
    L = orc.Lattice.from_scenario(s)
    f = L.rest()
    orc.run(L, None, f, nsteps=1000)
    _, uo = orc.fluid_velocity(L, f)
    _, ug = _gpu_u(lat)
    fl = s.solid.reshape(-1) == 0
    # FP64 rounding: populations (~0.05) agree to ~1e-14 relative; the velocity
    # is a difference of populations ~500x smaller than they are, so its
    # relative error is correspondingly larger
    fg = lat.populations_f64().cpu().numpy()
    assert np.abs(fg[:, fl] - f[:, fl]).max() < 1e-14
    assert rel_l2(ug, uo, fl) < 1e-10
    assert lat.steps_taken() == 1000
    # slip-corrected closed form (slowest mode still ~2.3e-4 of u_max)
    z = np.arange(1, s.nz - 1)
    ua = 3e-6 * (z - 0.5) * (14.5 - z) + 2.5e-7
    ux = ug[0].reshape(s.nz, s.ny, s.nx)[1:-1, 3, 5]
    assert np.abs(ux - ua).max() / ua.max() < 5e-4


@pytest.mark.parametrize("prec,tol", [("f32dev", 1e-5), ("f32", 2e-2)])
def test_poiseuille_f32_forms(orc, lbm, prec, tol):
    """FP32 deviation storage meets 1e-5 relative velocity error after 1000
    steps; plain FP32 storage is reported with a loose bound."""
    s = S.poiseuille()
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    lat.step(1000)
    L = orc.Lattice.from_scenario(s)
    f = L.rest()
    orc.run(L, None, f, nsteps=1000)
    _, uo = orc.fluid_velocity(L, f)
    _, ug = _gpu_u(lat)
    fl = s.solid.reshape(-1) == 0
    err = rel_l2(ug, uo, fl)
    print(f"poiseuille {prec}: velocity rel L2 error {err:.3e}")
    assert err < tol


def test_one_node_wide_channel(orc, lbm):
    """nx = ny = 1: every x/y link wraps onto the node itself."""
    s = S.poiseuille(1, 1, 16, tau=0.8, gx=1e-5)
    lat = lbm.Lattice.from_scenario(s, prec="f64")
    lat.step(3000)
    L = orc.Lattice.from_scenario(s)
    f = L.rest()
    orc.run(L, None, f, nsteps=3000)
    fl = s.solid.reshape(-1) == 0
    assert np.abs(lat.populations_f64().cpu().numpy()[:, fl] - f[:, fl]).max() < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32", "f32dev"])
def test_random_state_ragged_tiles(orc, lbm, prec):
    """nx = 100 (one full and one ragged 64-wide tile per row), a
    non-periodic y axis, random solid nodes, a random field G, a random
    non-equilibrium start: populations after 7 steps."""
    rng = np.random.default_rng(100)
    nx, ny, nz = 100, 7, 9
    solid = S.channel_mask(nx, ny, nz)
    solid |= (rng.uniform(size=solid.shape) < 0.08).astype(np.uint8)
    G = S.random_field(rng, (3, nz, ny, nx), 2e-4)
    per = (1, 0, 1)
    L = orc.Lattice(nx, ny, nz, 0.73, (3e-5, -1e-5, 2e-5), solid, per, G=G)
    f0 = _random_state(orc, L.N, rng)
    lat = lbm.Lattice(nx, ny, nz, 0.73, (3e-5, -1e-5, 2e-5), solid, prec, per, gfield=G)
    lat.load_f64(f0)
    f = f0.copy()
    orc.run(L, None, f, nsteps=7)
    lat.step(7)
    fg = lat.populations_f64().cpu().numpy()
    fl = solid.reshape(-1) == 0
    err = np.abs(fg[:, fl] - f[:, fl]).max()
    tol = {"f64": 1e-15, "f32": 5e-7, "f32dev": 2e-8}[prec]
    print(f"ragged {prec}: max population error {err:.3e}")
    assert err < tol
    _, ug = _gpu_u(lat)
    _, uo = orc.fluid_velocity(L, f)
    assert rel_l2(ug, uo, fl) < {"f64": 1e-13, "f32": 1e-4, "f32dev": 1e-5}[prec]
    sums = lat.sums()
    so = orc.mass_momentum(L, f)
    # plain FP32 storage rounds rho = sum f_i near 1 every step (the reason for
    # the deviation storage), so its mass drifts by ~1e-7 relative
    assert abs(sums[0] - so[0]) / so[0] < {"f64": 1e-14, "f32": 1e-6, "f32dev": 1e-9}[prec]


def test_zero_steps_and_state_pointer(lbm):
    s = S.poiseuille(64, 4, 6)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    before = lat.current().clone()
    lat.step(0)
    assert lat.steps_taken() == 0
    assert (lat.current() == before).all()
    assert (before == 0).all()  # deviations of the fluid at rest
    assert lat.current().data_ptr() == lat.f_a.data_ptr()
    lat.step(1)
    assert lat.current().data_ptr() == lat.f_b.data_ptr() and lat.steps_taken() == 1


def test_rest_state_exact_f32dev(lbm):
    """Deviation storage keeps a fluid at rest bit-exactly at rest."""
    s = S.posts_and_cells(96, 64, 24, posts_x=2, posts_y=1, ncells=0, gx=0.0)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    lat.step(200)
    assert (lat.current() == 0).all()


def test_mass_conservation_f32dev(lbm):
    s = S.posts_and_cells(128, 64, 32, posts_x=2, posts_y=1, ncells=0, gx=1e-5)
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    m0 = lat.sums()[0]
    lat.step(2000)
    m1 = lat.sums()
    assert abs(m1[0] - m0) / m0 < 1e-9
    assert m1[1] > 0  # the flow has started along +x


def test_periodic_box_momentum_f64(orc, lbm):
    rng = np.random.default_rng(7)
    nx, ny, nz = 70, 6, 5
    G = S.random_field(rng, (3, nz, ny, nx), 1e-3)
    g = (1e-4, -2e-4, 3e-4)
    lat = lbm.Lattice(nx, ny, nz, 0.9, g, None, "f64", gfield=G)
    f0 = _random_state(orc, nx * ny * nz, rng)
    lat.load_f64(f0)
    p0 = lat.sums()
    lat.step(50)
    p1 = lat.sums()
    Ftot = np.array(g) * nx * ny * nz + G.reshape(3, -1).sum(1)
    assert abs(p1[0] - p0[0]) < 1e-12 * p0[0]
    assert np.allclose(p1[1:], p0[1:] + 50 * Ftot, rtol=0, atol=1e-12 * p0[0])


@pytest.mark.parametrize("nx", [150, 700])
def test_row_workgroups_match_other_shapes(lbm, nx):
    """One channel: the automatic collide-stream shape (whole x rows per
    workgroup in natural order when a row is at most 8 tiles: nx = 150, 3
    tiles; 4 renumbered tiles otherwise: nx = 700, 11 tiles) gives bitwise
    the results of explicit shapes, with cells, posts and a ragged last
    tile."""
    import torch
    from paper_1110_0995_amd import scenario as S
    s = S.posts_and_cells(nx, 24, 16, posts_x=1, posts_y=1, post_radius=3, gap=6, ncells=2, cell_radius=3.0, level=2,
                          gx=1e-4, seed=5)
    out = []
    for waves in (0, 1, 4, 8):
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm.Mesh(lat, s.cells)
        lat.set_launch(waves, 0)
        lat.run(10, mesh, steps_per_graph=0)
        lat.run(10, mesh, steps_per_graph=10)
        torch.cuda.synchronize()
        out.append((lat.current().cpu().numpy(), mesh.positions()))
        lat.close()
    for f, x in out[1:]:
        assert np.array_equal(f, out[0][0]) and np.array_equal(x, out[0][1])


def test_step_timed_is_step(lbm):
    """lbm_step_timed takes the same step as lbm_step (bitwise, with cells,
    posts and a ragged last tile) and sets its two events to the pass
    kernel's own start and end (a positive duration no longer than events
    recorded around the call)."""
    import torch
    s = S.posts_and_cells(150, 24, 16, posts_x=1, posts_y=1, post_radius=3, gap=6, ncells=2, cell_radius=3.0,
                          level=2, gx=1e-4, seed=5)
    stream = torch.cuda.current_stream()
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ka.record(stream)
    kb.record(stream)
    out = []
    for timed in (False, True):
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm.Mesh(lat, s.cells)
        for _ in range(6):
            lat.couple(mesh)
            if timed:
                a.record(stream)
                lat.step_timed(ka.cuda_event, kb.cuda_event)
                b.record(stream)
                torch.cuda.synchronize()
                t_kernel, t_call = ka.elapsed_time(kb), a.elapsed_time(b)
                assert 0.0 < t_kernel <= t_call
            else:
                lat.step(1)
        torch.cuda.synchronize()
        out.append((lat.current().cpu().numpy(), mesh.positions()))
        if timed:  # a missing event is refused without stepping
            from paper_1110_0995_amd import _lib
            with pytest.raises(_lib.LbmError) as e:
                lat.step_timed(0, kb.cuda_event)
            assert e.value.code == _lib.LBM_EINVAL and lat.steps_taken() == 6
        lat.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
