"""GPU parity of the magnetic bead stage (Sec. 2.5, Eqs. Fstart and
interaction) against the FP64 oracle, through the mag_* C-ABI:

  - sheet field and gradient (closed form on the GPU, quadrature in the
    oracle) at points across the channel;
  - moments and total forces on small suspensions with a ragged last tile,
    beads in contact and next to the walls;
  - 60 overdamped steps;
  - fixing the beads into the solid mask, bitwise, with periodic wrap and
    clipping at the non-periodic faces;
  - a bead pair settling at the closed-form balance separation, chains
    forming along the field in a longer run;
  - at full size (16384 beads in the 512 x 256 x 128 channel, the launch
    the benchmark times) the forces on sampled beads."""
import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mag():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import magnet as mod
    return mod


def _oracle(orc, st):
    return orc.Magnet(st.sheets, st.bias, st.a, st.chi, st.eta, st.dt, rep=st.rep, dims=st.dims,
                      periodic=st.periodic, walls_z=st.walls_z)


def _small(n=300, seed=1, dims=None):
    dims = dims or ((96, 64, 32) if n > 400 else (64, 48, 32))
    return S.bead_stage(*dims, n=n, seed=seed)


def _touching(st, rng, pairs=12, walls=6):
    """Move some beads into contact and next to the walls, so that every
    force term acts: surface gaps in (0.35, 0.95) cut to the partner bead
    and (0.4, 0.9) cut to a wall, where the explicit update stays stable
    (mobility times contact stiffness below 2), and no other bead closer
    than 1.2 cut."""
    x = st.x.copy()
    a, cut = st.a, st.rep[2]
    L = np.array(st.dims, float)
    nz = st.dims[2]

    def clear(p, skip, wall=False):
        d = x - p
        d[:, :2] -= L[:2] * np.floor(d[:, :2] / L[:2] + 0.5)
        r = np.linalg.norm(d, axis=1)
        r[list(skip)] = np.inf
        return r.min() > 2 * a + 1.2 * cut and (wall or 0.5 + a + 1.2 * cut < p[2] < nz - 1.5 - a - 1.2 * cut)

    for k in range(pairs):
        i, j = 2 * k, 2 * k + 1
        for _ in range(1000):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            p = x[i] + (2 * a + rng.uniform(0.35, 0.95) * cut) * u
            if clear(p, (i, j)):
                x[j] = p
                break
        else:
            raise RuntimeError("no room for a contact pair")
    i = 2 * pairs
    for k in range(walls):
        g = rng.uniform(0.4, 0.9) * cut
        while True:
            p = x[i].copy()
            p[2] = 0.5 + a + g if k % 2 == 0 else nz - 1.5 - a - g
            i += 1
            if clear(p, (i - 1,), wall=True):
                x[i - 1] = p
                break
    return x


def test_field_and_gradient(orc, mag):
    st = _small()
    b = mag.Beads(st)
    G = _oracle(orc, st)
    rng = np.random.default_rng(0)
    nx, ny, nz = st.dims
    P = np.column_stack([rng.uniform(-20, nx + 20, 200), rng.uniform(-20, ny + 20, 200), rng.uniform(0.5, nz - 1.5, 200)])
    B, J = b.field(P, jacobian=True)
    Bo, Jo = G.field(P, jacobian=True)
    B, J = B.cpu().numpy().T, J.cpu().numpy().T.reshape(-1, 3, 3)
    for k in range(len(P)):
        assert np.abs(B[k] - Bo[k]).max() <= 1e-12 * np.abs(Bo[k]).max(), P[k]
        assert np.abs(J[k] - Jo[k]).max() <= 1e-12 * np.abs(Jo[k]).max(), P[k]


@pytest.mark.parametrize("n,rep_n", [(1, 2.0), (257, 2.0), (300, 2.0), (700, 2.0), (300, 2.5)])
def test_forces(orc, mag, n, rep_n):
    """rep_n = 2 takes the integer-power repulsion, 2.5 the general one."""
    st = _small(n=n, seed=n)
    st.rep = (st.rep[0], rep_n, st.rep[2])
    rng = np.random.default_rng(n)
    if n >= 40:
        st.x = _touching(st, rng)
    b = mag.Beads(st)
    m, F = b.forces()
    m, F = m.cpu().numpy().T, F.cpu().numpy().T
    mo, Fo = _oracle(orc, st).forces(st.x)
    assert np.abs(m - mo).max() <= 1e-12 * np.abs(mo).max()
    # sums of up to n terms in another order, and the closed-form gradient
    # against the oracle's quadrature
    assert np.abs(F - Fo).max() <= 1e-11 * np.abs(Fo).max()
    if n >= 40:
        # the contact and wall terms act: without repulsion the forces differ
        st0 = S.BeadStage(**{**st.__dict__, "rep": (0.0, st.rep[1], st.rep[2])})
        _, F0 = _oracle(orc, st0).forces(st.x)
        assert np.abs(F0 - Fo).max() > 1e-3 * np.abs(Fo).max()


def test_run_matches_oracle(orc, mag):
    import torch
    st = _small(n=300, seed=5)
    st.x = _touching(st, np.random.default_rng(5))
    b = mag.Beads(st)
    b.run(60)
    torch.cuda.synchronize()
    xg = b.positions()
    xo = _oracle(orc, st).run(st.x.copy(), 60)
    assert np.abs(xo - st.x).max() > 0.05  # the beads moved
    assert np.abs(xg - xo).max() < 1e-10


def test_freeze_bitwise(orc, mag):
    import torch
    nx, ny, nz = 40, 24, 20
    rng = np.random.default_rng(9)
    st = S.bead_stage(nx, ny, nz, n=60, a=2.0, seed=9)
    x = st.x.copy()
    # across the periodic faces, at the non-periodic faces, outside the box
    # along z, and centred on nodes (nodes exactly a away count)
    x[0] = (0.2, 0.3, 5.0)
    x[1] = (nx - 0.4, ny - 0.1, 9.5)
    x[2] = (13.0, 7.0, 0.3)
    x[3] = (21.0, 11.0, nz - 0.7)
    x[4] = (5.0, 5.0, 10.0)
    x[5] = (-3.5, ny + 2.25, 12.0)
    x[6] = (30.0, 4.0, -1.5)
    st.x = x
    base = np.zeros(nx * ny * nz, np.uint8)
    base[rng.choice(base.size, 50, replace=False)] = 1  # nodes already solid stay solid
    b = mag.Beads(st)
    solid = torch.as_tensor(base).cuda()
    b.freeze(solid)
    torch.cuda.synchronize()
    ref = _oracle(orc, st).freeze(st.x, base.copy())
    assert np.array_equal(solid.cpu().numpy(), ref)
    assert ref.sum() > base.sum() + 60 * 20


def test_pair_settles_at_balance(mag):
    import torch
    from scipy.optimize import brentq
    st = S.BeadStage(x=np.array([[10.0, 10.0, 10.0], [12.5, 10.5, 11.5]]), sheets=np.zeros((0, 6)),
                     bias=(0.0, 0.0, 1.5), a=1.0, chi=4.0, eta=1.0, dt=0.1, rep=(0.1, 2.0, 1.0), dims=(32, 32, 32),
                     periodic=(0, 0, 0), walls_z=False)
    b = mag.Beads(st)
    b.run(20000)
    torch.cuda.synchronize()
    x = b.positions()
    r = x[1] - x[0]
    m = 4 * np.pi * st.chi / (st.chi + 3) * 1.5
    g = brentq(lambda g: 2 * 0.1 * g ** -3 - 6 * m * m / (4 * np.pi * (2 + g) ** 4), 0.011, 1.0)
    assert np.linalg.norm(r) == pytest.approx(2 + g, rel=1e-9)
    assert np.abs(r[:2]).max() < 1e-9


def test_chains_form_and_freeze(mag):
    """A longer run of the small suspension: neighbours line up along the
    field (the mean squared cosine between a bead's nearest-neighbour
    direction and the field is 1/3 for isotropic directions, 1 for perfect
    chains; the run is chaotic, so only a clear majority alignment is
    asked), no two beads overlap, all stay between the walls; the fixed
    chains become solid nodes."""
    import torch
    st = _small(n=300, seed=2)
    b = mag.Beads(st)

    def order(x):
        L = np.array(st.dims, float)
        d = x[:, None, :] - x[None, :, :]
        d[..., :2] -= L[:2] * np.floor(d[..., :2] / L[:2] + 0.5)
        r = np.linalg.norm(d, axis=2) + np.eye(len(x)) * 1e9
        nn = d[np.arange(len(x)), r.argmin(1)]
        return np.mean((nn[:, 2] / np.linalg.norm(nn, axis=1)) ** 2), r.min()

    c0, _ = order(st.x)
    b.run(20000)
    torch.cuda.synchronize()
    x = b.positions()
    c1, rmin = order(x)
    assert np.isfinite(x).all()
    assert c0 < 0.5 and c1 > 0.8
    assert rmin > 2 * st.a
    assert x[:, 2].min() > 0.5 + st.a and x[:, 2].max() < st.dims[2] - 1.5 - st.a
    solid = torch.zeros(int(np.prod(st.dims)), dtype=torch.uint8, device="cuda")
    b.freeze(solid)
    frac = solid.float().mean().item()
    assert 0.5 * 300 * 4 / 3 * np.pi * st.a ** 3 / np.prod(st.dims) < frac < 2 * 300 * 4 / 3 * np.pi * st.a ** 3 / np.prod(st.dims)


def test_full_size_sampled_forces(orc, mag):
    st = S.bead_stage()
    b = mag.Beads(st)
    _, F = b.forces()
    F = F.cpu().numpy().T
    idx = np.random.default_rng(0).choice(st.n, 32, replace=False)
    Fo = _oracle(orc, st).forces_sample(st.x, idx)
    assert np.abs(F[idx] - Fo).max() <= 1e-11 * np.abs(Fo).max()


def test_forces_two_wave_blocks(orc, mag):
    """9000 beads: the pair kernel uses blocks of 128 (two waves); forces on
    sampled beads, including beads of the ragged last block."""
    st = S.bead_stage(192, 128, 64, n=9000, seed=8, sheets=False, bias=1.2)
    b = mag.Beads(st)
    _, F = b.forces()
    F = F.cpu().numpy().T
    idx = np.concatenate([np.random.default_rng(1).choice(st.n, 24, replace=False), np.arange(8990, 9000)])
    Fo = _oracle(orc, st).forces_sample(st.x, idx)
    assert np.abs(F[idx] - Fo).max() <= 1e-11 * np.abs(Fo).max()
