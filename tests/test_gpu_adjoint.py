"""GPU tests of the differentiation form: the reverse (adjoint) step and the
checkpointed autograd run, against the FP64 oracle.

  - ibm_force_jvp: F_el equals the oracle's membrane forces and the
    directional derivative equals a central difference of the oracle's
    forces;
  - lbm_adjoint_step, dot-product test: for random output adjoints lambda
    and input perturbations delta of each kind (populations, IB positions,
    IB velocities, forcing field G), <adjoint(lambda), delta> equals the
    central difference of <lambda, oracle_step(state + eps delta)>; with and
    without cells, in FP64 and in FP32 deviation storage;
  - CoupledRun (300 steps, checkpoints every 20) on the adjoint workload:
    the gradient of the objective along 16 seeded directions of G against
    FP64 oracle finite differences stored in tests/golden/adjoint_fd.json
    (written by tests/golden/make_adjoint_fd.py from the oracle only)."""
import json
import os

import numpy as np
import pytest

from paper_1110_0995_amd import scenario as S

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lbm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1110_0995_amd import lbm as mod
    return mod


def _small(ncells=2, posts=True, seed=11):
    return S.posts_and_cells(40, 32, 24, posts_x=1 if posts else 0, posts_y=1 if posts else 0, post_radius=4,
                             gap=6, ncells=ncells, cell_radius=3.0, level=2, tau=0.8, gx=1e-4, seed=seed,
                             moduli=(0.02, 0.005, 0.01, 0.1, 0.5))


def _to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype)


def test_force_jvp_matches_oracle(orc, lbm):
    import torch
    s = _small(ncells=3, posts=False)
    for prec in ("f64", "f32dev"):
        lat = lbm.Lattice.from_scenario(s, prec=prec)
        mesh = lbm.Mesh(lat, s.cells)
        M = orc.Mesh(s.cells)
        X0 = s.cells.positions()
        M.rest_shape(X0)
        rng = np.random.default_rng(3)
        X = X0 + 0.15 * rng.standard_normal(X0.shape)
        W = rng.standard_normal(X0.shape)
        off = X - s.cells.anchor[s.cells.vertex_cell()]
        f, jvp = mesh.force_jvp(_to_dev(off.T, torch.float64), _to_dev(W.T, torch.float64))
        f = f.cpu().numpy().T
        jvp = jvp.cpu().numpy().T
        Fo = M.forces(X)
        # FP64 throughout; in the FP32 context only the moduli are stored as floats (6e-8 relative)
        assert np.abs(f - Fo).max() <= (1e-12 if prec == "f64" else 1e-7) * np.abs(Fo).max()
        h = 1e-6
        fd = (M.forces(X + h * W) - M.forces(X - h * W)) / (2 * h)
        # central difference: truncation ~h^2, rounding ~1e-16 |F| / h
        assert np.abs(jvp - fd).max() <= 1e-6 * np.abs(fd).max()
        lat.close()


def _oracle_state(orc, s, G, nsteps=6, seed=0):
    """Oracle state after a few coupled steps from a deformed, moving start."""
    L = orc.Lattice.from_scenario(s, G=G)
    f = L.rest()
    if s.cells is None:
        for _ in range(nsteps):
            f = orc.step(L, None, f)
        return L, None, f, None, None
    M = orc.Mesh(s.cells)
    X = s.cells.positions()
    M.rest_shape(X)
    rng = np.random.default_rng(seed)
    X = X + 0.05 * rng.standard_normal(X.shape)
    V = 1e-3 * rng.standard_normal(X.shape)
    for _ in range(nsteps):
        f = orc.step(L, M, f, X, V)
    return L, M, f, X, V


W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _pack(lat, a, dtype):
    """[19, N] host array -> flat [19 * plane_stride] device buffer (per-node
    layout: the adjoints of the populations)."""
    import torch
    buf = torch.zeros(19, lat.stride, dtype=dtype, device="cuda")
    buf[:, :lat.N] = _to_dev(a, dtype)
    return buf.reshape(-1)


def _dot_test(orc, lbm, s, prec, tol, with_cells=True):
    import torch
    rng = np.random.default_rng(42)
    G = 1e-5 * rng.standard_normal((3, s.n))
    fluid = s.solid.reshape(-1) == 0
    L, M, f, X, V = _oracle_state(orc, s, G)
    lat = lbm.Lattice.from_scenario(s, prec=prec, gfield=G)
    R = lat.rdtype
    mesh = lbm.Mesh(lat, s.cells) if with_cells else None
    # output adjoints
    lf = rng.standard_normal((19, s.n)) * fluid
    lX = rng.standard_normal(X.shape) if with_cells else None
    lV = rng.standard_normal(X.shape) if with_cells else None
    # GPU reverse step; the state in the library's storage form (a population
    # bounced back from a solid node lies in that node's slot), via load_f64
    lat.load_f64(f)
    f_n = lat.current_buffer().clone()
    lam_next = _pack(lat, lf, R)
    lam = torch.zeros_like(lam_next)
    dG = torch.zeros(3, s.n, dtype=R, device="cuda")
    if with_cells:
        anchor = s.cells.anchor[s.cells.vertex_cell()]
        x_n = _to_dev((X - anchor).T, torch.float64)
        v_n = _to_dev(V.T, R)
        lx = _to_dev(lX.T, torch.float64)
        lv = _to_dev(lV.T, torch.float64)
    else:
        x_n = v_n = lx = lv = None
    lat.adjoint_step(mesh, f_n, x_n, v_n, lam_next, lam, lx, lv, dG)
    torch.cuda.synchronize()
    lam_f = lam.view(19, lat.stride)[:, :s.n].double().cpu().numpy()
    dG = dG.double().cpu().numpy()
    if with_cells:
        lam_x = lx.cpu().numpy().T
        lam_v = lv.cpu().numpy().T

    def J(df=0.0, dX=0.0, dV=0.0, dGf=0.0):
        Lp = orc.Lattice.from_scenario(s, G=G + dGf)
        if with_cells:
            X2, V2 = X + dX, V + dV
            f2 = orc.step(Lp, M, f + df, X2, V2)
            return float((lf * f2).sum() + (lX * X2).sum() + (lV * V2).sum())
        f2 = orc.step(Lp, None, f + df)
        return float((lf * f2).sum())

    cases = {"f": dict(df=1e-4 * rng.standard_normal(f.shape) * fluid),
             "G": dict(dGf=1e-4 * rng.standard_normal(G.shape) * fluid)}
    if with_cells:
        cases["X"] = dict(dX=1e-2 * rng.standard_normal(X.shape))
        cases["V"] = dict(dV=1e-3 * rng.standard_normal(X.shape))
    for name, d in cases.items():
        eps = 1e-3
        plus = {k: eps * v for k, v in d.items()}
        minus = {k: -eps * v for k, v in d.items()}
        fd = (J(**plus) - J(**minus)) / (2 * eps)
        if name == "f":
            ad = float((lam_f * d["df"]).sum())
        elif name == "G":
            ad = float((dG * d["dGf"]).sum())
        elif name == "X":
            ad = float((lam_x * d["dX"]).sum())
        else:
            ad = float((lam_v * d["dV"]).sum())
        assert abs(ad - fd) <= tol * abs(fd), f"{prec} {name}: adjoint {ad!r} vs finite difference {fd!r}"
    lat.close()


def test_adjoint_step_dot_product_f64(orc, lbm):
    # the step is smooth in every input here (no IB point crosses a lattice
    # plane within eps), so the central difference is exact to ~eps^2; the
    # bound leaves room for FP64 rounding of the differenced sums, while a
    # missing or transposed term would be off by O(1)
    _dot_test(orc, lbm, _small(), "f64", 1e-6)


def test_adjoint_step_dot_product_f32dev(orc, lbm):
    _dot_test(orc, lbm, _small(), "f32dev", 1e-3)


def test_adjoint_step_fluid_only(orc, lbm):
    s = _small(ncells=0)
    s.cells = None
    _dot_test(orc, lbm, s, "f64", 1e-6, with_cells=False)


def _run_grad(lbm, s, prec, dirs):
    import torch
    from paper_1110_0995_amd import adjoint
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    mesh = lbm.Mesh(lat, s.cells)
    x0 = mesh.x.clone()
    G = torch.zeros(3, s.n, dtype=lat.rdtype, device="cuda", requires_grad=True)
    fT, xT, vT = adjoint.run_with_grad(G, lat, mesh, s.steps, s.meta["checkpoint_every"])
    J = adjoint.objective(lat, mesh, fT, xT, G, x0)
    J.backward()
    g = G.grad.double().cpu().numpy().reshape(3, s.nz, s.ny, s.nx)
    x0_, x1_ = s.meta["design_x"]
    ad = [float((g[..., x0_:x1_] * d).sum()) for d in dirs]
    return float(J.item()), ad, lat, mesh


def test_coupled_run_gradient_matches_oracle_fd_f32dev(lbm):
    """FP32 deviation storage: every directional derivative within 1e-3
    relative of the FP64 oracle's central difference."""
    gold = json.load(open(os.path.join(HERE, "golden", "adjoint_fd.json")))
    s = S.adjoint_channel()
    dirs = S.random_directions(s, len(gold["fd"]))
    J, ad, lat, _ = _run_grad(lbm, s, "f32dev", dirs)
    fd = np.array(gold["fd"])
    assert abs(J - gold["J0"]) <= 1e-5 * abs(gold["J0"])
    err = np.abs(np.array(ad) - fd) / np.abs(fd)
    assert err.max() <= 1e-3, f"relative errors {err}"
    lat.close()


def test_coupled_run_gradient_matches_oracle_fd_f64(lbm):
    """FP64: the adjoint gradient is exact to rounding, so the comparison is
    limited by the stored central differences themselves; their truncation
    error, estimated from the two directions repeated at 2 eps (Richardson:
    (FD(2eps) - FD(eps)) / 3), is about 6e-8, so the bound is 1e-6 of the
    largest directional derivative."""
    gold = json.load(open(os.path.join(HERE, "golden", "adjoint_fd.json")))
    s = S.adjoint_channel()
    dirs = S.random_directions(s, len(gold["fd"]))
    J, ad, lat, _ = _run_grad(lbm, s, "f64", dirs)
    fd = np.array(gold["fd"])
    trunc = max(abs(b - a) / 3 for a, b in zip(gold["fd"], gold["fd_2eps"]))
    assert trunc < 1e-7 * np.abs(fd).max()
    assert abs(J - gold["J0"]) <= 1e-9 * abs(gold["J0"])
    err = np.abs(np.array(ad) - fd)
    assert err.max() <= 1e-6 * np.abs(fd).max(), f"absolute errors {err}"
    lat.close()


def test_coupled_run_leaves_final_state(lbm):
    """After backward the lattice and mesh hold the forward's final state."""
    import torch
    from paper_1110_0995_amd import adjoint
    s = _small()
    s.gfield = np.zeros((3, s.nz, s.ny, s.nx))
    s.meta["design_x"] = [8, 32]
    lat = lbm.Lattice.from_scenario(s, prec="f32dev")
    mesh = lbm.Mesh(lat, s.cells)
    G = torch.zeros(3, s.n, dtype=torch.float32, device="cuda", requires_grad=True)
    fT, xT, vT = adjoint.run_with_grad(G, lat, mesh, 30, 8)  # segments 8, 8, 8, 6
    f_end = lat.current().clone()
    x_end = mesh.x.clone()
    J = adjoint.objective(lat, mesh, fT, xT, G, None)
    J.backward()
    torch.cuda.synchronize()
    assert torch.equal(lat.current(), f_end) and torch.equal(mesh.x, x_end)
    assert torch.equal(lat.populations_f64(), fT)  # the forward's output: the final per-node populations
    assert torch.isfinite(G.grad).all() and G.grad.abs().max() > 0
    lat.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_record_matches_plain_steps(lbm, use_graph):
    """Recording steps (graph or not, with the membrane kernels on the
    second stream) gives bitwise the plain run's states:
    record k equals the state after k steps on every fluid node (records
    after the first are written by the streaming pass, which never writes
    the slots of solid nodes, and nothing reads them), and the final state
    matches."""
    import torch
    s = _small(seed=12)
    A = lbm.Lattice.from_scenario(s, prec="f32dev")
    MA = lbm.Mesh(A, s.cells)
    B = lbm.Lattice.from_scenario(s, prec="f32dev")
    MB = lbm.Mesh(B, s.cells)
    B.set_ibm_overlap(1)  # the recorded steps run the membrane on the second stream
    n = 6
    rec = B.record_buffers(n, MB)
    for rep in range(2):  # the second call replays the captured graph
        states = []
        for k in range(n):
            torch.cuda.synchronize()
            states.append((A.current_buffer().clone(), MA.x.clone(), MA.v.clone()))
            A.run(1, MA)
        B.run_record(n, MB, rec, use_graph=use_graph)
        torch.cuda.synchronize()
        fluid = torch.as_tensor(s.solid.reshape(-1) == 0, device="cuda")
        for k in range(n):
            got = rec[0][k].view(19, B.stride)[:, :s.n][:, fluid]
            ref = states[k][0].view(19, A.stride)[:, :s.n][:, fluid]
            assert torch.equal(got, ref), f"rep {rep} record {k}"
            assert torch.equal(rec[1][k], states[k][1]) and torch.equal(rec[2][k], states[k][2])
        assert torch.equal(A.current()[:, fluid], B.current()[:, fluid])
        assert torch.equal(MA.x, MB.x) and torch.equal(MA.v, MB.v)
        assert A.steps_taken() == B.steps_taken()


@pytest.mark.parametrize("n", [5, 6])
def test_adjoint_run_matches_stepwise(lbm, n):
    """The native reverse sweep (graph-captured, replayed twice) equals
    lbm_adjoint_step called step by step; only the order of the float adds
    that spread lambda_u differs, so FP64 agrees to rounding."""
    import torch
    s = _small(seed=13)
    rng = np.random.default_rng(5)
    G = 1e-5 * rng.standard_normal((3, s.n))
    lat = lbm.Lattice.from_scenario(s, prec="f64", gfield=G)
    mesh = lbm.Mesh(lat, s.cells)
    lat.run(3, mesh)
    rec = lat.record_buffers(n, mesh)
    lat.run_record(n, mesh, rec)
    fluid = torch.as_tensor(s.solid.reshape(-1) == 0, device="cuda")
    lam0 = torch.zeros(19, lat.stride, dtype=torch.float64, device="cuda")
    lam0[:, :s.n] = torch.as_tensor(rng.standard_normal((19, s.n)), device="cuda") * fluid
    lx0 = torch.as_tensor(rng.standard_normal((3, s.cells.nverts)), device="cuda")
    lv0 = torch.as_tensor(rng.standard_normal((3, s.cells.nverts)), device="cuda")
    # step by step
    la, lb = lam0.reshape(-1).clone(), torch.zeros(19 * lat.stride, dtype=torch.float64, device="cuda")
    lx, lv = lx0.clone(), lv0.clone()
    dG1 = torch.zeros(3, s.n, dtype=torch.float64, device="cuda")
    for k in range(n - 1, -1, -1):
        lat.adjoint_step(mesh, rec[0][k], rec[1][k], rec[2][k], la, lb, lx, lv, dG1)
        la, lb = lb, la
    for rep in range(2):
        a = lam0.reshape(-1).clone()
        b = torch.zeros_like(a)
        lx2, lv2 = lx0.clone(), lv0.clone()
        dG2 = torch.zeros_like(dG1)
        lat.adjoint_run(n, mesh, rec, a, b, lx2, lv2, dG2, use_graph=True)
        torch.cuda.synchronize()
        for got, ref in ((a, la), (lx2, lx), (lv2, lv), (dG2, dG1)):
            assert torch.allclose(got, ref, rtol=1e-11, atol=1e-13 * ref.abs().max().item()), f"rep {rep}"
