"""Differentiation of a coupled run with respect to the forcing field G.

``CoupledRun`` is a torch.autograd.Function: its forward takes nsteps
coupled steps (ibm_couple + lbm_step, Sec. 2.1-2.4) from the lattice's and
mesh's current state with the forcing field G, and returns the final
populations, IB-point offsets and velocities.  Its backward runs the
hand-written reverse kernels (lbm_adjoint_step) from the last step to the
first.  Memory is bounded by checkpointing: the forward keeps the state
every ``every`` steps; the backward recomputes one segment at a time from its
checkpoint, recording that segment's states (lbm_run_record), and walks it in
reverse (lbm_adjoint_run); both are captured HIP graphs replayed for every
segment of the same length.

``objective`` is the scalar studied on the adjoint workload: the x-momentum
flux through the outlet plane x = nx - 1 at the final step plus the squared
displacement of every cell's centroid.
"""
from __future__ import annotations

from typing import Optional

import torch


def _snapshot(lat, mesh):
    f = lat.current_buffer().clone()
    if mesh is None:
        return f, None, None
    return f, mesh.x.clone(), mesh.v.clone()


def _restore(lat, mesh, snap):
    f, x, v = snap
    lat.current_buffer().copy_(f)
    if mesh is not None:
        mesh.x.copy_(x)
        mesh.v.copy_(v)


class CoupledRun(torch.autograd.Function):
    """(f_T [19, N], x_T [3, nv], v_T [3, nv]) = run(G; initial state), with
    f_T the full FP64 populations of every node (per-node layout, as the
    adjoint of the populations is kept)."""

    @staticmethod
    def forward(ctx, G, lat, mesh, nsteps: int, every: int = 20):
        if lat.gfield is None:
            raise ValueError("the lattice was made without a forcing field; pass gfield= to Lattice")
        if every < 1 or nsteps < 0:
            raise ValueError("every must be >= 1 and nsteps >= 0")
        lat.gfield.copy_(G.detach().reshape(3, lat.N).to(lat.gfield.dtype))
        ckpts = []
        for t0 in range(0, nsteps, every):
            ckpts.append(_snapshot(lat, mesh))
            n = min(every, nsteps - t0)
            lat.run(n, mesh, steps_per_graph=n - n % 2)
        ctx.lat, ctx.mesh, ctx.nsteps, ctx.every = lat, mesh, nsteps, every
        ctx.ckpts = ckpts
        ctx.final = _snapshot(lat, mesh)
        ctx.G_shape, ctx.G_dtype = G.shape, G.dtype
        fT = lat.populations_f64()  # per-node populations (the storage keeps bounced ones in solid slots)
        if mesh is None:
            z = torch.zeros(3, 0, dtype=torch.float64, device=lat.device)
            return fT, z, z.clone()
        return fT, mesh.x.clone(), mesh.v.clone().double()

    @staticmethod
    def backward(ctx, gf, gx, gv):
        lat, mesh = ctx.lat, ctx.mesh
        N, st = lat.N, lat.stride
        # work buffers live on the lattice, so that the captured graphs of
        # the recording run and the reverse sweep (keyed by their buffer
        # addresses) are reused by later backward passes
        B = _buffers(lat, mesh, min(ctx.every, ctx.nsteps))
        lam, lam2, lx, lv, dG, rec = B["lam"], B["lam2"], B["lx"], B["lv"], B["dG"], B["rec"]
        lam.zero_()
        if gf is not None:
            lam.view(19, st)[:, :N].copy_(gf)
        dG.zero_()
        if mesh is not None:
            lx.copy_(gx) if gx is not None else lx.zero_()
            lv.copy_(gv) if gv is not None else lv.zero_()
        for seg in range(len(ctx.ckpts) - 1, -1, -1):
            _restore(lat, mesh, ctx.ckpts[seg])
            n = min(ctx.every, ctx.nsteps - seg * ctx.every)
            lat.run_record(n, mesh, rec)
            lat.adjoint_run(n, mesh, rec, lam, lam2, lx, lv, dG)
        _restore(lat, mesh, ctx.final)
        return dG.clone().reshape(ctx.G_shape).to(ctx.G_dtype), None, None, None, None


def _buffers(lat, mesh, every: int) -> dict:
    key = (every, id(mesh))
    cache = lat.__dict__.setdefault("_adjoint_buffers", {})
    if key not in cache:
        R, dev = lat.rdtype, lat.device
        B = {"lam": torch.zeros(19 * lat.stride, dtype=R, device=dev), "dG": torch.zeros(3, lat.N, dtype=R, device=dev),
             "rec": lat.record_buffers(every, mesh), "lx": None, "lv": None}
        B["lam2"] = torch.zeros_like(B["lam"])
        if mesh is not None:
            B["lx"] = torch.zeros(3, mesh.cells.nverts, dtype=torch.float64, device=dev)
            B["lv"] = torch.zeros_like(B["lx"])
        cache.clear()  # one set at a time
        cache[key] = B
    return cache[key]


def run_with_grad(G: torch.Tensor, lat, mesh, nsteps: int, every: int = 20):
    return CoupledRun.apply(G, lat, mesh, nsteps, every)


def objective(lat, mesh, fT: torch.Tensor, xT: torch.Tensor, G: torch.Tensor,
              x0_offsets: Optional[torch.Tensor]) -> torch.Tensor:
    """x-momentum flux (j_x + F_x/2 with F = g + G) summed over the fluid
    nodes of the plane x = nx - 1 at the final step, plus, for each cell,
    the squared displacement of its vertex centroid from x0_offsets'."""
    nx, ny, nz = lat.nx, lat.ny, lat.nz
    cxs = torch.tensor([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0],
                       dtype=fT.dtype, device=fT.device)
    idx = torch.arange(ny * nz, device=fT.device) * nx + (nx - 1)
    fluid = (lat.solid[idx] == 0)
    idx = idx[fluid]
    jx = (cxs[:, None] * fT[:, idx]).sum(0).double()
    Fx = lat.g[0] + G.reshape(3, lat.N)[0, idx].double()
    J = (jx + 0.5 * Fx).sum()
    if mesh is not None and x0_offsets is not None:
        off = mesh.cells.vert_off
        for c in range(len(off) - 1):
            a, b = int(off[c]), int(off[c + 1])
            d = xT[:, a:b].mean(1) - x0_offsets[:, a:b].mean(1)
            J = J + (d * d).sum()
    return J

