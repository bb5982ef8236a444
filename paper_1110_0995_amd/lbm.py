"""Python front end of the library: device buffers from torch, every step in
the HIP kernels behind the C ABI (include/lbmibm.h)."""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from .scenario import Cells, Scenario


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Lattice:
    """A D3Q19 lattice on one GPU (state buffers, mask, optional field G).

    prec: "f64", "f32" or "f32dev" (float deviations from the rest weights)."""

    def __init__(self, nx: int, ny: int, nz: int, tau: float, g: Sequence[float] = (0.0, 0.0, 0.0),
                 solid: Optional[np.ndarray] = None, prec: str = "f32dev",
                 periodic: Sequence[int] = (1, 1, 1), gfield: Optional[np.ndarray] = None,
                 device: str = "cuda", plane_stride: int = 0,
                 channels: Optional[Sequence[Tuple[int, int, int]]] = None):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the lattice kernels run only on an MI355X")
        self.device = torch.device(device)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        # channel k holds nodes [noff[k], noff[k+1]) of the concatenated index
        self.channels = [(self.nx, self.ny, self.nz)] if channels is None else [tuple(map(int, d)) for d in channels]
        self.noff = np.concatenate([[0], np.cumsum([a * b * c for a, b, c in self.channels])]).astype(np.int64)
        self.N = int(self.noff[-1])
        self.prec = prec
        self.code = _lib.PRECISIONS[prec]
        self.rdtype = torch.float64 if prec == "f64" else torch.float32
        self.stride = int(plane_stride) if plane_stride else int(self.lib.lbm_plane_stride(self.N, self.code))
        self.f_a = torch.empty(19 * self.stride, dtype=self.rdtype, device=self.device)
        self.f_b = torch.empty_like(self.f_a)
        if solid is None:
            solid = np.zeros(self.N, np.uint8)
        self.solid = torch.as_tensor(np.ascontiguousarray(np.asarray(solid, np.uint8).reshape(-1))).to(self.device)
        assert self.solid.numel() == self.N
        self.gfield = None
        if gfield is not None:
            self.gfield = torch.as_tensor(np.asarray(gfield, np.float64).reshape(3, self.N)).to(
                self.device, self.rdtype).contiguous()
        self.stream = torch.cuda.current_stream(self.device)
        self.params = _lib.LbmParams(self.nx, self.ny, self.nz, (C.c_int32 * 3)(*periodic), float(tau),
                                     (C.c_double * 3)(*g), self.code, self.stride, self.solid.data_ptr(),
                                     self.f_a.data_ptr(), self.f_b.data_ptr(),
                                     None if self.gfield is None else self.gfield.data_ptr(),
                                     self.stream.cuda_stream)
        self.tau, self.g = float(tau), tuple(float(v) for v in g)
        ctx = C.c_void_p()
        if channels is None:
            _lib.check(self.lib.lbm_init(C.byref(self.params), C.byref(ctx)))
        else:
            dims = (C.c_int32 * (3 * len(self.channels)))(*[v for d in self.channels for v in d])
            _lib.check(self.lib.lbm_init_channels(C.byref(self.params), len(self.channels), dims, C.byref(ctx)))
        self.ctx = ctx
        self.meshes = []

    @classmethod
    def from_scenario(cls, s: Scenario, prec: str = "f32dev", **kw) -> "Lattice":
        return cls(s.nx, s.ny, s.nz, s.tau, s.g, s.solid, prec, s.periodic,
                   kw.pop("gfield", s.gfield), **kw)

    @classmethod
    def batch(cls, scenarios: Sequence[Scenario], prec: str = "f32dev", **kw) -> "Lattice":
        """One context over independent channels (one per scenario), stepped
        together.  tau, g and the periodic axes must agree across them."""
        s0 = scenarios[0]
        for s in scenarios:
            if s.tau != s0.tau or tuple(s.g) != tuple(s0.g) or tuple(s.periodic) != tuple(s0.periodic):
                raise ValueError("batched channels must share tau, g and the periodic axes")
            if s.gfield is not None:
                raise ValueError("a forcing field is not supported in a batch")
        solid = np.concatenate([np.asarray(s.solid, np.uint8).reshape(-1) for s in scenarios])
        return cls(s0.nx, s0.ny, s0.nz, s0.tau, s0.g, solid, prec, s0.periodic, None,
                   channels=[(s.nx, s.ny, s.nz) for s in scenarios], **kw)

    def channel(self, k: int) -> slice:
        """Node range of channel k in the concatenated index."""
        return slice(int(self.noff[k]), int(self.noff[k + 1]))

    def set_launch(self, collide_waves_per_block: int = 0, list_blocks: int = 0) -> None:
        _lib.check(self.lib.lbm_set_launch(self.ctx, int(collide_waves_per_block), int(list_blocks)))

    def set_ibm_overlap(self, mode: int = -1) -> None:
        """1: membrane forces beside the velocity pass, 0: in order, -1: by mesh size."""
        _lib.check(self.lib.lbm_set_ibm_overlap(self.ctx, int(mode)))

    def set_node_records(self, mode: int = 1) -> None:
        """1: stencil-node velocities from the populations the last collide-stream
        pass recorded for them; 0: gathered from the lattice every step."""
        _lib.check(self.lib.lbm_set_node_records(self.ctx, int(mode)))

    def node_records_used(self):
        """(used, missed) of the last coupling: velocities read from the
        records, and whether a stencil node was missing from them."""
        u, m = C.c_int32(), C.c_int32()
        _lib.check(self.lib.lbm_node_records_used(self.ctx, C.byref(u), C.byref(m)))
        return bool(u.value), bool(m.value)

    def check_finite(self) -> bool:
        """Wait for the stream; False if a collide-stream pass met non-finite
        populations (the state is then lost), True otherwise."""
        bad = C.c_int32()
        rc = self.lib.lbm_check_finite(self.ctx, C.byref(bad))
        if rc not in (0, _lib.LBM_ENONFINITE):
            _lib.check(rc)
        return not bad.value

    # -- the four calls of the path --------------------------------------
    def step(self, nsteps: int = 1) -> None:
        _lib.check(self.lib.lbm_step(self.ctx, int(nsteps)))

    def step_timed(self, start_event: int, stop_event: int) -> None:
        """One step whose collide-stream kernel sets the two HIP events (raw
        hipEvent_t handles, e.g. torch.cuda.Event(enable_timing=True).cuda_event
        after one record) to its own start and end."""
        _lib.check(self.lib.lbm_step_timed(self.ctx, C.c_void_p(int(start_event)), C.c_void_p(int(stop_event))))

    def couple(self, mesh: "Mesh") -> None:
        _lib.check(self.lib.ibm_couple(self.ctx, C.byref(mesh.s)))

    def run(self, nsteps: int, mesh: Optional["Mesh"] = None, steps_per_graph: int = 0) -> None:
        """nsteps full steps (immersed-boundary coupling then collide-stream),
        replayed from a captured HIP graph in groups of steps_per_graph (even)
        when that is non-zero."""
        _lib.check(self.lib.lbm_run(self.ctx, None if mesh is None else C.byref(mesh.s), int(nsteps),
                                    int(steps_per_graph)))

    def fields(self):
        """(rho [N], u [3, N]) of the current state as device tensors."""
        rho = torch.empty(self.N, dtype=self.rdtype, device=self.device)
        u = torch.empty(3, self.N, dtype=self.rdtype, device=self.device)
        _lib.check(self.lib.lbm_read_fields(self.ctx, _ptr(rho), _ptr(u), None))
        return rho, u

    def sums(self) -> np.ndarray:
        """FP64 (sum rho, sum j) over fluid nodes; waits for the stream."""
        out = (C.c_double * 4)()
        _lib.check(self.lib.lbm_read_fields(self.ctx, None, None, out))
        return np.array(out[:])

    # -- state access -----------------------------------------------------
    def current(self) -> torch.Tensor:
        p = C.c_void_p()
        st = C.c_int64()
        _lib.check(self.lib.lbm_current(self.ctx, C.byref(p), C.byref(st)))
        buf = self.f_a if p.value == self.f_a.data_ptr() else self.f_b
        return buf.view(19, self.stride)[:, :self.N]

    def current_buffer(self) -> torch.Tensor:
        """The whole state buffer ([19 * plane_stride], storage type) that
        holds the current populations."""
        p = C.c_void_p()
        _lib.check(self.lib.lbm_current(self.ctx, C.byref(p), None))
        return self.f_a if p.value == self.f_a.data_ptr() else self.f_b

    def adjoint_step(self, mesh: Optional["Mesh"], f_n: torch.Tensor, x_n: Optional[torch.Tensor],
                     v_n: Optional[torch.Tensor], lam_next: torch.Tensor, lam: torch.Tensor,
                     lam_x: Optional[torch.Tensor], lam_v: Optional[torch.Tensor],
                     dgrad: Optional[torch.Tensor] = None) -> None:
        """One reverse step (lbm_adjoint_step): lam <- dJ/df_n from
        lam_next = dJ/df_{n+1}; lam_x, lam_v updated in place; dJ/dG of the
        step added to dgrad."""
        for t, dt in ((f_n, self.rdtype), (lam_next, self.rdtype), (lam, self.rdtype)):
            assert t.dtype == dt and t.is_contiguous() and t.numel() >= 19 * self.stride
        _lib.check(self.lib.lbm_adjoint_step(
            self.ctx, None if mesh is None else C.byref(mesh.s), _ptr(f_n), _ptr(x_n), _ptr(v_n), _ptr(lam_next),
            _ptr(lam), _ptr(lam_x), _ptr(lam_v), _ptr(dgrad)))

    def record_buffers(self, nsteps: int, mesh: Optional["Mesh"] = None):
        """Device buffers for lbm_run_record: (f_rec, x_rec, v_rec)."""
        f = torch.empty(nsteps, 19 * self.stride, dtype=self.rdtype, device=self.device)
        if mesh is None:
            return f, None, None
        nv = mesh.cells.nverts
        return (f, torch.empty(nsteps, 3, nv, dtype=torch.float64, device=self.device),
                torch.empty(nsteps, 3, nv, dtype=self.rdtype, device=self.device))

    def run_record(self, nsteps: int, mesh: Optional["Mesh"], rec, use_graph: bool = True) -> None:
        """nsteps coupled steps, recording the state at the start of each (lbm_run_record)."""
        f, x, v = rec
        assert f.shape[0] >= nsteps
        _lib.check(self.lib.lbm_run_record(self.ctx, None if mesh is None else C.byref(mesh.s), int(nsteps),
                                           _ptr(f), _ptr(x), _ptr(v), int(bool(use_graph))))

    def adjoint_run(self, nsteps: int, mesh: Optional["Mesh"], rec, lam_a: torch.Tensor, lam_b: torch.Tensor,
                    lam_x: Optional[torch.Tensor], lam_v: Optional[torch.Tensor],
                    dgrad: Optional[torch.Tensor] = None, use_graph: bool = True) -> None:
        """Reverse sweep over recorded steps (lbm_adjoint_run): lam_a goes
        from dJ/df at the end to dJ/df at the start."""
        f, x, v = rec
        _lib.check(self.lib.lbm_adjoint_run(self.ctx, None if mesh is None else C.byref(mesh.s), int(nsteps),
                                            _ptr(f), _ptr(x), _ptr(v), _ptr(lam_a), _ptr(lam_b), _ptr(lam_x),
                                            _ptr(lam_v), _ptr(dgrad), int(bool(use_graph))))

    def steps_taken(self) -> int:
        st = C.c_int64()
        _lib.check(self.lib.lbm_current(self.ctx, None, C.byref(st)))
        return st.value

    def populations_f64(self) -> torch.Tensor:
        out = torch.empty(19, self.N, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.lbm_store_f64(self.ctx, _ptr(out)))
        return out

    def load_f64(self, f) -> None:
        t = torch.as_tensor(np.ascontiguousarray(f, np.float64).reshape(19, self.N)).to(self.device)
        _lib.check(self.lib.lbm_load_f64(self.ctx, _ptr(t)))
        torch.cuda.synchronize(self.device)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.lib.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mesh:
    """Membrane population on a lattice's device (SoA arrays, rest shape computed on the GPU)."""

    def __init__(self, lat: Lattice, cells: Cells, cell_chan: Optional[np.ndarray] = None,
                 contact: Optional[dict] = None):
        """contact: None, or dict(a, n, rcut, roff, dmin, cell_cell, planes [np, 4], cyl [nc, 3],
        cyl_off [nch + 1] (optional), spheres [ns, 4] (optional)) of the soft-sphere contact forces
        (ibm_contact)."""
        dev, R = lat.device, lat.rdtype
        i32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32)).to(dev)
        self.cells = cells
        self.lat = lat
        self.cell_chan = None if cell_chan is None else i32(np.asarray(cell_chan).reshape(-1))
        self.contact = None
        if contact is not None:
            f64 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).to(dev)
            self._planes = f64(np.asarray(contact.get("planes", np.zeros((0, 4)))).reshape(-1, 4))
            self._cyl = f64(np.asarray(contact.get("cyl", np.zeros((0, 3)))).reshape(-1, 3))
            self._cyl_off = None if contact.get("cyl_off") is None else i32(contact["cyl_off"])
            self._sph = f64(np.asarray(contact.get("spheres", np.zeros((0, 4)))).reshape(-1, 4))
            self.contact = _lib.IbmContact(
                float(contact["a"]), float(contact["n"]), float(contact["rcut"]), float(contact.get("roff", 0.0)),
                float(contact.get("dmin", 0.05)), int(contact.get("cell_cell", 1)), self._planes.shape[0],
                self._planes.data_ptr() if self._planes.numel() else None, self._cyl.shape[0],
                self._cyl.data_ptr() if self._cyl.numel() else None,
                None if self._cyl_off is None else self._cyl_off.data_ptr(), self._sph.shape[0],
                self._sph.data_ptr() if self._sph.numel() else None)
        self.vert_off = i32(cells.vert_off)
        self.tri_off = i32(cells.tri_off)
        self.edge_off = i32(cells.edge_off)
        self.tri = i32(np.asarray(cells.tri).T)
        self.hinge = i32(np.asarray(cells.hinge).T)
        self.anchor = i32(np.asarray(cells.anchor).T)
        self.x = torch.as_tensor(np.ascontiguousarray(np.asarray(cells.offset, np.float64).T)).to(dev).contiguous()
        self.v = torch.zeros(3, cells.nverts, dtype=R, device=dev)
        self.f_el = torch.zeros_like(self.v)
        self.moduli = torch.as_tensor(np.ascontiguousarray(np.asarray(cells.moduli, np.float64).T)).to(dev, R).contiguous()
        f64 = dict(dtype=torch.float64, device=dev)
        self.l0 = torch.zeros(cells.nedges, **f64)
        self.th0 = torch.zeros(cells.nedges, **f64)
        self.a0 = torch.zeros(cells.ntris, **f64)
        self.a0c = torch.zeros(cells.ncells, **f64)
        self.v0c = torch.zeros(cells.ncells, **f64)
        self.avert = torch.zeros(cells.nverts, **f64)
        i32z = lambda n: torch.zeros(n, dtype=torch.int32, device=dev)
        self.vtri_off, self.vtri = i32z(cells.nverts + 1), i32z(3 * cells.ntris)
        self.vedge_off, self.vedge = i32z(cells.nverts + 1), i32z(4 * cells.nedges)
        p = lambda t: t.data_ptr()
        self.s = _lib.IbmMesh(cells.ncells, cells.nverts, cells.ntris, cells.nedges, p(self.vert_off),
                              p(self.tri_off), p(self.edge_off), p(self.tri), p(self.hinge), p(self.anchor),
                              None if self.cell_chan is None else p(self.cell_chan), p(self.x), p(self.v), p(self.f_el), p(self.moduli), p(self.l0), p(self.a0),
                              p(self.th0), p(self.a0c), p(self.v0c), p(self.avert), p(self.vtri_off), p(self.vtri),
                              p(self.vedge_off), p(self.vedge), float(cells.xi), float(cells.mass),
                              float(cells.dt), None if self.contact is None else C.pointer(self.contact),
                              int(getattr(cells, "stretch_law", 0)), 0, 0, 0, 0)
        _lib.check(lat.lib.ibm_rest_shape(lat.ctx, C.byref(self.s)))
        lat.meshes.append(self)

    def force_jvp(self, x: torch.Tensor, w: torch.Tensor):
        """(F_el(x), (dF_el/dx) w) in FP64 for offsets x and direction w,
        both [3, nverts] float64 device tensors."""
        f = torch.empty_like(x)
        jvp = torch.empty_like(x)
        _lib.check(self.lat.lib.ibm_force_jvp(self.lat.ctx, C.byref(self.s), _ptr(x.contiguous()),
                                              _ptr(w.contiguous()), _ptr(f), _ptr(jvp)))
        return f, jvp

    def positions(self) -> np.ndarray:
        """Absolute positions (float64 [nverts, 3]) = anchor + offset."""
        x = self.x.double().cpu().numpy().T
        return self.cells.anchor[self.cells.vertex_cell()].astype(np.float64) + x

    def point_mass(self) -> np.ndarray:
        """Mass of each IB point: the areal mass density times its rest area."""
        return self.cells.mass * self.avert.cpu().numpy()

    def velocities(self) -> np.ndarray:
        return self.v.double().cpu().numpy().T.copy()

    def set_offsets(self, offsets: np.ndarray) -> None:
        """Overwrite the positions (offsets from the anchors, [nverts, 3])."""
        self.x.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(offsets, np.float64).T)).to(self.x.device, self.x.dtype))
