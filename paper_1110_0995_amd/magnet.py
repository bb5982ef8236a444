"""The magnetic bead stage (Sec. 2.5) on the GPU: a thin wrapper over the
mag_* entry points of include/magnet.h (argument marshalling only; every step
runs in the library's kernels).

Bead arrays live on the device as [3][n] float64 tensors; the wrapper keeps
the positions and the work buffer the library asks for, and enqueues on the
current torch stream."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib
from .scenario import BeadStage


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


class Beads:
    """Beads of a BeadStage on cuda:0 (or `device`)."""

    def __init__(self, st: BeadStage, device: str = "cuda", x: Optional[np.ndarray] = None):
        self.L = _lib.load()
        self.device = torch.device(device)
        self.stage = st
        x = st.x if x is None else x
        p = _lib.MagParams()
        p.n = len(x)
        sheets = np.asarray(st.sheets, np.float64).reshape(-1, 6)
        if len(sheets) > _lib.MAG_MAX_SHEETS:
            raise ValueError(f"at most {_lib.MAG_MAX_SHEETS} sheets")
        p.nsheets = len(sheets)
        for s, row in enumerate(sheets):
            for i, v in enumerate(row):
                p.sheets[s][i] = float(v)
        for d in range(3):
            p.bias[d] = float(st.bias[d])
            p.periodic[d] = int(st.periodic[d])
        p.a, p.chi, p.eta, p.dt = float(st.a), float(st.chi), float(st.eta), float(st.dt)
        p.rep_a, p.rep_n, p.rep_cut = (float(v) for v in st.rep)
        p.nx, p.ny, p.nz = (int(v) for v in st.dims)
        p.walls_z = int(bool(st.walls_z))
        self.p = p
        self.x = torch.as_tensor(np.ascontiguousarray(np.asarray(x, np.float64).T)).to(self.device).contiguous()
        nbytes = self.L.mag_workspace_bytes(C.byref(p))
        if nbytes <= 0:
            _lib.check(_lib.LBM_EINVAL)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._work_ptr = (self.work.data_ptr() + 255) // 256 * 256

    @property
    def n(self) -> int:
        return self.p.n

    def _stream(self):
        self.p.stream = torch.cuda.current_stream(self.device).cuda_stream

    def positions(self) -> np.ndarray:
        """Bead centres [n, 3] (waits for the stream)."""
        return self.x.cpu().numpy().T.copy()

    def set_positions(self, x: np.ndarray) -> None:
        self.x.copy_(torch.as_tensor(np.ascontiguousarray(np.asarray(x, np.float64).T)))

    def field(self, pts: np.ndarray, jacobian: bool = False):
        """B [3][npts] (and J [9][npts]) at points pts [npts, 3], as tensors."""
        P = torch.as_tensor(np.ascontiguousarray(np.asarray(pts, np.float64).reshape(-1, 3).T)).to(self.device)
        P = P.contiguous()
        B = torch.empty_like(P)
        J = torch.empty((9, P.shape[1]), dtype=torch.float64, device=self.device) if jacobian else None
        self._stream()
        _lib.check(self.L.mag_field(C.byref(self.p), _ptr(P), P.shape[1], _ptr(B), _ptr(J)))
        return (B, J) if jacobian else B

    def forces(self):
        """Moments m and total forces F, [3][n] tensors, at the current positions."""
        m = torch.empty_like(self.x)
        F = torch.empty_like(self.x)
        self._stream()
        _lib.check(self.L.mag_forces(C.byref(self.p), _ptr(self.x), _ptr(m), _ptr(F), C.c_void_p(self._work_ptr)))
        return m, F

    def run(self, nsteps: int) -> None:
        """nsteps overdamped steps (enqueued; positions updated in place)."""
        self._stream()
        _lib.check(self.L.mag_run(C.byref(self.p), _ptr(self.x), int(nsteps), C.c_void_p(self._work_ptr)))

    def freeze(self, solid: torch.Tensor) -> torch.Tensor:
        """OR the bead spheres into the uint8 device mask solid [nx*ny*nz]."""
        nx, ny, nz = self.stage.dims
        if solid.dtype != torch.uint8 or solid.numel() != nx * ny * nz or not solid.is_contiguous() \
                or solid.device != self.x.device:
            raise ValueError("solid must be a contiguous uint8 tensor of nx*ny*nz nodes on the beads' device")
        self._stream()
        _lib.check(self.L.mag_freeze(C.byref(self.p), _ptr(self.x), _ptr(solid)))
        return solid
