"""FP64 CPU oracle for the D3Q19 BGK + immersed-boundary step (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product path never imports
this package.  The arithmetic lives in ``oracle.c`` (plain C, FP64, no fast
math); this module only marshals numpy arrays.  It shares nothing with the
GPU library.

Array conventions: populations ``f`` float64 [19, N]; vector fields [3, N];
IB points [nv, 3] absolute (unwrapped) positions; N = nx*ny*nz with node
``x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; load it with libasan preloaded)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_SO = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined"]

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
        cmd = ["gcc", *opt, "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-o", _SO + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Lat(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("periodic", C.c_int * 3),
                ("tau", C.c_double), ("g", C.c_double * 3),
                ("solid", C.POINTER(C.c_uint8)), ("G", _dp)]


class _Contact(C.Structure):
    _fields_ = [("a", C.c_double), ("n", C.c_double), ("rcut", C.c_double), ("roff", C.c_double),
                ("dmin", C.c_double), ("cell_cell", C.c_int), ("nplanes", C.c_int), ("planes", _dp),
                ("ncyl", C.c_int), ("cyl", _dp), ("nsph", C.c_int), ("sph", _dp)]


class _Mesh(C.Structure):
    _fields_ = [("ncells", C.c_int), ("nverts", C.c_int), ("ntris", C.c_int), ("nedges", C.c_int),
                ("vert_off", _ip), ("tri_off", _ip), ("edge_off", _ip), ("tri", _ip), ("hinge", _ip),
                ("moduli", _dp), ("xi", C.c_double), ("mass", C.c_double), ("dt", C.c_double),
                ("stretch_law", C.c_int), ("l0", _dp), ("A0", _dp), ("th0", _dp), ("A0c", _dp), ("V0c", _dp), ("Av", _dp),
                ("contact", C.POINTER(_Contact))]


class _Trace(C.Structure):
    _fields_ = [("uk", _dp), ("Fel", _dp), ("Fc", _dp), ("F", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        L.orc_membrane_energy.restype = C.c_double
        L.orc_contact_energy.restype = C.c_double
        L.orc_dipole_energy.restype = C.c_double
        L.orc_step.restype = C.c_int
        L.orc_run.restype = C.c_int
        L.orc_objective.restype = C.c_double
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


# ---------------------------------------------------------------------------

def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(lib().orc_threads())


def d3q19():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    o = np.zeros(19, np.int32)
    lib().orc_d3q19(_i(c), _d(w), _i(o))
    return c, w, o


def equilibrium(rho: float, u) -> np.ndarray:
    out = np.zeros(19)
    lib().orc_equilibrium(C.c_double(rho), _d(np.ascontiguousarray(u, dtype=np.float64)), _d(out))
    return out


def forcing(tau: float, u, F) -> np.ndarray:
    out = np.zeros(19)
    lib().orc_forcing(C.c_double(tau), _d(np.ascontiguousarray(u, dtype=np.float64)),
                      _d(np.ascontiguousarray(F, dtype=np.float64)), _d(out))
    return out


def collide_node(tau: float, f, F) -> np.ndarray:
    out = np.zeros(19)
    lib().orc_collide_node(C.c_double(tau), _d(np.ascontiguousarray(f, dtype=np.float64)),
                           _d(np.ascontiguousarray(F, dtype=np.float64)), _d(out))
    return out


class Lattice:
    """Lattice description: size, periodicity, tau, body force g, solid mask,
    optional forcing field G [3, nz, ny, nx]."""

    def __init__(self, nx, ny, nz, tau, g=(0.0, 0.0, 0.0), solid=None, periodic=(1, 1, 1), G=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.N = self.nx * self.ny * self.nz
        self.solid = np.ascontiguousarray(
            np.zeros(self.N, np.uint8) if solid is None else np.asarray(solid, np.uint8).reshape(-1))
        assert self.solid.size == self.N
        self.G = None if G is None else np.ascontiguousarray(np.asarray(G, np.float64).reshape(3, self.N))
        self.s = _Lat(self.nx, self.ny, self.nz, (C.c_int * 3)(*periodic), float(tau),
                      (C.c_double * 3)(*g), self.solid.ctypes.data_as(C.POINTER(C.c_uint8)),
                      _d(self.G) if self.G is not None else _dp())
        self.tau = float(tau)
        self.g = tuple(float(v) for v in g)

    @classmethod
    def from_scenario(cls, s, G=None):
        return cls(s.nx, s.ny, s.nz, s.tau, s.g, s.solid, s.periodic,
                   G if G is not None else s.gfield)

    def rest(self) -> np.ndarray:
        """f = w_i on every node (rho = 1, u = 0)."""
        _, w, _ = d3q19()
        return np.repeat(w[:, None], self.N, axis=1).copy()


class Mesh:
    """Membrane population; holds its own FP64 rest-shape arrays (edge
    lengths, triangle areas, hinge angles, cell area and volume, and the
    rest area Av carried by each vertex)."""

    def __init__(self, cells, moduli=None, contact=None, stretch_law=None):
        """contact: None, or dict(a, n, rcut, roff, dmin, cell_cell, planes [np, 4], cyl [nc, 3]) of
        the soft-sphere contact forces (see orc_contact in oracle.c).  stretch_law: 0 linear,
        1 neo-Hookean (default: the cells' own)."""
        self.cells = cells
        self.vert_off = np.ascontiguousarray(cells.vert_off, np.int32)
        self.tri_off = np.ascontiguousarray(cells.tri_off, np.int32)
        self.edge_off = np.ascontiguousarray(cells.edge_off, np.int32)
        self.tri = np.ascontiguousarray(cells.tri, np.int32)
        self.hinge = np.ascontiguousarray(cells.hinge, np.int32)
        self.moduli = np.ascontiguousarray(cells.moduli if moduli is None else moduli, np.float64)
        nc, nv, nt, ne = cells.ncells, cells.nverts, cells.ntris, cells.nedges
        self.l0 = np.zeros(ne)
        self.A0 = np.zeros(nt)
        self.th0 = np.zeros(ne)
        self.A0c = np.zeros(nc)
        self.V0c = np.zeros(nc)
        self.Av = np.zeros(nv)
        self.s = _Mesh(nc, nv, nt, ne, _i(self.vert_off), _i(self.tri_off), _i(self.edge_off),
                       _i(self.tri), _i(self.hinge), _d(self.moduli), float(cells.xi),
                       float(cells.mass), float(cells.dt),
                       int(getattr(cells, "stretch_law", 0) if stretch_law is None else stretch_law),
                       _d(self.l0), _d(self.A0), _d(self.th0), _d(self.A0c), _d(self.V0c), _d(self.Av),
                       None)
        self.nverts = nv
        self._contact = None
        if contact is not None:
            self.planes = np.ascontiguousarray(np.asarray(contact.get("planes", np.zeros((0, 4))), np.float64))
            self.cyl = np.ascontiguousarray(np.asarray(contact.get("cyl", np.zeros((0, 3))), np.float64))
            self.sph = np.ascontiguousarray(np.asarray(contact.get("spheres", np.zeros((0, 4))), np.float64))
            self._contact = _Contact(float(contact["a"]), float(contact["n"]), float(contact["rcut"]),
                                     float(contact.get("roff", 0.0)), float(contact.get("dmin", 0.05)),
                                     int(contact.get("cell_cell", 1)), len(self.planes),
                                     _d(self.planes) if len(self.planes) else _dp(),
                                     len(self.cyl), _d(self.cyl) if len(self.cyl) else _dp(),
                                     len(self.sph), _d(self.sph) if len(self.sph) else _dp())
            self.s.contact = C.pointer(self._contact)

    def contact_energy(self, L, X) -> float:
        return lib().orc_contact_energy(C.byref(L.s), C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)))

    def contact_forces(self, L, X) -> np.ndarray:
        F = np.zeros((self.nverts, 3))
        lib().orc_contact_forces(C.byref(L.s), C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)), _d(F))
        return F

    def rest_shape(self, X: np.ndarray) -> None:
        lib().orc_rest_shape(C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)))

    def point_mass(self) -> np.ndarray:
        """Mass of each IB point (mass density times its rest area)."""
        return self.cells.mass * self.Av

    def energy(self, X) -> float:
        return lib().orc_membrane_energy(C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)))

    def forces(self, X) -> np.ndarray:
        F = np.zeros((self.nverts, 3))
        lib().orc_membrane_forces(C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)), _d(F))
        return F

    def area_volume(self, X):
        nc = len(self.vert_off) - 1
        A, V = np.zeros(nc), np.zeros(nc)
        lib().orc_cell_area_volume(C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)), _d(A), _d(V))
        return A, V

    def geometry(self, X):
        l = np.zeros(len(self.hinge))
        th = np.zeros(len(self.hinge))
        A = np.zeros(len(self.tri))
        lib().orc_mesh_geometry(C.byref(self.s), _d(np.ascontiguousarray(X, np.float64)), _d(l), _d(A), _d(th))
        return l, A, th


def fluid_velocity(L: Lattice, f: np.ndarray):
    rho = np.zeros(L.N)
    u = np.zeros((3, L.N))
    lib().orc_fluid_velocity(C.byref(L.s), _d(f), _d(rho), _d(u))
    return rho, u


def mass_momentum(L: Lattice, f: np.ndarray) -> np.ndarray:
    out = np.zeros(4)
    lib().orc_mass_momentum(C.byref(L.s), _d(f), _d(out))
    return out


def collide_stream(L: Lattice, f: np.ndarray, F: np.ndarray, fnew: Optional[np.ndarray] = None):
    out = f.copy() if fnew is None else fnew
    lib().orc_collide_stream(C.byref(L.s), _d(f), _d(np.ascontiguousarray(F, np.float64)), _d(out))
    return out


def interpolate(L: Lattice, field: np.ndarray, X: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    out = np.zeros((len(X), 3))
    lib().orc_interpolate(C.byref(L.s), _d(np.ascontiguousarray(field, np.float64)), C.c_int(len(X)),
                          _d(X), _d(out))
    return out


def spread(L: Lattice, X: np.ndarray, Fk: np.ndarray, field: Optional[np.ndarray] = None) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    out = np.zeros((3, L.N)) if field is None else field
    lib().orc_spread(C.byref(L.s), C.c_int(len(X)), _d(X), _d(np.ascontiguousarray(Fk, np.float64)), _d(out))
    return out


def step(L: Lattice, M: Optional[Mesh], f: np.ndarray, X=None, V=None, trace: bool = False):
    """One coupled step.  Returns fnew; X and V (float64 [nv,3]) advance in place.
    With trace=True also returns dict(uk, Fel, Fc, F) of that step."""
    fnew = np.empty_like(f)
    nv = M.nverts if M is not None else 0
    tr = None
    arrs = {}
    if trace:
        arrs = dict(uk=np.zeros((nv, 3)), Fel=np.zeros((nv, 3)), Fc=np.zeros((nv, 3)), F=np.zeros((3, L.N)))
        tr = _Trace(_d(arrs["uk"]), _d(arrs["Fel"]), _d(arrs["Fc"]), _d(arrs["F"]))
    Xp = _d(X) if X is not None else _dp()
    Vp = _d(V) if V is not None else _dp()
    rc = lib().orc_step(C.byref(L.s), C.byref(M.s) if M is not None else None, _d(f), _d(fnew), Xp, Vp,
                        C.byref(tr) if tr is not None else None)
    if rc:
        raise MemoryError("orc_step failed")
    return (fnew, arrs) if trace else fnew


def run(L: Lattice, M: Optional[Mesh], f: np.ndarray, X=None, V=None, nsteps: int = 1) -> np.ndarray:
    """nsteps coupled steps; f, X, V are advanced in place and f is returned."""
    rc = lib().orc_run(C.byref(L.s), C.byref(M.s) if M is not None else None, _d(f),
                       _d(X) if X is not None else _dp(), _d(V) if V is not None else _dp(), C.c_int(nsteps))
    if rc:
        raise MemoryError("orc_run failed")
    return f


def objective(L: Lattice, M: Optional[Mesh], f: np.ndarray, X=None, X0=None) -> float:
    """Outflow through the plane x = nx-1 (sum of j_x + (g_x + G_x)/2 over
    its fluid nodes) plus each cell's squared centroid displacement X vs X0."""
    if M is None:
        return lib().orc_objective(C.byref(L.s), None, _d(f), _dp(), _dp())
    return lib().orc_objective(C.byref(L.s), C.byref(M.s), _d(f), _d(np.ascontiguousarray(X, np.float64)),
                               _d(np.ascontiguousarray(X0, np.float64)))


# ---------------------------------------------------------------------------
# magnetic bead stage

class _Mag(C.Structure):
    _fields_ = [("nsheets", C.c_int), ("sheets", _dp), ("bias", C.c_double * 3), ("a", C.c_double),
                ("chi", C.c_double), ("eta", C.c_double), ("dt", C.c_double), ("rep_a", C.c_double),
                ("rep_n", C.c_double), ("rep_cut", C.c_double), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("periodic", C.c_int * 3), ("walls_z", C.c_int), ("quad", C.c_int)]


class Magnet:
    """Bead-stage parameters (see orc_mag in oracle.c).  sheets [ns, 6] =
    (z, x0, x1, y0, y1, sigma); positions are [n, 3] arrays."""

    def __init__(self, sheets, bias, a, chi, eta, dt, rep=(1e-3, 2.0, 0.5), dims=(64, 64, 32),
                 periodic=(1, 1, 0), walls_z=True, quad=16):
        self.sheets = np.ascontiguousarray(np.asarray(sheets, np.float64).reshape(-1, 6))
        self.s = _Mag(len(self.sheets), _d(self.sheets) if len(self.sheets) else _dp(), (C.c_double * 3)(*bias),
                      float(a), float(chi), float(eta), float(dt), float(rep[0]), float(rep[1]), float(rep[2]),
                      int(dims[0]), int(dims[1]), int(dims[2]), (C.c_int * 3)(*periodic), int(bool(walls_z)),
                      int(quad))

    def field(self, p, jacobian: bool = False):
        """B [n, 3] at points p [n, 3]; with jacobian=True also
        J [n, 3, 3], J[k, i, j] = dB_i/dx_j."""
        p = np.ascontiguousarray(np.asarray(p, np.float64).reshape(-1, 3))
        B = np.zeros_like(p)
        J = np.zeros((len(p), 3, 3)) if jacobian else None
        lib().orc_mag_field(C.byref(self.s), _d(p), C.c_int(len(p)), _d(B), _d(J) if jacobian else None)
        return (B, J) if jacobian else B

    def forces(self, x):
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
        m, F = np.zeros_like(x), np.zeros_like(x)
        lib().orc_mag_forces(C.byref(self.s), _d(x), C.c_int(len(x)), _d(m), _d(F))
        return m, F

    def forces_sample(self, x, idx) -> np.ndarray:
        """Total forces [len(idx), 3] on the beads idx only."""
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
        idx = np.ascontiguousarray(idx, np.int32)
        F = np.zeros((len(idx), 3))
        if lib().orc_mag_forces_sample(C.byref(self.s), _d(x), C.c_int(len(x)),
                                       idx.ctypes.data_as(C.POINTER(C.c_int)), C.c_int(len(idx)), _d(F)):
            raise ValueError("orc_mag_forces_sample: bad index or no memory")
        return F

    def run(self, x, nsteps: int) -> np.ndarray:
        """nsteps overdamped steps; x [n, 3] advanced in place and returned."""
        if lib().orc_mag_run(C.byref(self.s), _d(x), C.c_int(len(x)), C.c_int(nsteps)):
            raise MemoryError("orc_mag_run failed")
        return x

    def freeze(self, x, solid) -> np.ndarray:
        """OR the nodes within a bead radius of a bead centre into solid (uint8 [N])."""
        x = np.ascontiguousarray(np.asarray(x, np.float64).reshape(-1, 3))
        lib().orc_mag_freeze(C.byref(self.s), _d(x), C.c_int(len(x)),
                             solid.ctypes.data_as(C.POINTER(C.c_uint8)))
        return solid


def dipole_force(m1, m2, r) -> np.ndarray:
    F = np.zeros(3)
    lib().orc_dipole_force(_d(np.ascontiguousarray(m1, np.float64)), _d(np.ascontiguousarray(m2, np.float64)),
                           _d(np.ascontiguousarray(r, np.float64)), _d(F))
    return F


def dipole_energy(m1, m2, r) -> float:
    return lib().orc_dipole_energy(_d(np.ascontiguousarray(m1, np.float64)), _d(np.ascontiguousarray(m2, np.float64)),
                                   _d(np.ascontiguousarray(r, np.float64)))
