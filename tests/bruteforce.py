"""A second, deliberately naive FP64 stepper used only to pin the oracle.

It is written independently of oracle.c: the D3Q19 set is generated here
from its definition (all c in {-1,0,1}^3 with |c|^2 <= 2, weights from
|c|^2), streaming walks explicit Python loops over nodes, and the
trilinear stencil enumerates corners directly.  It is meant for lattices of
a few hundred nodes.
"""
import itertools

import numpy as np


def lattice_set():
    """D3Q19 from its definition, returned in the oracle's ordering (rest,
    then +-x, +-y, +-z, then the 12 edges in pairs); the ordering is matched
    by looking velocities up, not by copying a table."""
    vel = [c for c in itertools.product((-1, 0, 1), repeat=3) if sum(v * v for v in c) <= 2]
    assert len(vel) == 19
    wt = {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}
    return vel, {c: wt[sum(v * v for v in c)] for c in vel}


class Brute:
    def __init__(self, c_table, nx, ny, nz, tau, g, solid, periodic=(1, 1, 1), G=None):
        # c_table: the oracle's ordering of velocities, used only to map slots
        vel, w = lattice_set()
        self.c = [tuple(int(v) for v in row) for row in c_table]
        assert sorted(self.c) == sorted(vel)
        self.w = [w[c] for c in self.c]
        self.dims = (nx, ny, nz)
        self.tau = tau
        self.g = np.array(g, float)
        self.solid = np.asarray(solid, np.uint8).reshape(nz, ny, nx)
        self.periodic = periodic
        self.G = None if G is None else np.asarray(G, float).reshape(3, nz, ny, nx)

    def slot(self, c):
        return self.c.index(tuple(c))

    def fext(self, x, y, z):
        F = self.g.copy()
        if self.G is not None:
            F += self.G[:, z, y, x]
        return F

    def moments(self, f, x, y, z):
        fl = f[:, z, y, x]
        rho = fl.sum()
        j = sum(fl[i] * np.array(self.c[i], float) for i in range(19))
        return rho, j

    def uext_field(self, f):
        nx, ny, nz = self.dims
        u = np.zeros((3, nz, ny, nx))
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            if self.solid[z, y, x]:
                continue
            rho, j = self.moments(f, x, y, z)
            u[:, z, y, x] = (j + 0.5 * self.fext(x, y, z)) / rho
        return u

    def corners(self, X):
        nx, ny, nz = self.dims
        base = np.floor(X).astype(int)
        fr = X - base
        out = []
        for b in itertools.product((0, 1), repeat=3):
            wgt = 1.0
            for d in range(3):
                wgt *= fr[d] if b[d] else 1.0 - fr[d]
            p = ((base[0] + b[0]) % nx, (base[1] + b[1]) % ny, (base[2] + b[2]) % nz)
            out.append((p, wgt))
        return out

    def interp(self, field, X):
        out = np.zeros((len(X), 3))
        for k, Xk in enumerate(X):
            for (x, y, z), wgt in self.corners(Xk):
                out[k] += wgt * field[:, z, y, x]
        return out

    def spread(self, X, Fk, field):
        for k, Xk in enumerate(X):
            for (x, y, z), wgt in self.corners(Xk):
                field[:, z, y, x] += wgt * Fk[k]

    def collide(self, fl, F):
        rho = fl.sum()
        j = sum(fl[i] * np.array(self.c[i], float) for i in range(19))
        u = (j + 0.5 * F) / rho
        out = np.empty(19)
        for i, c in enumerate(self.c):
            c = np.array(c, float)
            cu = c @ u
            feq = self.w[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (u @ u))
            src = (1 - 0.5 / self.tau) * self.w[i] * ((3 * (c - u) + 9 * cu * c) @ F)
            out[i] = fl[i] - (fl[i] - feq) / self.tau + src
        return out

    def step(self, f, X=None, V=None, Fel=None, xi=1.0, mass=1.0, dt=1.0):
        """f [19, nz, ny, nx].  Fel (elastic forces at the current X) is an
        input: the membrane forces are pinned on their own.  xi and mass may
        be per-point arrays [nv, 1]."""
        nx, ny, nz = self.dims
        F = np.zeros((3, nz, ny, nx))
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            F[:, z, y, x] = self.fext(x, y, z)
        Fc = None
        if X is not None and len(X):
            uk = self.interp(self.uext_field(f), X)
            Fc = xi * (uk - V)
            self.spread(X, -Fc, F)
        fn = f.copy()
        for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
            if self.solid[z, y, x]:
                continue
            fo = self.collide(f[:, z, y, x], F[:, z, y, x])
            for i, c in enumerate(self.c):
                p = [x + c[0], y + c[1], z + c[2]]
                out = False
                for d, n in enumerate(self.dims):
                    if p[d] < 0 or p[d] >= n:
                        if self.periodic[d]:
                            p[d] %= n
                        else:
                            out = True
                if out or self.solid[p[2], p[1], p[0]]:
                    fn[self.slot([-v for v in c]), z, y, x] = fo[i]
                else:
                    fn[i, p[2], p[1], p[0]] = fo[i]
        if Fc is not None:
            V = V + dt / mass * (Fel + Fc)
            X = X + dt * V
        return fn, X, V
