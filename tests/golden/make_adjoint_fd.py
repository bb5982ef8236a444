#!/usr/bin/env python3
"""Writes adjoint_fd.json: central finite differences, in FP64 with the
oracle, of the adjoint workload's objective along 16 seeded directions of
the forcing field G.

Workload: 128x64x32 channel (solid planes z = 0 and z = 31), tau 0.8,
g_x 1e-5, three cells of 162 vertices (icosphere level 2, radius 4, seed 5),
300 coupled steps from rest; G lives on the design slab 32 <= x < 96.
Objective J: x-momentum flux j_x + (g_x + G_x)/2 summed over the fluid
nodes of the plane x = 127 at step 300, plus the squared displacement of
each cell's vertex centroid.
The derivative along unit direction d is (J(eps d) - J(-eps d)) / (2 eps)
at G = 0; two directions are repeated at 2 eps to show the truncation error
is negligible.  Every value comes from the oracle (its stepper and its
objective); the seeded input generator supplies the workload.

Run from the repository root:  python tests/golden/make_adjoint_fd.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1110_0995_amd import scenario as S  # noqa: E402

EPS = 1e-4
NDIR = 16


def run(s, G):
    L = oracle.Lattice.from_scenario(s, G=G)
    M = oracle.Mesh(s.cells)
    X0 = s.cells.positions()
    X = X0.copy()
    M.rest_shape(X)
    V = np.zeros_like(X)
    f = oracle.run(L, M, L.rest(), X, V, nsteps=s.steps)
    return oracle.objective(L, M, f, X, X0)


def embed(s, d):
    x0, x1 = s.meta["design_x"]
    G = np.zeros((3, s.nz, s.ny, s.nx))
    G[..., x0:x1] = d
    return G


def main():
    oracle.build()
    s = S.adjoint_channel()
    dirs = S.random_directions(s, NDIR)
    t0 = time.time()
    J0 = run(s, np.zeros((3, s.nz, s.ny, s.nx)))
    fd, fd2 = [], []
    for k in range(NDIR):
        G = embed(s, dirs[k])
        fd.append((run(s, EPS * G) - run(s, -EPS * G)) / (2 * EPS))
        if k < 2:
            fd2.append((run(s, 2 * EPS * G) - run(s, -2 * EPS * G)) / (4 * EPS))
        print(f"direction {k}: {fd[-1]:.12e}  ({time.time() - t0:.0f} s)", flush=True)
    out = dict(workload="adjoint_channel 128x64x32, 3 cells level 2, tau 0.8, g_x 1e-5, 300 steps, seed 5",
               design_x=s.meta["design_x"], direction_seeds=list(range(NDIR)), eps=EPS, J0=J0,
               fd=fd, fd_2eps=fd2, threads=oracle.threads())
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
