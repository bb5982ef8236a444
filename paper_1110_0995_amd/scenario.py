"""Seeded synthetic inputs for the D3Q19 + immersed-boundary cell-flow step.

Geometry and bookkeeping only: solid masks (channel walls, cylindrical
microposts), icosphere membrane meshes with their edge/hinge connectivity,
seeded random sequential placement of cells, and the parameter records of the
workloads.  Nothing in this module evaluates lattice-Boltzmann or
immersed-boundary arithmetic (no equilibria, no forces, no reference lengths,
areas, angles or volumes): the GPU library and the CPU oracle both take these
arrays as plain inputs and derive everything else themselves.

Conventions shared by every consumer of these arrays
----------------------------------------------------
* Lattice arrays are indexed ``[z, y, x]`` with x fastest; node id
  ``n = x + nx*(y + ny*z)``.
* ``solid`` is uint8, 1 = solid (bounce-back) node, 0 = fluid node.  The
  paper distinguishes boundary and fluid nodes and places the wall between
  them (Sec. 2.4).
* A cell membrane is a closed triangle mesh.  ``tri[t] = (a, b, c)`` is
  ordered counter-clockwise seen from outside, so ``(b-a) x (c-a)`` points
  outward.  Every undirected edge appears once in ``hinge[e] = (p1, p2, qa,
  qb)``: triangle ``(p1, p2, qa)`` and triangle ``(p2, p1, qb)`` (both in the
  cyclic order of ``tri``) share it.  Indices are global vertex ids.
* IB-point positions are stored as an int32 anchor per cell plus a float32
  offset per vertex; the position is ``anchor + offset`` (evaluated exactly
  in float64 by anyone who wants absolute coordinates).
* ``moduli[c] = (k_s, k_b, k_al, k_ag, k_v)`` for cell c (Table 1 names:
  K^S, K^B, K^A_l, K^A_g, K^V).
"""
from __future__ import annotations

import dataclasses
import json
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Table 1 of the paper: elastic constants of the two cell models, in the
# order (k_s, k_b, k_al, k_ag, k_v).  The table gives no units; they are used
# as lattice-unit values.
MODULI_CTC = (0.0023, 0.000464, 0.0029, 0.29, 2.9)
MODULI_RBC = (0.008, 0.0016, 0.01, 1.0, 10.0)
# Membrane mass per unit area for red cells.  The explicit point update is
# linearly stable while the stiffest membrane mode satisfies
# lambda_max(H / m) < 2 + 2 (1 - xi/mass) (H the energy Hessian, friction xi
# per area); with the red-cell moduli on the biconcave disc lambda_max is
# about 14 / mass (the volume term dominates), so mass 2 is unstable and 8
# leaves a wide margin.  Tumour cells (sphere, CTC moduli: about 2.2 / mass)
# keep mass 2.
MASS_RBC = 8.0


# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------

def _icosahedron() -> Tuple[np.ndarray, np.ndarray]:
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        (-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
        (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
        (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
        (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
        (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
        (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], dtype=np.int64)
    return v, f


def _orient_outward(v: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Flip triangles of a star-shaped mesh (about the origin) to face outward."""
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    out = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) > 0
    g = f.copy()
    g[~out] = g[~out][:, [0, 2, 1]]
    return g


def icosphere(level: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: the icosahedron with each triangle split into four
    ``level`` times, new vertices pushed onto the sphere.  Returns (verts
    [V,3] float64, tris [T,3] int64), V = 10*4^level + 2, T = 20*4^level."""
    v, f = _icosahedron()
    verts: List[np.ndarray] = list(v)
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    v = np.array(verts, dtype=np.float64)
    return v, _orient_outward(v, f)


def hinges(tris: np.ndarray) -> np.ndarray:
    """Edge/hinge table of a closed oriented triangle mesh.

    Returns int64 [E,4] rows (p1, p2, qa, qb), p1 < p2, where (p1, p2, qa) is
    the cyclic order of one triangle and (p2, p1, qb) that of the other."""
    opp = {}
    for a, b, c in tris:
        for p, q, r in ((a, b, c), (b, c, a), (c, a, b)):
            key = (int(p), int(q))
            if key in opp:
                raise ValueError("mesh is not consistently oriented")
            opp[key] = int(r)
    rows = []
    for (p, q), r in opp.items():
        if p < q:
            if (q, p) not in opp:
                raise ValueError("mesh is not closed")
            rows.append((p, q, r, opp[(q, p)]))
    rows.sort()
    return np.array(rows, dtype=np.int64)


# ---------------------------------------------------------------------------
# solid masks
# ---------------------------------------------------------------------------

def channel_mask(nx: int, ny: int, nz: int, walls_z: bool = True) -> np.ndarray:
    """uint8 [nz, ny, nx]; the planes z = 0 and z = nz-1 are solid walls."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    if walls_z:
        m[0] = 1
        m[nz - 1] = 1
    return m


def add_posts(mask: np.ndarray, centres: Sequence[Tuple[float, float]], radius: float) -> None:
    """Cylinders with axis along z over the full height: node (x, y) is solid
    iff (x-xc)^2 + (y-yc)^2 <= r^2 (no periodic images)."""
    nz, ny, nx = mask.shape
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for xc, yc in centres:
        inside = (xx - xc) ** 2 + (yy - yc) ** 2 <= radius * radius
        mask[:, inside] = 1


def post_array_centres(nx: int, ny: int, gaps_x: Sequence[int], gaps_y: Sequence[int],
                       radius: int) -> List[Tuple[float, float]]:
    """Rectangular post array, centred in the (x, y) plane.  Neighbouring
    centres are 2*radius + gap apart (gap = surface-to-surface distance);
    the array is shifted by an integer so every centre stays on a node."""
    xs = np.concatenate([[0], np.cumsum(2 * radius + np.asarray(gaps_x, dtype=np.int64))])
    ys = np.concatenate([[0], np.cumsum(2 * radius + np.asarray(gaps_y, dtype=np.int64))])
    xs = xs + (nx // 2 - int(round(xs.mean())))
    ys = ys + (ny // 2 - int(round(ys.mean())))
    return [(float(x), float(y)) for y in ys for x in xs]


# ---------------------------------------------------------------------------
# cell placement
# ---------------------------------------------------------------------------

def place_cells(rng: np.random.Generator, n: int, radius: float, dims: Tuple[int, int, int],
                posts: Sequence[Tuple[float, float]] = (), post_radius: float = 0.0,
                clearance: float = 1.0, walls_z: bool = True, max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition of n spheres (centres float64 [n,3]).

    Centres are uniform over the fluid box; a candidate is kept if it stays
    ``clearance`` away from every kept sphere (periodic minimum image in x
    and y), from the wall planes z = 0.5 and z = nz-1.5, and from every
    post surface."""
    nx, ny, nz = dims
    zlo, zhi = (0.5, nz - 1.5) if walls_z else (0.0, float(nz))
    cen: List[np.ndarray] = []
    tries = 0
    while len(cen) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could only place {len(cen)} of {n} cells")
        lo = zlo + radius + clearance if walls_z else 0.0
        hi = zhi - radius - clearance if walls_z else float(nz)
        p = np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(lo, hi)])
        ok = True
        for xc, yc in posts:
            dx = (p[0] - xc + nx / 2) % nx - nx / 2
            dy = (p[1] - yc + ny / 2) % ny - ny / 2
            if math.hypot(dx, dy) < post_radius + 0.5 + radius + clearance:
                ok = False
                break
        if ok:
            for q in cen:
                d = p - q
                d[0] = (d[0] + nx / 2) % nx - nx / 2
                d[1] = (d[1] + ny / 2) % ny - ny / 2
                if not walls_z:
                    d[2] = (d[2] + nz / 2) % nz - nz / 2
                if np.linalg.norm(d) < 2 * radius + clearance:
                    ok = False
                    break
        if ok:
            cen.append(p)
    return np.array(cen, dtype=np.float64).reshape(n, 3)


# ---------------------------------------------------------------------------
# scenario record
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Cells:
    """A population of closed membranes in one lattice."""
    vert_off: np.ndarray   # int32 [ncells+1]
    tri_off: np.ndarray    # int32 [ncells+1]
    edge_off: np.ndarray   # int32 [ncells+1]
    tri: np.ndarray        # int32 [ntris, 3]   global vertex ids
    hinge: np.ndarray      # int32 [nedges, 4]  global vertex ids
    anchor: np.ndarray     # int32 [ncells, 3]
    offset: np.ndarray     # float32 [nverts, 3]
    moduli: np.ndarray     # float64 [ncells, 5]  (k_s, k_b, k_al, k_ag, k_v)
    xi: float = 1.0        # coupling friction per unit membrane area
    mass: float = 2.0      # membrane mass per unit area (IB-point mass = mass * its rest area)
    dt: float = 1.0        # IB time step (one per lattice step)
    stretch_law: int = 0   # 0: linear edge springs, 1: neo-Hookean edge springs

    @property
    def ncells(self) -> int:
        return len(self.vert_off) - 1

    @property
    def nverts(self) -> int:
        return int(self.vert_off[-1])

    @property
    def ntris(self) -> int:
        return int(self.tri_off[-1])

    @property
    def nedges(self) -> int:
        return int(self.edge_off[-1])

    def vertex_cell(self) -> np.ndarray:
        return np.repeat(np.arange(self.ncells, dtype=np.int32), np.diff(self.vert_off))

    def positions(self) -> np.ndarray:
        """Absolute (unwrapped) IB-point positions, float64 [nverts, 3]."""
        return self.anchor[self.vertex_cell()].astype(np.float64) + self.offset.astype(np.float64)


def morton_order(unit: np.ndarray, bits: int = 10) -> np.ndarray:
    """Permutation sorting points of [-1,1]^3 along a Z-order curve."""
    q = np.clip(((unit + 1.0) * 0.5 * ((1 << bits) - 1)).round().astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(unit), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


# Evans-Fung biconcave profile of a red blood cell (Evans and Fung 1972):
# half-thickness h(rho) = (R/2) sqrt(1 - rho^2) (C0 + C1 rho^2 + C2 rho^4)
# at rho = r/R, R the disc radius.
EVANS_FUNG = (0.207161, 2.002558, -1.122762)


def biconcave(unit: np.ndarray) -> np.ndarray:
    """Map unit-sphere points onto the biconcave disc of radius 1 (axis z):
    (x, y) kept, z replaced by sign(z) h(rho) with rho^2 = x^2 + y^2."""
    c0, c1, c2 = EVANS_FUNG
    rho2 = np.clip(unit[:, 0] ** 2 + unit[:, 1] ** 2, 0.0, 1.0)
    h = 0.5 * np.sqrt(1.0 - rho2) * (c0 + c1 * rho2 + c2 * rho2 ** 2)
    return np.stack([unit[:, 0], unit[:, 1], np.sign(unit[:, 2]) * h], axis=1)


def make_cells(centres: np.ndarray, radius: float, level: int,
               moduli: Sequence[float] = MODULI_CTC, xi: float = 1.0, shape: str = "sphere",
               stretch_law: int = 0, mass: float = 2.0, rotations: Optional[np.ndarray] = None) -> Cells:
    """Icosphere cells of the given radius around ``centres`` [n,3]; with
    shape="rbc" the icosphere is mapped onto the biconcave disc of that
    radius (red blood cell, Table 1 geometry); ``rotations`` [n,3,3]
    optionally turns each cell's template.

    The template's vertices are numbered along a Z-order curve, so
    consecutive vertex ids are neighbours on the surface (and so are the
    lattice nodes their stencils touch)."""
    unit, tris = icosphere(level)
    if shape == "rbc":
        unit = biconcave(unit)
    elif shape != "sphere":
        raise ValueError(f"unknown cell shape {shape}")
    perm = morton_order(unit)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    unit = unit[perm]
    tris = inv[tris]
    tris = tris[np.argsort(tris.min(axis=1), kind="stable")]
    hin = hinges(tris)
    nv, nt, ne = len(unit), len(tris), len(hin)
    n = len(centres)
    anchor = np.floor(centres).astype(np.int32)
    shaped = radius * unit[None, :, :]
    if rotations is not None:
        shaped = np.einsum("cij,vj->cvi", np.asarray(rotations, np.float64), radius * unit)
    off = (shaped + (centres - anchor)[:, None, :]).astype(np.float32)
    base = (np.arange(n) * nv)[:, None, None]
    return Cells(
        vert_off=(np.arange(n + 1) * nv).astype(np.int32),
        tri_off=(np.arange(n + 1) * nt).astype(np.int32),
        edge_off=(np.arange(n + 1) * ne).astype(np.int32),
        tri=(tris[None] + base).reshape(-1, 3).astype(np.int32),
        hinge=(hin[None] + base).reshape(-1, 4).astype(np.int32),
        anchor=anchor,
        offset=off.reshape(-1, 3),
        moduli=np.tile(np.asarray(moduli, dtype=np.float64), (n, 1)),
        xi=xi, mass=float(mass), stretch_law=int(stretch_law))


@dataclasses.dataclass
class Scenario:
    """One lattice workload: geometry, fluid parameters and (optionally) cells."""
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    g: Tuple[float, float, float]
    solid: np.ndarray                 # uint8 [nz, ny, nx]
    steps: int
    periodic: Tuple[int, int, int] = (1, 1, 1)
    cells: Optional[Cells] = None
    gfield: Optional[np.ndarray] = None   # float64 [3, nz, ny, nx] external forcing field G
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def fluid_fraction(self) -> float:
        return float(1.0 - self.solid.mean())


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def poiseuille(nx: int = 64, ny: int = 16, nz: int = 16, tau: float = 1.0, gx: float = 1e-6,
               steps: int = 1000) -> Scenario:
    """Plain D3Q19 channel, solid planes z = 0 and z = nz-1, body force along x.

    Defaults: 64x16x16, tau = 1, g_x = 1e-6, 1000 steps."""
    return Scenario("poiseuille", nx, ny, nz, tau, (gx, 0.0, 0.0), channel_mask(nx, ny, nz), steps)


def posts_and_cells(nx: int = 256, ny: int = 128, nz: int = 64, *, posts_x: int = 4, posts_y: int = 2,
                    post_radius: int = 8, gap: int = 12, ncells: int = 20, cell_radius: float = 4.0,
                    level: int = 3, tau: float = 0.8, gx: float = 1e-5, steps: int = 2000,
                    seed: int = 2, moduli=MODULI_CTC) -> Scenario:
    """Channel with a regular post array and seeded cells.

    Defaults: 256x128x64, 4x2 posts of radius 8 with gap 12, 20 cells of
    radius 4 (icosphere level 3, 642 vertices), tau = 0.8, g_x = 1e-5."""
    rng = np.random.default_rng(seed)
    mask = channel_mask(nx, ny, nz)
    centres = post_array_centres(nx, ny, [gap] * (posts_x - 1), [gap] * (posts_y - 1), post_radius) \
        if posts_x * posts_y else []
    add_posts(mask, centres, post_radius)
    cells = None
    if ncells:
        cen = place_cells(rng, ncells, cell_radius, (nx, ny, nz), centres, post_radius)
        cells = make_cells(cen, cell_radius, level, moduli)
    return Scenario("posts_cells", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                    meta=dict(post_centres=centres, post_radius=post_radius, seed=seed))


def throughput(nx: int = 512, ny: int = 256, nz: int = 128, *, posts_x: int = 8, posts_y: int = 4,
               post_radius: int = 8, gap_range=(6, 14), ncells: int = 400, cell_radius: float = 10.0,
               level: int = 3, tau: float = 0.7, gx: float = 1e-5, steps: int = 1000,
               seed: int = 3) -> Scenario:
    """Large channel: 8x4 posts with integer gaps drawn from U{6..14}, 400
    cells of 642 vertices (radius 10 gives about 10 % volume fraction)."""
    rng = np.random.default_rng(seed)
    mask = channel_mask(nx, ny, nz)
    gx_ = rng.integers(gap_range[0], gap_range[1] + 1, size=posts_x - 1)
    gy_ = rng.integers(gap_range[0], gap_range[1] + 1, size=posts_y - 1)
    centres = post_array_centres(nx, ny, gx_, gy_, post_radius)
    add_posts(mask, centres, post_radius)
    cen = place_cells(rng, ncells, cell_radius, (nx, ny, nz), centres, post_radius)
    cells = make_cells(cen, cell_radius, level)
    vol = ncells * 4.0 / 3.0 * math.pi * cell_radius ** 3 / (nx * ny * nz)
    return Scenario("throughput", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                    meta=dict(post_centres=centres, post_radius=post_radius, seed=seed,
                              gaps_x=gx_.tolist(), gaps_y=gy_.tolist(), volume_fraction=vol))


def gap_sweep(nch: int = 64, *, lengths=(64, 128, 192, 256), ny: int = 64, nz: int = 32,
              gap_range=(4, 16), post_radius: int = 8, ncells: int = 5, cell_radius: float = 4.0,
              level: int = 3, tau: float = 0.8, gx: float = 1e-5, steps: int = 2000,
              seed: int = 4) -> List[Scenario]:
    """Independent channels of uneven length, each with one post pair across
    the channel (gap drawn from U{4..16}) in front of which cells are seeded."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(nch):
        L = int(rng.choice(lengths))
        gap = int(rng.integers(gap_range[0], gap_range[1] + 1))
        mask = channel_mask(L, ny, nz)
        centres = [(L / 2.0, ny / 2.0 - (post_radius + gap / 2.0)),
                   (L / 2.0, ny / 2.0 + (post_radius + gap / 2.0))]
        add_posts(mask, centres, post_radius)
        cells = None
        if ncells:
            cen = place_cells(rng, ncells, cell_radius, (L, ny, nz), centres, post_radius)
            cells = make_cells(cen, cell_radius, level)
        out.append(Scenario(f"channel{c}", L, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                            meta=dict(gap=gap, post_centres=centres, post_radius=post_radius)))
    return out


# Soft-sphere contact law (a reading: the paper names the potential, not its
# parameters): U(d) = a d^-n for d in (0, rcut), linear below dmin.
CONTACT = dict(a=1e-4, n=2.0, rcut=1.0, roff=0.0, dmin=0.05, cell_cell=1)


def contact_walls(s: Scenario):
    """Analytic wall surfaces of a channel scenario for the contact forces:
    the halfway-bounce-back planes of the solid z layers (z = 1/2 and
    z = nz - 3/2, unit normals into the fluid) and, for each post, a z-axis
    cylinder of radius post_radius + 1/2 (the staircase surface of the
    solid nodes within post_radius).  Returns (planes [np, 4], cyl [nc, 3])."""
    planes = np.array([[0.0, 0.0, 1.0, 0.5], [0.0, 0.0, -1.0, -(s.nz - 1.5)]])
    cen = s.meta.get("post_centres", [])
    r = float(s.meta.get("post_radius", 0)) + 0.5
    cyl = np.array([[float(cx), float(cy), r] for cx, cy in cen]).reshape(-1, 3)
    return planes, cyl


def contact_params(s: Scenario, **kw) -> dict:
    planes, cyl = contact_walls(s)
    d = dict(CONTACT, planes=planes, cyl=cyl)
    d.update(kw)
    return d


def bead_spheres(x: np.ndarray, a: float) -> np.ndarray:
    """Contact spheres [n, 4] of frozen beads: centre and radius a + 1/2
    (the staircase surface of the solid nodes within a of the centre), as
    for the posts."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    return np.column_stack([x, np.full(len(x), a + 0.5)])


def contact_params_batch(scenarios: Sequence[Scenario], **kw) -> dict:
    """Contact walls of batched channels: each channel's posts as a run of
    cylinders (cyl_off [nch + 1]); the z planes are shared, so the channels
    must have the same nz."""
    if len({s.nz for s in scenarios}) != 1:
        raise ValueError("batched contact walls need channels of one height")
    parts = [contact_walls(s) for s in scenarios]
    cyl = np.concatenate([c for _, c in parts]).reshape(-1, 3)
    off = np.concatenate([[0], np.cumsum([len(c) for _, c in parts])]).astype(np.int32)
    d = dict(CONTACT, planes=parts[0][0], cyl=cyl, cyl_off=off)
    d.update(kw)
    return d


def concat_cells(populations: Sequence[Cells]) -> Cells:
    """One population from several (vertex, triangle and edge ids renumbered)."""
    cells, _ = _concat([(0, c) for c in populations])
    return cells


def batch_cells(scenarios: Sequence[Scenario]) -> Tuple[Optional[Cells], np.ndarray]:
    """Concatenate the cell populations of several channels into one (vertex,
    triangle and edge ids renumbered) and give the channel of each cell."""
    parts = [(k, s.cells) for k, s in enumerate(scenarios) if s.cells is not None]
    if not parts:
        return None, np.zeros(0, np.int32)
    return _concat(parts)


def _concat(parts) -> Tuple[Cells, np.ndarray]:
    vo, to, eo = [0], [0], [0]
    tri, hin, anc, off, mod, chan = [], [], [], [], [], []
    for k, c in parts:
        tri.append(c.tri + vo[-1])
        hin.append(c.hinge + vo[-1])
        vo.extend((c.vert_off[1:] + vo[-1]).tolist())
        to.extend((c.tri_off[1:] + to[-1]).tolist())
        eo.extend((c.edge_off[1:] + eo[-1]).tolist())
        anc.append(c.anchor)
        off.append(c.offset)
        mod.append(c.moduli)
        chan.append(np.full(c.ncells, k, np.int32))
    c0 = parts[0][1]
    for _, c in parts:
        if (c.xi, c.mass, c.dt, c.stretch_law) != (c0.xi, c0.mass, c0.dt, c0.stretch_law):
            raise ValueError("batched cells must share xi, mass, dt and the stretching law")
    cells = Cells(np.asarray(vo, np.int32), np.asarray(to, np.int32), np.asarray(eo, np.int32),
                  np.concatenate(tri).astype(np.int32), np.concatenate(hin).astype(np.int32),
                  np.concatenate(anc).astype(np.int32), np.concatenate(off), np.concatenate(mod),
                  xi=c0.xi, mass=c0.mass, dt=c0.dt, stretch_law=c0.stretch_law)
    return cells, np.concatenate(chan)


def gap_pair(nx: int = 64, ny: int = 32, nz: int = 24, *, gap: int = 8, post_radius: int = 4,
             cell_centre=(14.0, None, None), cell_radius: float = 3.0, level: int = 2,
             moduli: Sequence[float] = MODULI_CTC, tau: float = 0.8, gx: float = 5e-5, steps: int = 1200) -> Scenario:
    """One channel with a post pair across it at x = nx/2 (centres
    y = ny/2 -+ (post_radius + gap/2)) and one cell upstream, centred on the
    gap unless cell_centre says otherwise."""
    mask = channel_mask(nx, ny, nz)
    centres = [(nx / 2.0, ny / 2.0 - (post_radius + gap / 2.0)), (nx / 2.0, ny / 2.0 + (post_radius + gap / 2.0))]
    add_posts(mask, centres, post_radius)
    c = [cell_centre[0], ny / 2.0 if cell_centre[1] is None else cell_centre[1],
         (nz - 1) / 2.0 if cell_centre[2] is None else cell_centre[2]]
    cells = make_cells(np.array([c], np.float64), cell_radius, level, moduli)
    return Scenario(f"gap{gap}", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                    meta=dict(gap=gap, post_centres=centres, post_radius=post_radius))


# Table 1 cell diameters in micrometres.  The gap ladder takes one lattice
# spacing as one micrometre, so the paper's 1 um gap steps are 1 LU steps.
DIAMETER_RBC = 8.0
DIAMETER_CTC = 16.0
# the disc's axis turned from z onto x: a red cell meets the opening face-on
_AXIS_Z_TO_X = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])


def slit_posts(nx: int, ny: int, gap: int, post_radius: int, pitch: Optional[int] = None):
    """Centres of a row of overlapping z-axis posts across the whole width of
    a y-periodic channel at x = nx/2, leaving one opening.  At x = nx/2 the
    fluid nodes of the opening are y0 .. y0 + gap - 1 (y0 = ny/2 - gap//2),
    so its halfway bounce-back surfaces are exactly ``gap`` apart; posts
    ``pitch`` apart (default the radius) overlap, so nothing else is open.
    The two posts bounding the opening come first.  Returns (centres, the
    y of the opening's midline)."""
    if gap < 1:
        raise ValueError("the opening needs at least one fluid node")
    p = post_radius if pitch is None else pitch
    xc = nx / 2.0
    y0 = ny // 2 - gap // 2
    lo, hi = y0 - 1 - post_radius, y0 + gap + post_radius
    cen = [(xc, float(lo)), (xc, float(hi))]
    y = hi + p
    while y - p <= ny - 1:
        cen.append((xc, float(y)))
        y += p
    y = lo - p
    while y + p >= 0:
        cen.append((xc, float(y)))
        y -= p
    return cen, y0 + (gap - 1) / 2.0


def gap_ladder(cell: str, gaps: Sequence[int], *, nx: int = 80, ny: int = 32, nz: int = 24,
               post_radius: int = 4, level: int = 3, tau: float = 0.8, gx: float = 5e-5,
               clearance: float = 1.5, steps: int = 20000) -> List[Scenario]:
    """The minimum-gap experiment of Sec. 3 for one cell type: one channel
    per gap (gaps in lattice units = micrometres), each closed across its
    width by a row of posts (slit_posts) except for the opening, and one cell
    centred on the opening's midline and at mid-height, its front
    ``clearance`` upstream of the posts' surface.  cell = "tumour": sphere
    of diameter 16 with the tumour-cell moduli of Table 1; cell = "red":
    biconcave disc of diameter 8 facing the opening, red-cell moduli.  Both
    use neo-Hookean stretching and the red cells' membrane mass (so one
    batch can hold both).  The channels share their shape, so a ladder of
    each type can be stepped as one batch."""
    if cell == "tumour":
        radius, moduli, shape, rot = DIAMETER_CTC / 2.0, MODULI_CTC, "sphere", None
    elif cell == "red":
        radius, moduli, shape, rot = DIAMETER_RBC / 2.0, MODULI_RBC, "rbc", _AXIS_Z_TO_X
    else:
        raise ValueError(f"unknown cell type {cell}")
    unit, _ = icosphere(level)
    if shape == "rbc":
        unit = biconcave(unit)
    tmpl = radius * unit if rot is None else radius * unit @ rot.T
    half_x = float(np.abs(tmpl[:, 0]).max())
    out = []
    for g in gaps:
        g = int(g)
        mask = channel_mask(nx, ny, nz)
        cen, ymid = slit_posts(nx, ny, g, post_radius)
        add_posts(mask, cen, post_radius)
        face = nx / 2.0 - post_radius - 0.5  # upstream surface of the posts (halfway bounce-back)
        c = np.array([[face - clearance - half_x, ymid, (nz - 1) / 2.0]])
        cells = make_cells(c, radius, level, moduli, shape=shape, stretch_law=1, mass=MASS_RBC,
                           rotations=None if rot is None else rot[None])
        out.append(Scenario(f"{cell}_gap{g}", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                            meta=dict(gap=g, cell=cell, post_centres=cen, post_radius=post_radius,
                                      exit_x=nx / 2.0 + post_radius + 0.5, midline=ymid)))
    return out


def adjoint_channel(nx: int = 128, ny: int = 64, nz: int = 32, *, ncells: int = 3,
                    cell_radius: float = 4.0, level: int = 2, tau: float = 0.8, gx: float = 1e-5,
                    steps: int = 300, seed: int = 5, design_x=(32, 96)) -> Scenario:
    """Channel without posts, 3 cells of 162 vertices; the forcing field G
    lives on the design slab design_x[0] <= x < design_x[1] (all y, z)."""
    rng = np.random.default_rng(seed)
    mask = channel_mask(nx, ny, nz)
    cen = place_cells(rng, ncells, cell_radius, (nx, ny, nz))
    cells = make_cells(cen, cell_radius, level)
    return Scenario("adjoint", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                    gfield=np.zeros((3, nz, ny, nx)),
                    meta=dict(design_x=list(design_x), checkpoint_every=20, seed=seed))


def design_region_size(s: Scenario) -> int:
    x0, x1 = s.meta["design_x"]
    return (x1 - x0) * s.ny * s.nz


def random_directions(s: Scenario, count: int = 16, seed0: int = 0) -> np.ndarray:
    """Seeded unit directions over the design region, [count, 3, nz, ny, x1-x0]."""
    x0, x1 = s.meta["design_x"]
    out = np.empty((count, 3, s.nz, s.ny, x1 - x0))
    for k in range(count):
        v = np.random.default_rng(seed0 + k).standard_normal((3, s.nz, s.ny, x1 - x0))
        out[k] = v / np.linalg.norm(v)
    return out


def random_field(rng: np.random.Generator, shape, amp: float) -> np.ndarray:
    """Seeded uniform noise in [-amp, amp] (float64), e.g. a forcing field G."""
    return amp * rng.uniform(-1.0, 1.0, size=shape)


def to_json(s: Scenario) -> str:
    d = dict(name=s.name, nx=s.nx, ny=s.ny, nz=s.nz, tau=s.tau, g=list(s.g), steps=s.steps,
             periodic=list(s.periodic), ncells=(s.cells.ncells if s.cells else 0),
             nverts=(s.cells.nverts if s.cells else 0), meta=s.meta)
    return json.dumps(d, default=float)


# ---------------------------------------------------------------------------
# magnetic bead stage (Sec. 2.5): the inputs of the chain-forming stage
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class BeadStage:
    """Inputs of the bead stage: bead centres x [n, 3] (float64), charge
    sheets [ns, 6] = (z, x0, x1, y0, y1, sigma), homogeneous bias field,
    bead radius a, susceptibility chi, viscosity eta, time step dt, bead
    repulsion rep = (A, n, cut), lattice dims, periodic axes, walls at
    z = 1/2 and nz - 3/2."""
    x: np.ndarray
    sheets: np.ndarray
    bias: Tuple[float, float, float]
    a: float
    chi: float
    eta: float
    dt: float
    rep: Tuple[float, float, float]
    dims: Tuple[int, int, int]
    periodic: Tuple[int, int, int] = (1, 1, 0)
    walls_z: bool = True
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.x)


def place_beads(rng: np.random.Generator, n: int, a: float, dims: Tuple[int, int, int], zlim: Tuple[float, float],
                min_gap: float, xlim: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Random sequential addition of n bead centres in xlim (default
    [0, nx)) x [0, ny) x zlim, pairwise centre distances > 2a + min_gap
    (minimum image in x and y), using a uniform grid of bins no smaller than
    that distance."""
    nx, ny, _ = dims
    xlo, xhi = xlim if xlim is not None else (0.0, float(nx))
    dmin = 2 * a + min_gap
    nbx, nby = max(1, int(nx // dmin)), max(1, int(ny // dmin))
    nbz = max(1, int((zlim[1] - zlim[0]) // dmin))
    bins: dict = {}
    out = np.zeros((n, 3))
    k = tries = 0
    while k < n:
        tries += 1
        if tries > 200 * n + 10000:
            raise RuntimeError(f"could not place {n} beads (placed {k})")
        p = np.array([rng.uniform(xlo, xhi), rng.uniform(0, ny), rng.uniform(*zlim)])
        b = (int(p[0] / nx * nbx) % nbx, int(p[1] / ny * nby) % nby,
             min(nbz - 1, int((p[2] - zlim[0]) / (zlim[1] - zlim[0]) * nbz)))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in bins.get(((b[0] + dx) % nbx, (b[1] + dy) % nby, b[2] + dz), ()):
                        d = p - out[q]
                        d[0] -= nx * np.floor(d[0] / nx + 0.5)
                        d[1] -= ny * np.floor(d[1] / ny + 0.5)
                        if d @ d <= dmin * dmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out[k] = p
            bins.setdefault(b, []).append(k)
            k += 1
    return out


def bead_stage(nx: int = 512, ny: int = 256, nz: int = 128, *, n: int = 16384, a: float = 1.5, chi: float = 4.0,
               sigma: float = 1.0, bias: float = 0.5, sheet_gap: float = 6.0, eta: float = 0.1, dt: float = 0.012,
               rep: Tuple[float, float, float] = (0.5, 2.0, 1.0), seed: int = 0,
               xband: Optional[Tuple[float, float]] = None, sheets: bool = True) -> BeadStage:
    """Beads between two charge sheets above and below the channel with
    opposite charge (bottom +sigma, top -sigma: the field inside points
    along +z), each 1/8 of the channel wider than it on every side, plus a
    bias field along +z.  eta is the lattice fluid's dynamic viscosity at
    tau = 0.8 ((tau - 1/2)/3).  rep balances the contact attraction of two
    beads in the mid-channel field (about 8 force units) at a surface gap of
    about 0.5; dt keeps the explicit overdamped update stable for a chain:
    its fastest mode has stiffness 4k (k = n (n + 1) A g^-(n+2) at that gap,
    about 44), and mobility * 4k = dt/(6 pi eta a) * 176 is about 0.75,
    well below 2.
    Defaults: the 512 x 256 x 128 channel with 16384 beads of radius 1.5
    (about 1.4 % volume fraction).  xband limits the beads to a band of x
    (a filter section of the channel); sheets=False leaves the bias field
    alone (its field then equals the mid-channel one only roughly)."""
    rng = np.random.default_rng(seed)
    zlo, zhi = 0.5 + a + 0.5, nz - 1.5 - a - 0.5
    x = place_beads(rng, n, a, (nx, ny, nz), (zlo, zhi), 1.0, xband)
    mx, my = nx / 8, ny / 8
    sh = np.array([[0.5 - sheet_gap, -mx, nx + mx, -my, ny + my, sigma],
                   [nz - 1.5 + sheet_gap, -mx, nx + mx, -my, ny + my, -sigma]]) if sheets else np.zeros((0, 6))
    return BeadStage(x=x, sheets=sh, bias=(0.0, 0.0, bias), a=a, chi=chi, eta=eta, dt=dt, rep=tuple(rep),
                     dims=(nx, ny, nz), periodic=(1, 1, 0), walls_z=True,
                     meta=dict(seed=seed, sigma=sigma if sheets else 0.0, bias=bias, sheet_gap=sheet_gap, xband=xband))


def chain_filter_inputs(nx: int = 512, ny: int = 256, nz: int = 128, *, nbeads: int = 4096,
                        band: Tuple[float, float] = (192.0, 320.0), ncells: int = 400, cell_radius: float = 4.0,
                        level: int = 3, seed: int = 5) -> Tuple[BeadStage, Cells]:
    """Inputs of the staged filter run at the throughput channel's size:
    beads in a band of x between the charge sheets (they form the chains of
    the filter), and cells (642 vertices, tumour-cell moduli) seeded
    upstream of the band, at least 16 lattice units from it."""
    st = bead_stage(nx, ny, nz, n=nbeads, seed=seed, xband=band)
    rng = np.random.default_rng(seed + 1)
    cen = place_cells(rng, ncells, cell_radius, (int(band[0]) - 16, ny, nz))
    return st, make_cells(cen, cell_radius, level, MODULI_CTC)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n rotation matrices, uniform over the rotation group (QR of Gaussian
    matrices with the sign fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    q = q * np.sign(np.diagonal(r, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def red_cell_suspension(nx: int = 512, ny: int = 256, nz: int = 128, *, posts_x: int = 8, posts_y: int = 4,
                        post_radius: int = 8, gap_range=(6, 14), nred: int = 1000, red_radius: float = 5.0,
                        ntumour: int = 40, tumour_radius: float = 10.0, level: int = 3, tau: float = 0.7,
                        gx: float = 1e-5, steps: int = 1000, seed: int = 6) -> Scenario:
    """The throughput channel (8x4 posts, gaps U{6..14}) with a suspension of
    red cells (biconcave discs of radius 5, randomly oriented, red-cell
    moduli) and tumour cells (spheres of radius 10, tumour-cell moduli), all
    642 vertices, neo-Hookean stretching, membrane mass 8 (the red cells'
    stability bound); placed by random sequential addition of bounding
    spheres, tumour cells first, 1 LU apart and clear of posts and walls."""
    rng = np.random.default_rng(seed)
    mask = channel_mask(nx, ny, nz)
    gx_ = rng.integers(gap_range[0], gap_range[1] + 1, size=posts_x - 1)
    gy_ = rng.integers(gap_range[0], gap_range[1] + 1, size=posts_y - 1)
    posts = post_array_centres(nx, ny, gx_, gy_, post_radius)
    add_posts(mask, posts, post_radius)
    radii = np.concatenate([np.full(ntumour, tumour_radius), np.full(nred, red_radius)])
    placed: List[np.ndarray] = []
    prad: List[float] = []
    pc = np.asarray(posts, np.float64).reshape(-1, 2)
    for r in radii:
        for _ in range(200000):
            p = np.array([rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0.5 + r + 1.0, nz - 1.5 - r - 1.0)])
            if len(pc):
                d = pc - p[:2]
                d -= np.array([nx, ny]) * np.floor(d / [nx, ny] + 0.5)
                if (np.hypot(d[:, 0], d[:, 1]) < post_radius + 0.5 + r + 1.0).any():
                    continue
            if placed:
                d = np.asarray(placed) - p
                d[:, 0] -= nx * np.floor(d[:, 0] / nx + 0.5)
                d[:, 1] -= ny * np.floor(d[:, 1] / ny + 0.5)
                if (np.linalg.norm(d, axis=1) < np.asarray(prad) + r + 1.0).any():
                    continue
            placed.append(p)
            prad.append(r)
            break
        else:
            raise RuntimeError(f"could only place {len(placed)} of {len(radii)} cells")
    cen = np.asarray(placed)
    tum = make_cells(cen[:ntumour], tumour_radius, level, MODULI_CTC, stretch_law=1, mass=MASS_RBC)
    red = make_cells(cen[ntumour:], red_radius, level, MODULI_RBC, shape="rbc", stretch_law=1, mass=MASS_RBC,
                     rotations=random_rotations(rng, nred))
    cells = concat_cells([tum, red])
    return Scenario("red_cells", nx, ny, nz, tau, (gx, 0.0, 0.0), mask, steps, cells=cells,
                    meta=dict(post_centres=posts, post_radius=post_radius, seed=seed, nred=nred, ntumour=ntumour))
