"""The staged run of the filter (Sec. 2.5 and the list of stages that closes
it): the magnetic bead stage forms chains, the chains are fixed in space --
their beads become solid (bounce-back) nodes of the lattice and fixed
contact spheres of the collision law -- and the fluid with the cells then
runs through them.  Every step runs in the library's kernels; this module
only hands arrays from one stage to the next."""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from . import magnet
from . import scenario as S


@dataclasses.dataclass
class ChainFilter:
    scenario: S.Scenario   # lattice workload whose solid mask holds the frozen chains
    beads: np.ndarray      # frozen bead centres [n, 3]
    contact: dict          # collision law with the walls and the beads as fixed spheres


def freeze_chains(st: S.BeadStage, steps: int, device: str = "cuda"):
    """Run the bead stage for `steps` steps on the GPU, then fix the beads
    into the channel's solid mask (walls z = 0 and nz - 1).  Returns the
    bead centres [n, 3] and the mask [nz, ny, nx]."""
    nx, ny, nz = st.dims
    b = magnet.Beads(st, device=device)
    b.run(steps)
    solid = torch.as_tensor(S.channel_mask(nx, ny, nz).reshape(-1)).to(device)
    b.freeze(solid)
    return b.positions(), solid.cpu().numpy().reshape(nz, ny, nx)


def chain_filter(st: S.BeadStage, bead_steps: int, cells: Optional[S.Cells], *, tau: float = 0.8,
                 gx: float = 1e-5, steps: int = 1000, device: str = "cuda", **contact) -> ChainFilter:
    """The lattice workload of the chain filter: the bead stage's chains
    frozen into a channel of the same size, with `cells`."""
    nx, ny, nz = st.dims
    x, solid = freeze_chains(st, bead_steps, device)
    s = S.Scenario("chain_filter", nx, ny, nz, tau, (gx, 0.0, 0.0), solid, steps, cells=cells,
                   meta=dict(beads=len(x), bead_radius=st.a, bead_steps=bead_steps))
    law = S.contact_params(s, spheres=S.bead_spheres(x, st.a), **contact)
    return ChainFilter(scenario=s, beads=x, contact=law)
