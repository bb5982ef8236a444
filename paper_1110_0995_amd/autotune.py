"""Launch-shape autotuner for a lattice (one channel or a batch).

Three knobs change speed but never results (the kernels compute the same
values in the same order whatever the launch shape):
  - collide_waves_per_block: 64-node tiles per collide-stream workgroup
    (0: whole x rows of one channel per workgroup, the row groups chosen
    per channel length);
  - list_blocks: workgroups of the kernels that walk the list of tiles
    under a membrane stencil (0 = sized from the lattice);
  - steps_per_graph: coupled steps captured in one HIP graph launch.

The search is coordinate-wise (waves, then list workgroups, then graph
length), timing a few coupled steps per candidate with device events.  The
lattice and mesh state is saved before and restored after, so tuning
leaves the simulation where it was (only the library's step counter
advances).  Results are cached in a JSON file keyed by the batch shape.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional

import torch

WAVES = (0, 1, 2, 4, 8)
LIST_BLOCKS = (0, 256, 1024, 4096)
GRAPH_STEPS = (2, 10, 50)


def signature(lat, mesh) -> str:
    """Key of a tuning result: library build, device, precision, channel
    sizes, mesh counts."""
    from . import _lib
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as fh:
        h.update(hashlib.sha256(fh.read()).digest())
    h.update(torch.cuda.get_device_name(lat.device).encode())
    h.update(lat.prec.encode())
    h.update(json.dumps(lat.channels).encode())
    if mesh is not None:
        c = mesh.cells
        h.update(json.dumps([c.ncells, c.nverts, c.ntris, c.nedges]).encode())
    return h.hexdigest()[:20]


def default_cache() -> str:
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "paper_1110_0995_amd", "launch_tuning.json")


def _time(lat, mesh, waves, blocks, graph, steps) -> float:
    lat.set_launch(waves, blocks)
    stream = torch.cuda.current_stream(lat.device)
    lat.run(graph, mesh, steps_per_graph=graph)  # capture and warm
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = max(graph, steps - steps % graph)
    a.record(stream)
    lat.run(n, mesh, steps_per_graph=graph)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / n


def tune(lat, mesh=None, steps: int = 20, cache: Optional[str] = None, force: bool = False) -> Dict[str, int]:
    """Best (collide_waves_per_block, list_blocks, steps_per_graph) for this
    lattice and mesh; applies the launch shape and returns it with the
    measured ms per step."""
    path = cache or default_cache()
    key = signature(lat, mesh)
    table = {}
    if os.path.exists(path):
        try:
            with open(path) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
    if key in table and not force:
        best = table[key]
        lat.set_launch(best["collide_waves_per_block"], best["list_blocks"])
        return best
    saved = [t.clone() for t in (lat.f_a, lat.f_b)]
    msaved = [t.clone() for t in (mesh.x, mesh.v, mesh.f_el)] if mesh is not None else []
    # even step counts only: the state buffers end where they started
    w, lb, g = 0, 0, 10
    ms = {}
    for cand in WAVES:
        ms[("w", cand)] = _time(lat, mesh, cand, lb, g, steps)
    w = min(WAVES, key=lambda c: ms[("w", c)])
    if mesh is not None:
        for cand in LIST_BLOCKS:
            ms[("l", cand)] = _time(lat, mesh, w, cand, g, steps)
        lb = min(LIST_BLOCKS, key=lambda c: ms[("l", c)])
    for cand in GRAPH_STEPS:
        ms[("g", cand)] = _time(lat, mesh, w, lb, cand, max(steps, cand))
    g = min(GRAPH_STEPS, key=lambda c: ms[("g", c)])
    torch.cuda.synchronize(lat.device)
    for dst, src in zip((lat.f_a, lat.f_b), saved):
        dst.copy_(src)
    if mesh is not None:
        for dst, src in zip((mesh.x, mesh.v, mesh.f_el), msaved):
            dst.copy_(src)
    torch.cuda.synchronize(lat.device)
    best = {"collide_waves_per_block": w, "list_blocks": lb, "steps_per_graph": g,
            "ms_per_step": round(ms[("g", g)], 5)}
    lat.set_launch(w, lb)
    table[key] = best
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    except OSError:
        pass  # a read-only cache location only costs a re-tune next time
    return best
