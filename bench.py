#!/usr/bin/env python3
"""Benchmark of the D3Q19 + immersed-boundary step on one MI355X.

One "step" is one full coupled step of the hot path: membrane forces, IBM
interpolation/coupling/spreading/point update, and the fused collide-stream
of the whole lattice.  The default workload is the throughput channel:
512x256x128 lattice, 8x4 posts (gaps U{6..14}), 400 cells of 642 vertices,
tau 0.7, FP32 deviation storage.  A second leg times the batched form: the
64-channel gap sweep as one batch against the same channels run one after
another; a third the differentiation form: a checkpointed 300-step run and
its backward pass against the plain forward run; a fourth the cost of the
contact forces (collisions) on the main workload; a fifth the minimum-gap
experiment (gap ladders of tumour and red cells, run until each cell has
passed or stalled); then the magnetic bead stage, the staged filter run
through frozen bead chains and a red-cell suspension.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
LAUNCH_SAMPLES = 40  # collide-stream launches timed by events inside the timed region (about)


def sample_stride(steps: int) -> int:
    """Odd stride between timed collide-stream launches, so that launches of
    both workgroup orders are sampled, giving about LAUNCH_SAMPLES of them (a
    sampled step runs ~25 us longer: the event records and the timed launch's
    own marker)."""
    return max(1, steps // LAUNCH_SAMPLES) | 1

# Algorithmic bytes per lattice node of one collide-stream launch: the 19
# populations read and written once (4 B each in FP32 storage, 8 B in FP64)
# plus the tile's solid and wall masks (16 B per 64-node tile, 0.25 B per
# node).  The sparse immersed-boundary force (read and cleared only on tiles
# that received spread force) is not counted, which makes the achieved
# figure conservative.
def bytes_per_node(prec: str) -> float:
    s = 8 if prec == "f64" else 4
    return 2 * 19 * s + 16 / 64


# HBM traffic of one collide-stream launch on the throughput workload, from
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled by the same
# counters on a plain copy kernel; see profiles/.  Valid only while the
# kernel source hashes to "sha".
MEASURED_TRAFFIC = {"sha": "cfef06e28d057875", "bytes_per_launch": 2.6709e9}
KERNEL_SOURCES = ["paper_1110_0995_amd/csrc/lattice_kernels.hpp", "paper_1110_0995_amd/csrc/d3q19.hpp"]


def whole_step(lattice_bytes: float, ms_step: float) -> dict:
    """The collide-stream's algorithmic bytes over the time of the whole
    coupled step (membrane, IBM and lattice pass): the fraction of the HBM
    peak the step as a whole runs at.  The immersed-boundary kernels' own
    bytes are not added (a few per cent of the lattice's), so the figure is
    a slight underestimate."""
    gbs = lattice_bytes / (ms_step * 1e-3) / 1e9
    return {"bytes": int(lattice_bytes), "ms": round(ms_step, 5), "achieved": round(gbs, 1),
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name: str):
    """throughput (the default), posts_cells, poiseuille; and two references
    for the collide-stream pass alone: throughput_lattice (the throughput
    lattice with its posts and walls, no cells, so no immersed-boundary
    force) and periodic_box (the same 512x256x128 nodes, no solid node at
    all, periodic on every axis: the pass's bare access pattern)."""
    import dataclasses
    from paper_1110_0995_amd import scenario as S
    if name == "throughput":
        return S.throughput(), "f32dev"
    if name == "throughput_lattice":
        return dataclasses.replace(S.throughput(), name="throughput_lattice", cells=None), "f32dev"
    if name == "periodic_box":
        return S.Scenario("periodic_box", 512, 256, 128, 0.7, (1e-5, 0.0, 0.0), S.channel_mask(512, 256, 128, walls_z=False),
                          1000, periodic=(1, 1, 1)), "f32dev"
    if name == "posts_cells":
        return S.posts_and_cells(), "f32dev"
    if name == "poiseuille":
        return S.poiseuille(), "f64"
    raise SystemExit(f"unknown workload {name}")


def describe(s, prec):
    d = {"workload": s.name, "lattice": [s.nx, s.ny, s.nz], "nodes": s.n, "tau": s.tau, "g": list(s.g),
         "storage": prec, "fluid_fraction": round(s.fluid_fraction(), 4)}
    if s.cells is not None:
        d.update(cells=s.cells.ncells, ib_points=s.cells.nverts, triangles=s.cells.ntris)
    if "post_centres" in s.meta:
        d["posts"] = len(s.meta["post_centres"])
    return d


def cpu_baseline(s, prec, steps, err_steps, lbm_mod):
    """The FP64 oracle on the host cores: its rate is timed over the first
    ``steps`` coupled steps of the same workload; it then goes on to
    ``err_steps`` steps, where the GPU's state (same start, same number of
    steps) is compared with it."""
    import oracle
    oracle.build()
    L = oracle.Lattice.from_scenario(s)
    M = None
    X = V = None
    if s.cells is not None:
        M = oracle.Mesh(s.cells)
        X = s.cells.positions()
        M.rest_shape(X)
        V = np.zeros_like(X)
    f = L.rest()
    t0 = time.perf_counter()
    f = oracle.run(L, M, f, X, V, nsteps=steps)
    dt = time.perf_counter() - t0
    if err_steps > steps:
        f = oracle.run(L, M, f, X, V, nsteps=err_steps - steps)
    n_err = max(steps, err_steps)
    # GPU from the same start
    lat = lbm_mod.Lattice.from_scenario(s, prec=prec)
    mesh = lbm_mod.Mesh(lat, s.cells) if s.cells is not None else None
    lat.run(n_err, mesh)
    rho_g, ug = lat.fields()
    ug = ug.double().cpu().numpy()
    rho_g = rho_g.double().cpu().numpy()
    rho_o, uo = oracle.fluid_velocity(L, f)
    fl = s.solid.reshape(-1) == 0
    err = float(np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl]))
    merr = abs(float(rho_g[fl].sum()) - float(np.asarray(rho_o)[fl].sum())) / float(np.asarray(rho_o)[fl].sum())
    perr = float(np.abs(mesh.positions() - X).max()) if mesh is not None else None
    lat.close()
    return ({"value": s.n * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
             "sample": f"the first {steps} full coupled steps of the same workload in FP64 ({dt:.1f} s)"},
            {"u_rel_l2": err, "mass_rel_err": merr, "max_position_err": perr, "steps": n_err})


def batched_leg(lbm_mod, steps: int, warmup: int, cpu: bool, err_steps: int = 200) -> dict:
    """The 64-channel gap sweep stepped as one batch (one launch per kernel
    for all channels, graph-captured steps, autotuned launch shape) against
    the same 64 channels run one after another as plain single-channel
    contexts with ordinary launches.  The batch's collide-stream launch is
    timed with HIP events over eager steps after the graph-timed run."""
    import torch
    from paper_1110_0995_amd import autotune
    from paper_1110_0995_amd import scenario as S
    scs = S.gap_sweep()
    prec = "f32dev"  # FP32 storage in the deviation form (same bytes as plain FP32)
    cells, chan = S.batch_cells(scs)
    lat = lbm_mod.Lattice.batch(scs, prec=prec)
    mesh = lbm_mod.Mesh(lat, cells, chan)
    stream = torch.cuda.current_stream()
    out = {"workload": "gap_sweep", "channels": len(scs), "nodes": lat.N, "ib_points": cells.nverts,
           "cells": cells.ncells, "storage": prec, "lengths": sorted({s.nx for s in scs}), "steps": steps}
    err = None
    if cpu:
        # error of the shortest channel against the oracle after the first
        # coupled steps (they count as warm-up)
        import oracle
        k = min(range(len(scs)), key=lambda i: scs[i].n)
        s = scs[k]
        lat.run(err_steps, mesh)
        _, ug = lat.fields()
        ug = ug[:, lat.channel(k)].double().cpu().numpy()
        L = oracle.Lattice.from_scenario(s)
        M = oracle.Mesh(s.cells)
        X = s.cells.positions()
        M.rest_shape(X)
        f = oracle.run(L, M, L.rest(), X, np.zeros_like(X), nsteps=err_steps)
        _, uo = oracle.fluid_velocity(L, f)
        fl = s.solid.reshape(-1) == 0
        err = {"channel": k, "u_rel_l2": float(np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl])),
               "steps": err_steps}
    best = autotune.tune(lat, mesh)
    g = best["steps_per_graph"]
    K = max(g, steps - steps % g)
    lat.run(max(g, warmup - warmup % g), mesh, steps_per_graph=g)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    lat.run(K, mesh, steps_per_graph=g)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / K
    # the collide-stream launch alone: eager steps, its kernel's own start
    # and end (lbm_step_timed), and events recorded around the call
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ka.record(stream)  # torch creates an event at its first record
    kb.record(stream)
    cs, cs_dispatch = [], []
    for _ in range(10):
        lat.couple(mesh)
        a.record(stream)
        lat.step_timed(ka.cuda_event, kb.cuda_event)
        b.record(stream)
        torch.cuda.synchronize()
        cs.append(ka.elapsed_time(kb))
        cs_dispatch.append(a.elapsed_time(b))
    ms_cs = float(np.mean(cs))
    sums = lat.sums()
    lat.close()
    del lat, mesh
    torch.cuda.empty_cache()
    # the same channels one after another, plain contexts, ordinary launches
    runs = []
    for s in scs:
        la = lbm_mod.Lattice.from_scenario(s, prec=prec)
        ma = lbm_mod.Mesh(la, s.cells)
        la.run(2, ma)
        runs.append((la, ma))
    torch.cuda.synchronize()
    a.record(stream)
    for la, ma in runs:
        la.run(K, ma)
    b.record(stream)
    torch.cuda.synchronize()
    ms_seq = a.elapsed_time(b) / K
    for la, _ in runs:
        la.close()
    N = out["nodes"]
    bpn = bytes_per_node(prec)
    gbs = bpn * N / (ms_cs * 1e-3) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "k_collide_stream", "bytes_per_node": bpn,
                       "ms_per_launch": round(ms_cs, 5),
                       "ms_per_launch_with_dispatch": round(float(np.mean(cs_dispatch)), 5),
                       "launches_timed": len(cs), "achieved": round(gbs, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["whole_step"] = whole_step(bpn * N, ms)
    out.update(steps=K, ms_per_step=round(ms, 5), mlups=round(N / (ms * 1e-3) / 1e6, 1),
               sequential_ms_per_step=round(ms_seq, 5), sequential_mlups=round(N / (ms_seq * 1e-3) / 1e6, 1),
               speedup=round(ms_seq / ms, 3), launch=best, mass=sums[0])
    if err is not None:
        out["error_vs_oracle"] = err
    return out


def adjoint_leg(lbm_mod) -> dict:
    """The differentiation form on the adjoint workload (128x64x32, 3 cells,
    300 steps, checkpoints every 20): the plain forward run against the
    checkpointed forward plus the backward (segment recompute + reverse
    kernels).  The gradient of the objective along the 16 seeded directions
    of G is compared with the FP64 oracle's central differences stored by
    tests/golden/make_adjoint_fd.py."""
    import torch
    from paper_1110_0995_amd import adjoint
    from paper_1110_0995_amd import scenario as S
    s = S.adjoint_channel()
    every = s.meta["checkpoint_every"]
    prec = "f32dev"
    lat = lbm_mod.Lattice.from_scenario(s, prec=prec)
    mesh = lbm_mod.Mesh(lat, s.cells)
    x0 = mesh.x.clone()
    start = [t.clone() for t in (lat.current_buffer(), mesh.x, mesh.v)]
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def reset():
        lat.current_buffer().copy_(start[0])
        mesh.x.copy_(start[1])
        mesh.v.copy_(start[2])

    spg = every - every % 2  # the plain run takes graphs of the same length as the checkpointed one
    lat.run(s.steps, mesh, steps_per_graph=spg)  # warm-up and capture
    reset()
    torch.cuda.synchronize()
    ev[0].record(stream)
    lat.run(s.steps, mesh, steps_per_graph=spg)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t_plain = ev[0].elapsed_time(ev[1])
    t_first = None
    for rep in range(2):  # the first pass captures the graphs; the second is timed
        reset()
        G = torch.zeros(3, s.n, dtype=lat.rdtype, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        ev[0].record(stream)
        fT, xT, vT = adjoint.run_with_grad(G, lat, mesh, s.steps, every)
        ev[1].record(stream)
        J = adjoint.objective(lat, mesh, fT, xT, G, x0)
        ev[2].record(stream)
        J.backward()
        ev[3].record(stream)
        torch.cuda.synchronize()
        t_fwd = ev[0].elapsed_time(ev[1])
        t_bwd = ev[2].elapsed_time(ev[3])
        if rep == 0:
            t_first = t_fwd + t_bwd
    out = {"workload": "adjoint_channel", "lattice": [s.nx, s.ny, s.nz], "nodes": s.n, "steps": s.steps,
           "checkpoint_every": every, "ib_points": s.cells.nverts, "storage": prec,
           "plain_forward_ms": round(t_plain, 3), "checkpointed_forward_ms": round(t_fwd, 3),
           "backward_ms": round(t_bwd, 3), "backward_over_forward": round(t_bwd / t_plain, 3),
           "first_pass_ms_with_graph_capture": round(t_first, 3),
           "total_over_forward": round((t_fwd + t_bwd) / t_plain, 3),
           "forward_mlups": round(s.n * s.steps / (t_plain * 1e-3) / 1e6, 1)}
    gold_path = os.path.join(ROOT, "tests", "golden", "adjoint_fd.json")
    if os.path.exists(gold_path):
        with open(gold_path) as fh:
            gold = json.load(fh)
        dirs = S.random_directions(s, len(gold["fd"]))
        g = G.grad.double().cpu().numpy().reshape(3, s.nz, s.ny, s.nx)
        xa, xb = s.meta["design_x"]
        ad = np.array([float((g[..., xa:xb] * d).sum()) for d in dirs])
        fd = np.array(gold["fd"])
        out["error_vs_oracle"] = {"max_rel_dir_err": float(np.max(np.abs(ad - fd) / np.abs(fd))),
                                  "directions": len(fd), "J_rel_err": abs(float(J.item()) - gold["J0"]) / abs(gold["J0"])}
    lat.close()
    return out


def contact_leg(lbm_mod, steps: int) -> dict:
    """The throughput workload with the contact forces of the collisions
    (soft-sphere repulsion between cells and from the walls and posts)
    switched on, against the same steps without them."""
    import torch
    from paper_1110_0995_amd import scenario as S
    s = S.throughput()
    out = {"workload": "throughput + contact", "steps": steps, "law": {k: S.CONTACT[k] for k in
                                                                      ("a", "n", "rcut", "roff", "dmin")}}
    stream = torch.cuda.current_stream()
    for name, contact in (("without", None), ("with", S.contact_params(s))):
        lat = lbm_mod.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm_mod.Mesh(lat, s.cells, contact=contact)
        lat.run(20, mesh, steps_per_graph=10)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        lat.run(steps, mesh, steps_per_graph=10)
        b.record(stream)
        torch.cuda.synchronize()
        out[f"ms_per_step_{name}"] = round(a.elapsed_time(b) / steps, 5)
        lat.close()
        del lat, mesh
        torch.cuda.empty_cache()
    out["overhead"] = round(out["ms_per_step_with"] / out["ms_per_step_without"] - 1.0, 4)
    return out


LADDER_GAPS = {"tumour": range(2, 17), "red": range(1, 9)}


def sweep_leg(lbm_mod, max_steps: int, drivings=(5e-5, 2.5e-5)) -> dict:
    """The minimum-gap experiment of Sec. 3 as gap ladders: one channel per
    gap (1 LU = 1 um steps; tumour cells 2..16, red cells 1..8), closed across
    its width except for the opening, one Table 1 cell centred on the
    opening; both ladders stepped as one batch with the contact forces
    until every cell has passed the posts or stalled in front of them.
    Reports per cell type the pass / stall curve and the smallest passing
    gap, for each driving body force (the physical calibration of the
    paper's 460 um/s is not available, so the result is given against the
    driving)."""
    import torch
    from paper_1110_0995_amd import scenario as S
    from paper_1110_0995_amd import sweep
    out = {"workload": "gap ladders 80x32x24 per channel, 1 cell per channel, contact, f32dev",
           "gaps": {k: [min(v), max(v)] for k, v in LADDER_GAPS.items()}, "max_steps": max_steps,
           "check_every": 250, "stall": "centroid advanced < 0.05 LU over 2000 steps, after 2000 steps",
           "runs": []}
    for gx in drivings:
        scs = [s for cell, gaps in LADDER_GAPS.items() for s in S.gap_ladder(cell, gaps, gx=gx)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = sweep.run_ladder(lbm_mod, scs, max_steps, check_every=250)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        nodes = sum(s.n for s in scs)
        summ = sweep.ladder_summary(tr.results())
        out["runs"].append({"gx": gx, "channels": len(scs), "steps_run": tr.steps_run, "stopped": tr.stopped,
                            "wall_s": round(dt, 3),
                            "mlups_incl_setup_and_tracking": round(nodes * tr.steps_run / dt / 1e6, 1),
                            "per_type": {cell: {k: d[k] for k in ("gaps", "outcome", "steps", "monotone",
                                                                  "min_passing_gap", "max_stalling_gap",
                                                                  "undecided", "non_finite")}
                                         for cell, d in summ.items()}})
    return out


# FP64 operations of one dipole pair (Eq. interaction) plus the repulsion
# test, counting a square root or a division as one: separation 3, |r|^2 5,
# |r| 1, 3/(4 pi |r|^5) 3, the three dot products 15, 5 (m1.r)(m2.r)/|r|^2 3,
# the bracket and scale 19, accumulation 3, surface gap 1
FLOPS_PER_PAIR = 53
FP64_VECTOR_PEAK_TFLOPS = 78.6


def magnet_executed_flops(n: int, periodic_axes: int) -> float:
    """FP64 operations the pair kernel issues for n beads: it splits the
    beads into blocks of 64 w (w waves per workgroup, the largest of 4, 2
    giving at least 2048 block pairs, else 1); a diagonal block evaluates all
    c^2 ordered pairs of its c beads (the bead with itself masked, not
    skipped), an off-diagonal block pair each unordered pair once, adding
    the reaction to the partner's sum (3 more).  Each evaluation also does the
    minimum image on the periodic axes (a product and a fused multiply-add,
    3 per axis)."""
    w = 1
    for cand in (4, 2):
        nb = -(-n // (64 * cand))
        if nb * (nb + 1) // 2 >= 2048:
            w = cand
            break
    B = 64 * w
    sizes = [min(B, n - i) for i in range(0, n, B)]
    diag = sum(c * c for c in sizes)
    off = (n * n - diag) // 2
    per = 3 * periodic_axes
    return float(off * (FLOPS_PER_PAIR + 3 + per) + diag * (FLOPS_PER_PAIR + per))


def magnet_leg(steps: int) -> dict:
    """The magnetic bead stage (Sec. 2.5): 16384 beads between two charge
    sheets in the 512 x 256 x 128 channel, FP64, all-pairs dipole
    interaction; the chains it forms are then fixed into the solid mask
    (timed separately)."""
    import torch
    from paper_1110_0995_amd import magnet
    from paper_1110_0995_amd import scenario as S
    st = S.bead_stage()
    b = magnet.Beads(st)
    stream = torch.cuda.current_stream()
    b.run(20)
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    b.run(steps)
    a1.record(stream)
    torch.cuda.synchronize()
    ms = a0.elapsed_time(a1) / steps
    solid = torch.zeros(st.dims[0] * st.dims[1] * st.dims[2], dtype=torch.uint8, device="cuda")
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    b.freeze(solid)
    f1.record(stream)
    torch.cuda.synchronize()
    x = b.positions()
    pairs = st.n * (st.n - 1)
    tflops = pairs * FLOPS_PER_PAIR / (ms * 1e-3) / 1e12
    exe = magnet_executed_flops(st.n, int(sum(st.periodic))) / (ms * 1e-3) / 1e12
    return {"workload": "bead_stage 512x256x128, 16384 beads a=1.5, 2 sheets + bias, f64", "steps": steps,
            "ms_per_step": round(ms, 5), "pair_interactions_per_s": round(pairs / (ms * 1e-3), 1),
            "definition_equivalent": {
                "what": "n(n-1) ordered pairs x 53 FP64 ops over the whole step (the all-pairs sum as written)",
                "tflops": round(tflops, 2), "frac_of_fp64_vector_peak": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4)},
            "executed": {
                "what": "FP64 ops the pair kernel issues (each unordered pair once + reaction, diagonal blocks "
                        "all c^2, minimum image) over the whole step",
                "tflops": round(exe, 2), "frac_of_fp64_vector_peak": round(exe / FP64_VECTOR_PEAK_TFLOPS, 4)},
            "flops_per_pair": FLOPS_PER_PAIR, "freeze_ms": round(f0.elapsed_time(f1), 4),
            "solid_fraction_after_freeze": round(float(solid.float().mean().item()), 5),
            "finite": bool(np.isfinite(x).all())}


def chain_filter_leg(bead_steps: int, steps: int) -> dict:
    """The staged filter run at the throughput channel's size: the bead
    stage (4096 beads in a band between the sheets) forms chains, they are
    fixed into the solid mask and as contact spheres, then 400 cells and the
    fluid run through them (FP32 deviation storage); the coupled steps are
    timed with and without the contact forces."""
    import torch
    from paper_1110_0995_amd import lbm, pipeline
    from paper_1110_0995_amd import scenario as S
    st, cells = S.chain_filter_inputs()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cf = pipeline.chain_filter(st, bead_steps, cells, gx=1e-5, steps=steps)
    torch.cuda.synchronize()
    stage_s = time.perf_counter() - t0
    s = cf.scenario
    out = {"workload": "chain_filter 512x256x128, 4096 beads in x [192, 320), 400 cells x 642 vertices, f32dev",
           "bead_steps": bead_steps, "stage_and_freeze_s": round(stage_s, 3), "steps": steps,
           "solid_fraction": round(float(s.solid.mean()), 5), "spheres": len(cf.beads)}
    stream = torch.cuda.current_stream()
    for name, contact in (("without", None), ("with", cf.contact)):
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm.Mesh(lat, cells, contact=contact)
        lat.run(20, mesh, steps_per_graph=10)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        lat.run(steps, mesh, steps_per_graph=10)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[f"ms_per_step_{name}_contact"] = round(ms, 5)
        out[f"mlups_{name}_contact"] = round(s.n / (ms * 1e-3) / 1e6, 1)
        out[f"finite_{name}_contact"] = bool(np.isfinite(mesh.positions()).all())
        lat.close()
        del lat, mesh
        torch.cuda.empty_cache()
    return out


def red_cells_leg(steps: int) -> dict:
    """Red blood cells in the throughput channel: 1000 randomly oriented
    biconcave discs (red-cell moduli) and 40 tumour cells, 642 vertices each,
    neo-Hookean stretching, contact forces on, FP32 deviation storage; the
    same cells with the linear stretching law for comparison."""
    import dataclasses
    import torch
    from paper_1110_0995_amd import lbm
    from paper_1110_0995_amd import scenario as S
    s = S.red_cell_suspension()
    out = {"workload": "red_cells 512x256x128, 1000 red + 40 tumour cells x 642 vertices, neo-Hookean, contact, "
                       "f32dev", "ib_points": int(s.cells.nverts), "steps": steps}
    stream = torch.cuda.current_stream()
    for name, law in (("neo_hookean", 1), ("linear", 0)):
        cells = dataclasses.replace(s.cells, stretch_law=law)
        lat = lbm.Lattice.from_scenario(s, prec="f32dev")
        mesh = lbm.Mesh(lat, cells, contact=S.contact_params(s))
        lat.run(20, mesh, steps_per_graph=10)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        lat.run(steps, mesh, steps_per_graph=10)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        out[f"ms_per_step_{name}"] = round(ms, 5)
        out[f"mlups_{name}"] = round(s.n / (ms * 1e-3) / 1e6, 1)
        out[f"finite_{name}"] = bool(np.isfinite(mesh.positions()).all())
        lat.close()
        del lat, mesh
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="throughput")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps timed for the CPU baseline")
    ap.add_argument("--error-steps", type=int, default=100,
                    help="coupled steps after which the GPU state is compared with the oracle's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000,
                    help="steps of the 64-channel gap sweep, batched and sequential (0 skips the leg)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-vs-forward leg")
    ap.add_argument("--sweep-steps", type=int, default=40000,
                    help="most steps of the gap-ladder runs (0 skips the leg); they stop once every cell is decided")
    ap.add_argument("--contact-steps", type=int, default=100,
                    help="steps of the throughput workload with and without contact forces (0 skips the leg)")
    ap.add_argument("--magnet-steps", type=int, default=200,
                    help="steps of the magnetic bead stage, 16384 beads (0 skips the leg)")
    ap.add_argument("--chain-filter-steps", type=int, default=100,
                    help="coupled steps of the staged filter run through frozen bead chains (0 skips the leg)")
    ap.add_argument("--red-cells-steps", type=int, default=100,
                    help="coupled steps of the red-cell suspension, neo-Hookean and linear (0 skips the leg)")
    ap.add_argument("--node-records", type=int, default=0, choices=(0, 1),
                    help="1: stencil-node velocities from the records of the collide-stream pass; 0: the lattice gather")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (reference kernel for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1110_0995_amd import lbm

    s, prec = make_workload(args.workload)
    lat = lbm.Lattice.from_scenario(s, prec=prec)
    lat.set_node_records(args.node_records)
    mesh = lbm.Mesh(lat, s.cells) if s.cells is not None else None
    stream = torch.cuda.current_stream()

    def one_step():
        if mesh is not None:
            lat.couple(mesh)
        lat.step(1)

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()

    # timed region: K whole steps.  Every sample_stride(K)-th
    # collide-stream launch goes through lbm_step_timed, which hands the
    # kernel a pair of HIP events that the runtime sets to the kernel's own
    # start and end (its duration, as the kernel trace has it); events
    # recorded around the same call on the stream the library enqueues on
    # (torch's current stream) also take in the dispatch gaps.  Each record
    # opens a gap of a few microseconds between the kernels around it, which
    # the other steps are spared.
    every = sample_stride(args.steps)
    sampled = range(0, args.steps, every)
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in sampled}
    kev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in sampled}
    for pair in kev.values():  # torch creates an event at its first record
        for e in pair:
            e.record(stream)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for k in range(args.steps):
        if mesh is not None:
            lat.couple(mesh)
        e = ev.get(k)
        if e:
            e[0].record(stream)
            lat.step_timed(kev[k][0].cuda_event, kev[k][1].cuda_event)
            e[1].record(stream)
        else:
            lat.step(1)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    ms_cs = float(np.mean([a.elapsed_time(b) for a, b in kev.values()]))
    ms_bracket = float(np.mean([a.elapsed_time(b) for a, b in ev.values()]))
    sums = lat.sums()

    mlups = s.n * args.steps / (ms_total * 1e-3) / 1e6
    nfluid = int((s.solid == 0).sum())
    bpn = bytes_per_node(prec)
    achieved = bpn * s.n / (ms_cs * 1e-3) / 1e9
    sha = kernel_sha()
    traffic = MEASURED_TRAFFIC["bytes_per_launch"] if MEASURED_TRAFFIC["sha"] == sha else None

    out = {
        "metric": "D3Q19+IBM MLUPS & % HBM peak; batched sweep and adjoint vs plain",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "f64" else "f32",
        "precision": ("FP64 throughout" if prec == "f64" else
                      "lattice populations stored as FP32 deviations from the weights, collision in FP32; global "
                      "sums FP64; IB point positions, velocities, membrane geometry and elastic forces FP64"),
        "data": "synthetic",
        "config": describe(s, prec),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "B/launch",
                     "kernel": "k_collide_stream", "bytes_per_node": bpn, "ms_per_launch": round(ms_cs, 5),
                     "ms_per_launch_with_dispatch": round(ms_bracket, 5), "launches_timed": len(ev),
                     "kernel_sha": sha},
        "whole_step": whole_step(bpn * s.n, ms_step),
        "fluid_mlups": round(nfluid * args.steps / (ms_total * 1e-3) / 1e6, 1),
        "ibm_ms_per_step": round(ms_step - ms_cs, 5) if mesh is not None else 0.0,
        "mass": sums[0],
    }
    if not args.no_cpu_baseline:
        cb, perr = cpu_baseline(s, prec, args.cpu_steps, args.error_steps, lbm)
        out["cpu_baseline"] = cb
        out["error_vs_oracle"] = perr
    lat.close()
    del lat, mesh
    torch.cuda.empty_cache()
    if args.batched_steps > 0:
        out["batched"] = batched_leg(lbm, args.batched_steps, 20, not args.no_cpu_baseline)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(lbm)
    if args.contact_steps > 0:
        out["contact"] = contact_leg(lbm, args.contact_steps)
    if args.sweep_steps > 0:
        out["sweep"] = sweep_leg(lbm, args.sweep_steps)
    if args.magnet_steps > 0:
        out["magnet"] = magnet_leg(args.magnet_steps)
    if args.chain_filter_steps > 0:
        out["chain_filter"] = chain_filter_leg(5000, args.chain_filter_steps)
    if args.red_cells_steps > 0:
        out["red_cells"] = red_cells_leg(args.red_cells_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
