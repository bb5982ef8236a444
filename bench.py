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
contact forces (collisions) on the main workload; a fifth the gap pass /
no-pass sweep with those forces.  Prints ONE JSON line.
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
LAUNCH_SAMPLE_EVERY = 5  # collide-stream launches bracketed by HIP events: every 5th step

# Algorithmic bytes per lattice node of one collide-stream launch: the 19
# populations read and written once (4 B each in FP32 storage, 8 B in FP64)
# plus the 1-byte node class.  The sparse immersed-boundary force (read and
# cleared only on tiles that received spread force) is not counted, which
# makes the achieved figure conservative.
def bytes_per_node(prec: str) -> int:
    s = 8 if prec == "f64" else 4
    return 2 * 19 * s + 1


# HBM traffic of one collide-stream launch on the throughput workload, from
# two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) scaled by the same
# counters on a plain copy kernel; see profiles/.  Valid only while the
# kernel source hashes to "sha".
MEASURED_TRAFFIC = {"sha": "347e02d5cf2a226b", "bytes_per_launch": 2.6229e9}
KERNEL_SOURCES = ["paper_1110_0995_amd/csrc/lattice_kernels.hpp", "paper_1110_0995_amd/csrc/d3q19.hpp"]


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name: str):
    from paper_1110_0995_amd import scenario as S
    if name == "throughput":
        return S.throughput(), "f32dev"
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


def cpu_baseline(s, prec, steps, lbm_mod):
    """The FP64 oracle on the host cores for a bounded number of steps of the
    same workload; also the GPU's error against it after those steps."""
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
    oracle.run(L, M, f, X, V, nsteps=steps)
    dt = time.perf_counter() - t0
    # GPU from the same start
    lat = lbm_mod.Lattice.from_scenario(s, prec=prec)
    mesh = lbm_mod.Mesh(lat, s.cells) if s.cells is not None else None
    lat.run(steps, mesh)
    _, ug = lat.fields()
    ug = ug.double().cpu().numpy()
    _, uo = oracle.fluid_velocity(L, f)
    fl = s.solid.reshape(-1) == 0
    err = float(np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl]))
    perr = float(np.abs(mesh.positions() - X).max()) if mesh is not None else None
    lat.close()
    return ({"value": s.n * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
             "sample": f"{steps} full coupled steps of the same workload in FP64 ({dt:.1f} s)"},
            {"u_rel_l2": err, "max_position_err": perr, "steps": steps})


def batched_leg(lbm_mod, steps: int, warmup: int, cpu: bool) -> dict:
    """The 64-channel gap sweep stepped as one batch (one launch per kernel
    for all channels, graph-captured steps, autotuned launch shape) against
    the same 64 channels run one after another as plain single-channel
    contexts with ordinary launches."""
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
        lat.run(4, mesh)
        _, ug = lat.fields()
        ug = ug[:, lat.channel(k)].double().cpu().numpy()
        L = oracle.Lattice.from_scenario(s)
        M = oracle.Mesh(s.cells)
        X = s.cells.positions()
        M.rest_shape(X)
        f = oracle.run(L, M, L.rest(), X, np.zeros_like(X), nsteps=4)
        _, uo = oracle.fluid_velocity(L, f)
        fl = s.solid.reshape(-1) == 0
        err = {"channel": k, "u_rel_l2": float(np.linalg.norm(ug[:, fl] - uo[:, fl]) / np.linalg.norm(uo[:, fl])),
               "steps": 4}
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


def sweep_leg(lbm_mod, steps: int) -> dict:
    """The gap pass / no-pass experiment on the 64-channel sweep: the batch
    stepped with the contact forces of the collisions, every cell tracked
    through its channel's post pair; reports the gaps passed, the smallest
    one, and the wall-clock rate including the tracking."""
    import torch
    from paper_1110_0995_amd import scenario as S
    from paper_1110_0995_amd import sweep
    scs = S.gap_sweep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr = sweep.run_sweep(lbm_mod, scs, steps, check_every=100)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    summ = tr.summary()
    nodes = sum(s.n for s in scs)
    return {"workload": "gap_sweep + contact", "channels": len(scs), "steps": steps, "check_every": 100,
            "wall_s": round(dt, 3), "mlups_incl_setup_and_tracking": round(nodes * steps / dt / 1e6, 1),
            "gaps": sorted({r["gap"] for r in summ}),
            "passed_gaps": sorted({r["gap"] for r in summ if r["passed"]}),
            "through": sum(r["through"] for r in summ), "around": sum(r["around"] for r in summ),
            "min_passing_gap": tr.min_passing_gap()}


# FP64 operations of one dipole pair (Eq. interaction) plus the repulsion
# test, counting a square root or a division as one: separation 3, |r|^2 5,
# |r| 1, 3/(4 pi |r|^5) 3, the three dot products 15, 5 (m1.r)(m2.r)/|r|^2 3,
# the bracket and scale 19, accumulation 3, surface gap 1
FLOPS_PER_PAIR = 53
FP64_VECTOR_PEAK_TFLOPS = 78.6


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
    return {"workload": "bead_stage 512x256x128, 16384 beads a=1.5, 2 sheets + bias, f64", "steps": steps,
            "ms_per_step": round(ms, 5), "pair_interactions_per_s": round(pairs / (ms * 1e-3), 1),
            "fp64_tflops_step": round(tflops, 2), "frac_of_fp64_vector_peak": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4),
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
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=200,
                    help="steps of the 64-channel gap sweep, batched and sequential (0 skips the leg)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-vs-forward leg")
    ap.add_argument("--sweep-steps", type=int, default=2000,
                    help="steps of the gap pass / no-pass sweep with contact forces (0 skips the leg)")
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

    # timed region: K whole steps; events bracket every LAUNCH_SAMPLE_EVERY-th
    # collide-stream launch on the stream the library enqueues on (torch's
    # current stream).  Each event record opens a gap of a few microseconds
    # between the kernels around it, which the other steps are spared; the
    # stride is odd, so launches of both workgroup orders are sampled.
    every = LAUNCH_SAMPLE_EVERY if args.steps >= 2 * LAUNCH_SAMPLE_EVERY else 1
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in range(0, args.steps, every)}
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
        lat.step(1)
        if e:
            e[1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    ms_cs = float(np.mean([a.elapsed_time(b) for a, b in ev.values()]))
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
        "data": "synthetic",
        "config": describe(s, prec),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_unit": "B/launch",
                     "kernel": "k_collide_stream", "bytes_per_node": bpn, "ms_per_launch": round(ms_cs, 5),
                     "launches_timed": len(ev),
                     "kernel_sha": sha},
        "fluid_mlups": round(nfluid * args.steps / (ms_total * 1e-3) / 1e6, 1),
        "ibm_ms_per_step": round(ms_step - ms_cs, 5) if mesh is not None else 0.0,
        "mass": sums[0],
    }
    if not args.no_cpu_baseline:
        cb, perr = cpu_baseline(s, prec, args.cpu_steps, lbm)
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
