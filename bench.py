#!/usr/bin/env python3
"""Throughput of the immersed-boundary lattice Boltzmann step on one MI355X.

Workload: the single-fish, accelerating-local-frame configuration -
384x192x192 D3Q27 lattice (tau = 0.6), a 12,000-marker synthetic fish on a
10-joint chain of length 96 driven by a travelling body wave, frame
acceleration a(n) = 1e-5 sin(2 pi n / 400), velocity inlet / zero-gradient
outlet. One step = skinning, tile binning, interpolation, direct forcing,
spreading, the fused collide-stream with the frame force and open faces, and
the body wrench (the whole path), all through the C interface. The headline
step is one launch (k_step_overlap): 32 workgroups take the immersed-boundary
chain (macros, interpolation, forcing, spreading, the collide of the cells
that carry an immersed force, then the next step's skinning and tile binning)
while the others stream the collide of every other cell; the "sequential"
form runs every phase in its own launch (k_collide alone).

Prints one JSON line: MLUPS (lattice updates per second / 1e6, every node
counted), the main launch's achieved bandwidth (the collide's 216 B per cell
over the launch's average duration, from HIP events on its stream) against
the 8 TB/s HBM peak, and the FP64 oracle's throughput on the host cores for a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"f32": 216, "f16": 108, "bf16": 108}
METRIC = "MLUPS and % of HBM roofline per GPU; adjoint/forward time ratio"
# The headline step runs the immersed-boundary phases in this many workgroups
# beside the collide, in one launch (k_step_overlap); 0 runs them in launches
# of their own before the collide (k_collide).
HEADLINE_IB_WORKGROUPS = 32
_CSRC = os.path.join(ROOT, "paper_2206_01683_amd", "csrc")
# the sources each main kernel is compiled from, and its committed HBM traffic summary
KERNEL_SOURCES = {
    "k_collide": [os.path.join(_CSRC, f) for f in ("lattice.hpp", "env.hpp", "fluid.hpp")],
    "k_step_overlap": [os.path.join(_CSRC, f) for f in ("lattice.hpp", "env.hpp", "fluid.hpp", "ib.hpp", "step.hpp")],
}
TRAFFIC_FILES = {
    "k_collide": os.path.join(ROOT, "profiles", "collide_traffic.txt"),
    "k_step_overlap": os.path.join(ROOT, "profiles", "step_overlap_traffic.txt"),
}


def main_kernel(ib_workgroups: int) -> str:
    return "k_step_overlap" if ib_workgroups > 0 else "k_collide"


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES[kernel]:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it is missing or was taken on other kernel source."""
    path = TRAFFIC_FILES[kernel]
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash(kernel):
        return None
    key = f"hbm_bytes_per_launch_{storage}"
    return float(vals[key]) if key in vals else None


def run_gpu(storage: str, steps: int, warmup: int, block=(0, 0), collision: int = 0, variant=None,
            ib_workgroups: int = 0):
    """The fish workload; variant (optional) edits it first (faces, frames)."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm

    w = I.fish_workload(nsteps=warmup + steps)
    if variant is not None:
        variant(w)
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=storage, max_markers=w.markers.n,
                         max_bones=w.markers.nbones, block=block, collision=collision, bc_y=w.bc_y, bc_z=w.bc_z,
                         ib_workgroups=ib_workgroups)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses, np.float32), device="cuda")
    wrench = torch.zeros((warmup + steps, 8), dtype=torch.float32, device="cuda")
    if warmup:
        sim.step(w.frames[:warmup], dm, poses[:warmup], wrench[:warmup])
    torch.cuda.synchronize()
    sim.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(w.frames[warmup:], dm, poses[warmup:], wrench[warmup:])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ib_ms, col_ms, timed = sim.profile_collect()
    status = sim.check()
    ncell = w.ncell
    mlups = ncell * steps / wall / 1e6
    col_avg_s = col_ms / 1000.0 / max(timed, 1)
    alg_bytes = BYTES_PER_CELL[storage] * ncell
    res = {
        "workload": w, "ncell": ncell, "wall": wall, "mlups": mlups, "status": status,
        "collide_avg_ms": col_avg_s * 1e3, "ib_avg_ms": ib_ms / max(timed, 1), "timed": timed,
        "collide_gbs": alg_bytes / col_avg_s / 1e9, "alg_bytes": alg_bytes,
        "wrench_last": wrench[-1].cpu().tolist(), "rows_layout": sim.rows_layout,
    }
    del sim
    torch.cuda.empty_cache()
    return res


def run_graph(storage: str, steps: int, warmup: int, block=(0, 0), ib_workgroups: int = 0):
    """The headline step loop captured into one HIP graph (through torch):
    `steps` steps per replay after an eager warm-up, then one warm-up replay
    and one timed replay, wall clock between synchronizations. An even step
    count keeps each replay on the same buffers."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm

    steps += steps & 1
    w = I.fish_workload(nsteps=warmup + steps)
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=storage, max_markers=w.markers.n,
                         max_bones=w.markers.nbones, block=block, ib_workgroups=ib_workgroups)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses, np.float32), device="cuda")
    wrench = torch.zeros((warmup + steps, 8), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    sim.set_stream(side)
    with torch.cuda.stream(side):
        if warmup:
            sim.step(w.frames[:warmup], dm, poses[:warmup], wrench[:warmup])
    side.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        sim.step(w.frames[warmup:], dm, poses[warmup:], wrench[warmup:])
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = sim.check()
    del g, sim
    torch.cuda.empty_cache()
    return {"mlups": round(w.ncell * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
            "steps_per_replay": steps, "status": status}


BATCH_GROUPS = 2  # concurrent groups of the per-phase driver


def run_batch(nenv: int, nsteps: int, seed: int = 4):
    """Batched environments: nenv fish environments of uneven sizes (seeded
    draw), nsteps steps per run, one run = one graph replay. Returns MLUPS
    per driver with autotuned tile shapes, F32 storage, and of the per-phase
    driver with FP16 and BF16 storage."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm

    envs = I.batch_workloads(count=nenv, seed=seed, nsteps=nsteps)
    b = lbm.Batch(envs, nsteps)
    shapes = b.autotune(reps=3)
    ncell = b.ncell
    out = {"envs": nenv, "steps_per_run": nsteps, "cells": ncell,
           "markers": int(sum(w.markers.n for w in envs)),
           "shapes": {f"{bx}x{by}": int(((shapes[:, 0] == bx) & (shapes[:, 1] == by)).sum())
                      for bx, by in lbm.BATCH_SHAPES}}
    def timed(b, mode, bytes_per_cell):
        b.run(nsteps, mode=mode, graph=True)  # capture + warm-up replay
        b.synchronize()
        t0 = time.perf_counter()
        b.run(nsteps, mode=mode, graph=True)
        b.synchronize()
        dt = time.perf_counter() - t0
        return {"mlups": round(ncell * nsteps / dt / 1e6, 1), "ms_per_step": round(dt * 1e3 / nsteps, 4),
                f"hbm_frac_{bytes_per_cell}B": round(ncell * nsteps * bytes_per_cell / dt / (HBM_PEAK_GBS * 1e9), 4)}

    for mode in ("persistent", "phases"):
        out[mode] = timed(b, mode, 216)
    # the per-phase driver as concurrent cell-balanced groups, one stream each
    b.set_groups(BATCH_GROUPS)
    out[f"phases_groups{BATCH_GROUPS}"] = timed(b, "phases", 216)
    out["status"] = b.check()
    b.close()
    del b
    torch.cuda.empty_cache()
    # 2-byte storage (108 B per cell), per-phase driver: same environments
    for fmt in ("f16", "bf16"):
        b = lbm.Batch(envs, nsteps, storage=fmt)
        b.autotune(reps=3)
        out[f"phases_{fmt}"] = timed(b, "phases", 108)
        b.set_groups(BATCH_GROUPS)
        out[f"phases_{fmt}_groups{BATCH_GROUPS}"] = timed(b, "phases", 108)
        out[f"phases_{fmt}"]["status"] = b.check()
        b.close()
        del b
        torch.cuda.empty_cache()
    return out


def run_two_fish(steps: int = 200, warmup: int = 20):
    """Two bodies in one lattice: the 150x50x100 two-fish domain, 2 x 2,000
    markers on 2 x 10 bones, inertial frame with inflow. MLUPS of the whole
    step and the IB share from the library's HIP events."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm

    w = I.two_fish_workload(nsteps=warmup + steps)
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=w.markers.n,
                         max_bones=w.markers.nbones, u0=w.u0.astype(np.float32))
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses, np.float32), device="cuda")
    wrench = torch.zeros((warmup + steps, 8), dtype=torch.float32, device="cuda")
    sim.step(w.frames[:warmup], dm, poses[:warmup], wrench[:warmup])
    torch.cuda.synchronize()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(w.frames[warmup:], dm, poses[warmup:], wrench[warmup:])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ib_ms, col_ms, timed = sim.profile_collect()
    status = sim.check()
    del sim
    torch.cuda.empty_cache()
    return {"workload": w.name, "markers": w.markers.n, "bones": w.markers.nbones, "steps": steps,
            "mlups": round(w.ncell * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
            "ib_ms_per_step": round(ib_ms / max(timed, 1), 5),
            "collide_GBps": round(216 * w.ncell / (col_ms / 1e3 / max(timed, 1)) / 1e9, 1), "status": status}


def run_ib_schemes(steps: int = 100, warmup: int = 10):
    """The 384x192x192 fish (12,000 markers) with each immersed-boundary
    scheme: explicit direct forcing (1 pass), multi-direct forcing (4 passes)
    and the implicit velocity correction (1 and 4 conjugate-gradient steps).
    MLUPS of the whole step and the IB share from the library's HIP events."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm

    w = I.fish_workload(nsteps=warmup + steps)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses, np.float32), device="cuda")
    out = {"workload": w.name, "markers": w.markers.n, "steps": steps}
    for name, scheme, k in (("direct_1", lbm.IB_DIRECT, 1), ("mdf_4", lbm.IB_DIRECT, 4),
                            ("implicit_1", lbm.IB_IMPLICIT, 1), ("implicit_4", lbm.IB_IMPLICIT, 4)):
        sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=w.markers.n,
                             max_bones=w.markers.nbones, u0=w.u0.astype(np.float32), mdf_iters=k, ib_scheme=scheme)
        sim.step(w.frames[:warmup], dm, poses[:warmup])
        torch.cuda.synchronize()
        sim.profile(True)
        t0 = time.perf_counter()
        sim.step(w.frames[warmup:], dm, poses[warmup:])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ib_ms, _, timed = sim.profile_collect()
        out[name] = {"mlups": round(w.ncell * steps / wall / 1e6, 1), "ms_per_step": round(wall * 1e3 / steps, 4),
                     "ib_ms_per_step": round(ib_ms / max(timed, 1), 5), "status": sim.check()}
        del sim
        torch.cuda.empty_cache()
    return out


def run_free_swimmer(steps: int = 100, warmup: int = 10):
    """Two-way coupling: the 384x192x192 fish (12,000 markers) swimming freely,
    as dense as the fluid (an artificial added mass equal to its own keeps the
    coupling stable), free yaw; each step the host body dynamics
    (lbm_swimmer_*) set the poses and the frame, the GPU runs the step, and the
    step's wrench comes back (one 32-byte device-to-host copy and a stream
    synchronization per step). Milliseconds per coupled step."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import inputs as I
    from paper_2206_01683_amd import lbm
    from paper_2206_01683_amd import swim

    w = I.fish_workload(nsteps=1)
    ms = w.markers
    n = warmup + steps
    psi, psid = I.wave_headings(96.0, 10, np.arange(n + 1))
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=ms.n, max_bones=ms.nbones)
    dm = lbm.DeviceMarkers(ms)
    sw = swim.FreeSwimmer(ms, 96.0, (160.0, 96.0, 96.0), rho_body=1.0, added_mass=1.0)
    sw.init(psi[0], psid[0])
    swim.swim(sim, dm, sw, psi[:warmup + 1], psid[:warmup + 1], warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = swim.swim(sim, dm, sw, psi[warmup:], psid[warmup:], steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    status = sim.check()
    del sim
    torch.cuda.empty_cache()
    return {"workload": w.name, "steps": steps, "ms_per_step": round(wall * 1e3 / steps, 4),
            "mlups": round(w.ncell * steps / wall / 1e6, 1), "final_velocity": [float(v) for v in out["vel"][-1]],
            "final_heading": float(out["heading"][-1]), "rho_body_over_rho_fluid": 1.0, "added_mass": 1.0,
            "status": status}


def run_adjoint(nsteps: int = 400, every: int = 20, record: bool = False):
    """Differentiation form: the 128x64x64 swimmer with 3,000 markers,
    J = time-averaged thrust over nsteps steps. Forward = the steps with a
    population checkpoint every `every` steps; backward = recompute of each
    segment into a ring of states plus one adjoint step per step, then the
    8-parameter gradient. Wall-clock of each, after one untimed pass."""
    import numpy as np
    import torch

    from paper_2206_01683_amd import adjoint as AD
    from paper_2206_01683_amd import inputs as I

    prob = AD.FinProblem(nsteps=nsteps, every=every, record=record)
    theta = np.asarray(I.C5_BASE, dtype=np.float64)
    _, tape = prob.value(theta)
    prob.pose_gradient(tape)
    del tape  # its buffers return to torch's cache for the timed pass
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, tape = prob.value(theta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pb = prob.pose_gradient(tape)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = prob.gradient(theta, tape)
    status = prob.sim.check()
    w = prob.workload
    prob.close()
    tf, tb = t1 - t0, t2 - t1
    return {"workload": w.name, "steps": nsteps, "checkpoint_every": every, "J": J,
            "grad_norm": float(np.linalg.norm(g)), "forward_ms_per_step": round(tf * 1e3 / nsteps, 4),
            "backward_ms_per_step": round(tb * 1e3 / nsteps, 4), "adjoint_over_forward": round(tb / tf, 3),
            "finite": bool(np.isfinite(pb.cpu().numpy()).all()), "status": status}


def _precision_vs_oracle(w, f_ref, prm, nsteps: int) -> dict:
    """Velocity relative L2 (non-face nodes) of the GPU after nsteps steps of
    workload w, per storage format, against the oracle's populations f_ref."""
    import numpy as np
    import torch

    import oracle
    from paper_2206_01683_amd import lbm

    _, u_ref = oracle.macros(prm, f_ref, w.frames[nsteps - 1])
    u_ref = u_ref[..., 1:-1]
    out = {"steps": nsteps, "metric": "velocity relative L2 over the non-face nodes"}
    for st in ("f32", "f16", "bf16"):
        sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=st, max_markers=w.markers.n,
                             max_bones=w.markers.nbones, rho0=np.ones((w.nz, w.ny, w.nx), np.float32),
                             u0=w.u0.astype(np.float32))
        dm = lbm.DeviceMarkers(w.markers)
        poses = torch.as_tensor(np.ascontiguousarray(w.poses[:nsteps], np.float32), device="cuda")
        sim.step(w.frames[:nsteps], dm, poses)
        _, u = sim.macros(w.frames[nsteps - 1])
        u = u.cpu().numpy().astype(np.float64)[..., 1:-1]
        out[st] = float(np.linalg.norm((u - u_ref).ravel()) / np.linalg.norm(u_ref.ravel()))
        sim.close()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(sample_steps: int):
    """The FP64 oracle as it stands, on the host cores, on the first
    sample_steps steps of the same workload (same domain, fish and frames);
    then the GPU's velocity error against that sample's end state."""
    import numpy as np

    import oracle
    from paper_2206_01683_amd import inputs as I

    w = I.fish_workload(nsteps=max(sample_steps, 2))
    prm = oracle.params(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi)
    f0 = oracle.equilibrium_field(np.ones((w.nz, w.ny, w.nx)), w.u0)
    t0 = time.perf_counter()
    ref = oracle.run(prm, f0.copy(), w.frames, w.markers, w.poses, sample_steps)
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    # one core as well: a 2-step run less a 1-step run, so that the set-up of
    # a call (buffer allocation and first touch) cancels
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.run(prm, f0.copy(), w.frames, w.markers, w.poses, 1)
    t2 = time.perf_counter()
    oracle.run(prm, f0, w.frames, w.markers, w.poses, 2)
    dt1 = (time.perf_counter() - t2) - (t2 - t1)
    oracle.set_threads(cores)
    model = None
    if os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        import psutil
        physical = psutil.cpu_count(logical=False)
    except Exception:
        physical = None
    return {"value": round(w.ncell * sample_steps / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{sample_steps} steps of the {w.nx}x{w.ny}x{w.nz} fish workload from rest "
                      f"({w.ncell * sample_steps} node updates, {dt:.1f} s, FP64)",
            "one_core_value": round(w.ncell / max(dt1, 1e-9) / 1e6, 3), "cpu_model": model,
            "openmp_threads": cores, "physical_cores_visible": physical,
            "logical_cpus_usable": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "gpu_precision_vs_oracle": _precision_vs_oracle(w, ref["f"], prm, sample_steps)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_CELL))
    ap.add_argument("--cpu-steps", type=int, default=24, help="oracle sample length (0: skip)")
    ap.add_argument("--forms",
                    default="graph,sequential,ceiling,f16,bf16,trt,faces_frames,batched,adjoint,two_fish,"
                            "free_swimmer,ib_schemes",
                    help="comma-separated extra forms to measure: graph, sequential, ceiling, f16, bf16, trt, "
                         "faces_frames, batched, adjoint, two_fish, free_swimmer, ib_schemes")
    ap.add_argument("--no-forms", action="store_true", help="measure no extra form")
    ap.add_argument("--block", type=int, nargs=2, default=(0, 0))
    ap.add_argument("--batch-envs", type=int, default=64, help="batched form: environments (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200, help="batched form: steps per graph replay")
    ap.add_argument("--ib-steps", type=int, default=100, help="ib_schemes form: timed steps per scheme")
    ap.add_argument("--ib-workgroups", type=int, default=HEADLINE_IB_WORKGROUPS,
                    help="headline step: immersed-boundary workgroups beside the collide (0: launches of their own)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); this "
              "build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    nib = max(0, args.ib_workgroups)
    kernel = main_kernel(nib)
    main_run = run_gpu(args.storage, args.steps, args.warmup, tuple(args.block), ib_workgroups=nib)
    w = main_run["workload"]
    want = set() if args.no_forms else {f.strip() for f in args.forms.split(",") if f.strip()}
    forms = {}
    if "graph" in want:
        # the headline step loop as one captured graph, replayed
        forms["graph"] = run_graph(args.storage, args.steps, args.warmup, tuple(args.block), ib_workgroups=nib)
    seq = main_run if nib == 0 else None
    if nib > 0 and want & {"sequential", "ceiling"}:
        # the same step with the immersed-boundary phases in launches of their own before the collide: the
        # collide kernel alone against the roofline and the practical ceiling
        seq = run_gpu(args.storage, args.steps, args.warmup, tuple(args.block), ib_workgroups=0)
        t = measured_traffic(args.storage, "k_collide")
        forms["sequential"] = {"mlups": round(seq["mlups"], 1), "kernel": "k_collide",
                               "collide_avg_ms": round(seq["collide_avg_ms"], 5),
                               "collide_GBps": round(seq["collide_gbs"], 1),
                               "collide_frac_of_hbm_peak": round(seq["collide_gbs"] / HBM_PEAK_GBS, 4),
                               "collide_traffic": None if t is None else round(t, 0),
                               "ib_ms_per_step": round(seq["ib_avg_ms"], 5), "status": seq["status"]}
    if "ceiling" in want:
        # the practical ceiling: reference streaming kernels on the fish's sizes
        from paper_2206_01683_amd import hbm_ceiling
        c = hbm_ceiling.measure(w.nx, w.ny, w.nz)
        # the pattern in the collide's layout, at whichever occupancy it ran
        # faster (uncapped, or three 256-cell blocks per compute unit as the F32
        # collide runs)
        if seq["rows_layout"]:
            same = max(("pull27_rows", "pull27_rows_3_blocks_per_cu"), key=lambda k: c[k]["GBps"])
        else:
            same = "pull27_planes"
        c["collide_over_pull27_same_layout"] = round(seq["collide_gbs"] / c[same]["GBps"], 4)
        c["pull27_same_layout"] = same
        c["collide_over_copy"] = round(seq["collide_gbs"] / c["copy"]["GBps"], 4)
        forms["ceiling"] = c
    if args.storage == "f32":
        for st in sorted(want & {"f16", "bf16"}):
            r = run_gpu(st, args.steps, args.warmup, tuple(args.block))
            forms[st] = {"mlups": round(r["mlups"], 1), "collide_GBps": round(r["collide_gbs"], 1),
                         "collide_frac_of_hbm_peak": round(r["collide_gbs"] / HBM_PEAK_GBS, 4),
                         "bytes_per_cell": BYTES_PER_CELL[st], "status": r["status"]}
    if "trt" in want:
        from paper_2206_01683_amd import lbm as _lbm
        r = run_gpu(args.storage, args.steps, args.warmup, tuple(args.block), collision=_lbm.COLLIDE_TRT)
        forms["trt"] = {"mlups": round(r["mlups"], 1), "collide_GBps": round(r["collide_gbs"], 1),
                        "collide_frac_of_hbm_peak": round(r["collide_gbs"] / HBM_PEAK_GBS, 4),
                        "lambda": _lbm.TRT_MAGIC, "status": r["status"]}
    if "faces_frames" in want:
        from paper_2206_01683_amd import inputs as _I

        def open_faces(w):  # far field entering through every face
            w.bc_y = (_I.BC_VELOCITY, _I.BC_VELOCITY)
            w.bc_z = (_I.BC_VELOCITY, _I.BC_VELOCITY)

        def rotating(w):  # the frame also turns about z through its origin (the fish's centre)
            w.frames[:, 3:6] = (0.0, 0.0, 2e-4)

        forms["faces_frames"] = {}
        for name, fn in (("open_faces", open_faces), ("rotating_frame", rotating)):
            r = run_gpu(args.storage, args.steps, args.warmup, tuple(args.block), variant=fn)
            forms["faces_frames"][name] = {"mlups": round(r["mlups"], 1), "collide_GBps": round(r["collide_gbs"], 1),
                                           "collide_frac_of_hbm_peak": round(r["collide_gbs"] / HBM_PEAK_GBS, 4),
                                           "ib_ms_per_step": round(r["ib_avg_ms"], 5), "status": r["status"]}
    if "batched" in want and args.batch_envs > 0:
        forms["batched"] = run_batch(args.batch_envs, args.batch_steps)
    if "adjoint" in want:
        forms["adjoint"] = run_adjoint()
        # the same run keeping every state of the horizon in HBM (lbm_adjoint_record: 400 x 56.6 MB plus the
        # IB data of every step), so that the reverse sweep recomputes nothing (lbm_adjoint_sweep)
        a1 = run_adjoint(record=True)
        forms["adjoint"]["record_every_state"] = {k: a1[k] for k in ("forward_ms_per_step", "backward_ms_per_step",
                                                                       "adjoint_over_forward", "J", "grad_norm",
                                                                       "finite", "status")}
    if "two_fish" in want:
        forms["two_fish"] = run_two_fish()
    if "free_swimmer" in want:
        forms["free_swimmer"] = run_free_swimmer()
    if "ib_schemes" in want:
        forms["ib_schemes"] = run_ib_schemes(args.ib_steps)
    traffic = measured_traffic(args.storage, kernel)
    ach = main_run["collide_gbs"]
    out = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["wall"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"fish-{w.nx}x{w.ny}x{w.nz}", "lattice": "D3Q27", "tau": w.tau,
                   "markers": w.markers.n, "bones": w.markers.nbones, "storage": args.storage,
                   "boundaries": "x: velocity inlet / zero-gradient outlet; y, z periodic",
                   "frame": "a(n) = 1e-5 sin(2 pi n / 400) e_x"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic, 0),
                     "kernel": kernel, "bytes_per_cell": BYTES_PER_CELL[args.storage],
                     "cells_per_launch": main_run["ncell"],
                     "avg_launch_ms": round(main_run["collide_avg_ms"], 5)},
        "step_hbm_frac": round(main_run["mlups"] * 1e6 * BYTES_PER_CELL[args.storage] / (HBM_PEAK_GBS * 1e9), 4),
        "ib_workgroups": nib,
        # launches before the main one per step: every immersed-boundary phase (nib = 0); with the chain beside
        # the collide, only the first step's skinning and tile binning, over all timed steps
        "pre_launch_ms_per_step": round(main_run["ib_avg_ms"], 5),
        "device_status": main_run["status"],
        "forms": forms,
    }
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
