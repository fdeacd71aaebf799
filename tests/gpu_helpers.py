"""Shared helpers for the GPU parity tests: run a workload through the HIP
library (via the binding) and through the FP64 oracle from the same inputs."""
import sys

import numpy as np
import torch

import oracle
from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_sim(w, storage="f32", f0=None, block=(0, 0), mdf_iters=None, max_active_tiles=0, ib_workgroups=0):
    """A context for workload w (its faces, IB scheme and passes)."""
    nb = w.markers.nbones if w.markers is not None else 1
    nm = w.markers.n if w.markers is not None else 0
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=storage, max_markers=nm,
                         max_bones=nb, mdf_iters=mdf_iters or w.mdf_iters, ib_alpha=w.ib_alpha,
                         rho0=None if f0 is not None else np.ones((w.nz, w.ny, w.nx), np.float32),
                         u0=None if f0 is not None else w.u0.astype(np.float32), block=block,
                         max_active_tiles=max_active_tiles, bc_y=w.bc_y, bc_z=w.bc_z, ib_scheme=w.ib_scheme,
                         collision=w.collision, trt_lambda=w.trt_lambda, wall_mode=w.wall_mode,
                         ib_workgroups=ib_workgroups)
    if f0 is not None:
        sim.load_populations(f0)
    return sim


def gpu_run(w, nsteps=None, storage="f32", f0=None, block=(0, 0), mdf_iters=None, chunk=None, ib_workgroups=0):
    """Returns (sim, markers-or-None, wrench (nsteps, 8) numpy)."""
    nsteps = nsteps or w.nsteps
    sim = gpu_sim(w, storage, f0, block, mdf_iters, ib_workgroups=ib_workgroups)
    dm = lbm.DeviceMarkers(w.markers) if w.markers is not None else None
    poses = torch.as_tensor(np.ascontiguousarray(w.poses[:nsteps], np.float32), device="cuda") if dm else None
    wrench = torch.zeros((nsteps, 8), dtype=torch.float32, device="cuda")
    chunk = chunk or nsteps
    for s0 in range(0, nsteps, chunk):
        s1 = min(nsteps, s0 + chunk)
        sim.step(w.frames[s0:s1], dm, poses[s0:s1] if dm is not None else None, wrench[s0:s1])
    torch.cuda.synchronize()
    return sim, dm, wrench.cpu().numpy()


def oracle_run(w, nsteps=None, f0=None, mdf_iters=None):
    prm = oracle.params(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, mdf_iters or w.mdf_iters, w.ib_alpha, w.bc_y,
                        w.bc_z, w.ib_scheme, w.collision, w.trt_lambda, w.wall_mode)
    if f0 is None:
        f0 = oracle.equilibrium_field(np.ones((w.nz, w.ny, w.nx)), w.u0.astype(np.float32).astype(np.float64))
    res = oracle.run(prm, np.array(f0, dtype=np.float64), w.frames, w.markers, w.poses, nsteps or w.nsteps)
    res["prm"] = prm
    return res


def interior(a, w):
    """Drop the planes of open faces (their pre-collision values are never used)."""
    if w.bc_lo != I.BC_PERIODIC:
        a = a[..., 1:-1]
    if w.bc_y[0] != I.BC_PERIODIC:
        a = a[..., 1:-1, :]
    if w.bc_z[0] != I.BC_PERIODIC:
        a = a[..., 1:-1, :, :]
    return a


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def random_state(w, seed, du=0.03, noise=1e-4):
    """Seeded near-equilibrium pre-collision populations, float32-exact."""
    shape = (w.nz, w.ny, w.nx)
    rho = I.random_density(shape, 0.01, seed)
    u = I.perturbed_velocity(shape, (0.02, -0.01, 0.01), du, seed + 1)
    f = oracle.equilibrium_field(rho, u) + I.random_offsets((27,) + shape, noise, seed + 2)
    return f.astype(np.float32)
