"""The immersed-boundary phases beside the collide in one launch
(k_step_overlap, lbm_params.ib_workgroups > 0, the benchmark's headline
configuration) against the same phases in launches of their own before the
collide (ib_workgroups = 0 or -1):
the arithmetic is the same inline code, so every result must agree bit for
bit, for any number of chain workgroups, with multi-direct forcing passes,
2-byte storage, TRT, open y/z faces, a rotating frame, a body across the
periodic corner of a ragged lattice, and band cells on open faces beyond
their source tile."""
import numpy as np
import pytest
import torch

from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _run(w, nsteps, ib_workgroups, storage="f32", collision=0, mdf=None, block=(0, 0), max_active_tiles=0,
         status=lbm.OK, ib_scheme=lbm.IB_DIRECT):
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, storage=storage, max_markers=w.markers.n,
                         max_bones=w.markers.nbones, u0=w.u0.astype(np.float32), bc_y=w.bc_y, bc_z=w.bc_z,
                         collision=collision, mdf_iters=mdf or w.mdf_iters, ib_workgroups=ib_workgroups,
                         block=block, max_active_tiles=max_active_tiles, ib_scheme=ib_scheme)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses[:nsteps], np.float32), device="cuda")
    wrench = torch.zeros((nsteps, 8), dtype=torch.float32, device="cuda")
    sim.step(w.frames[:nsteps], dm, poses, wrench)
    assert sim.check() == status
    rho, u = sim.macros(w.frames[nsteps - 1])
    out = dict(f=sim.read_populations().cpu().numpy(), rho=rho.cpu().numpy(), u=u.cpu().numpy(),
               F=dm.F.cpu().numpy(), X=dm.X.cpu().numpy(), wrench=wrench.cpu().numpy())
    sim.close()
    return out


def _ragged():
    nx, ny, nz = 37, 21, 13
    ms = I.fibonacci_sphere(300, 3.0, (0.4, 20.3, 12.6))
    ms.xrest[0] %= nx
    ms.xrest[1] %= ny
    ms.xrest[2] %= nz
    n = 6
    return I.Workload("ragged", nx, ny, nz, 0.7, I.BC_PERIODIC, I.BC_PERIODIC, n,
                      I.perturbed_velocity((nz, ny, nx), (0.02, 0.01, 0.0), 1e-3, 3), ms, I.identity_poses(n),
                      I.make_frames(n, origin=(0.4, 20.3, 12.6)), np.array([-1.0, 0, 0]))


def _open_yz_rotating():
    w = I.sphere_workload(nsteps=8)
    w.bc_y = (I.BC_VELOCITY, I.BC_OUTFLOW)
    w.bc_z = (I.BC_OUTFLOW, I.BC_VELOCITY)
    w.frames = w.frames.copy()
    w.frames[:, 3:6] = (0.0, 0.0, 3e-4)
    w.frames[:, 9:12] = (20.0, 16.0, 16.0)
    return w


def _hi_faces():
    """Every face open, each dimension 8k + 1 (the last tile one node wide),
    and a body whose stencils reach node n - 2 on each axis: the face nodes
    n - 1 take their populations and force from the tile before theirs."""
    nx, ny, nz = 41, 25, 17
    u_in = np.array([0.03, 0.01, 0.0])
    n = 6
    w = I.Workload("hi-faces", nx, ny, nz, 0.6, I.BC_VELOCITY, I.BC_OUTFLOW, n,
                   I.perturbed_velocity((nz, ny, nx), u_in, 1e-3, 5), I.fibonacci_sphere(400, 3.0, (34.4, 18.4, 10.4)),
                   I.identity_poses(n), I.make_frames(n, origin=(34.4, 18.4, 10.4), u_lo=u_in, u_hi=u_in),
                   np.array([-1.0, 0, 0]))
    w.bc_y = (I.BC_VELOCITY, I.BC_OUTFLOW)
    w.bc_z = (I.BC_VELOCITY, I.BC_OUTFLOW)
    return w


def _fin():
    return I.fin_workload(I.C5_BASE, nsteps=10, nx=48, ny=32, nz=32, length=16.0, n=600, head=(12.0, 16.0, 16.0))


CASES = {
    "sphere-f32": (lambda: I.sphere_workload(nsteps=10), 10, dict()),
    "sphere-mdf3": (lambda: I.sphere_workload(nsteps=6), 6, dict(mdf=3)),
    "sphere-f16": (lambda: I.sphere_workload(nsteps=10), 10, dict(storage="f16")),
    "sphere-bf16-trt": (lambda: I.sphere_workload(nsteps=10), 10, dict(storage="bf16", collision=lbm.COLLIDE_TRT)),
    "sphere-2d-blocks": (lambda: I.sphere_workload(nsteps=6), 6, dict(block=(64, 8))),
    "ragged-37x21x13": (_ragged, 6, dict()),
    "open-yz-rotating": (_open_yz_rotating, 8, dict()),
    "hi-faces-41x25x17": (_hi_faces, 6, dict()),
    "hi-faces-f16-trt": (_hi_faces, 6, dict(storage="f16", collision=lbm.COLLIDE_TRT)),
    "fin-48x32x32": (_fin, 10, dict()),
    # more active tiles than the capacity: the tiles past it get no slot, no
    # force and no band cells, the same way in either schedule, and the
    # capacity guard is raised
    "sphere-capacity-8-tiles": (lambda: I.sphere_workload(nsteps=4), 4,
                                dict(max_active_tiles=8, status=lbm.ERR_CAPACITY)),
    # the implicit correction keeps its phases in launches of their own
    # whatever ib_workgroups asks
    "sphere-implicit-2": (lambda: I.sphere_workload(nsteps=4), 4, dict(ib_scheme=lbm.IB_IMPLICIT, mdf=2)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_overlapped_step_matches_separate_launches_bitwise(case):
    make, n, kw = CASES[case]
    w = make()
    say(f"overlap: {case}, {n} steps")
    ref = _run(w, n, -1, **kw)
    for nib in (1, 7, 64):
        got = _run(w, n, nib, **kw)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (nib, k)
    assert np.abs(ref["wrench"][:, 0]).max() > 0


def test_chain_beyond_what_the_device_holds_is_held_to_it():
    """ib_workgroups = 1024, more workgroups than the device runs at once:
    the library holds the chain to what the device holds, so its barriers
    complete, and every result is the separate launches' bits."""
    w = I.sphere_workload(nsteps=4)
    say("overlap: 1024 chain workgroups requested")
    ref = _run(w, 4, -1)
    got = _run(w, 4, 1024)
    for k in ref:
        assert np.array_equal(ref[k], got[k]), k
