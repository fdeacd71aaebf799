"""Open faces on every axis (non-equilibrium extrapolation on y and z faces,
edges and corners from the diagonal inward neighbour) against the FP64
oracle: one step from a random state with every combination of open axes and
face kinds, a sphere in a fully open box over 40 steps, the batched form with
such environments, and the adjoint refusing them."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import gpu_run, interior, oracle_run, random_state, rel_l2, say

pytestmark = pytest.mark.gpu

V, O, P = I.BC_VELOCITY, I.BC_OUTFLOW, I.BC_PERIODIC


def _box(nx, ny, nz, faces, nsteps, frames=None):
    u0 = np.zeros((3, nz, ny, nx))
    fr = frames if frames is not None else I.make_frames(nsteps, u_lo=(0.03, -0.01, 0.02), u_hi=(0.02, 0.0, 0.0))
    w = I.Workload("box", nx, ny, nz, 0.6, faces[0][0], faces[0][1], nsteps, u0, None, np.zeros((nsteps, 1, 24)),
                   fr, heading=np.array([-1.0, 0.0, 0.0]))
    w.bc_y, w.bc_z = faces[1], faces[2]
    return w


@pytest.mark.parametrize("faces", [
    ((P, P), (V, O), (P, P)),
    ((P, P), (P, P), (O, V)),
    ((V, O), (V, V), (O, O)),
    ((O, V), (O, O), (V, O)),
    ((V, V), (V, V), (V, V)),
])
def test_one_step_open_faces_against_oracle(faces):
    w = _box(37, 21, 19, faces, 1)
    w.frames[:, 0:3] = (2e-4, -1e-4, 5e-5)  # a frame acceleration, so F_b is nonzero on the faces
    f0 = random_state(w, 11)
    sim, _, _ = gpu_run(w, 1, f0=f0)
    got = sim.read_populations().cpu().numpy().astype(np.float64)
    ref = oracle_run(w, 1, f0=f0.astype(np.float64))
    # compare pre-collision values of the nodes off the open faces
    d = np.abs(interior(got, w) - interior(ref["f"], w)).max()
    say(f"faces {faces}: max |df| off the faces {d:.3e}")
    assert d < 1e-6


def test_sphere_in_fully_open_box_40_steps():
    sw = I.sphere_workload(nsteps=40)
    w = dataclasses.replace(sw)
    w.bc_y, w.bc_z = (V, O), (O, V)
    u_in = np.array([0.05, 0.0, 0.0])
    w.frames = I.make_frames(40, origin=(20.0, 16.0, 16.0), u_lo=u_in, u_hi=u_in)
    sim, dm, wr = gpu_run(w, 40)
    _, u = sim.macros(w.frames[39])
    torch.cuda.synchronize()
    assert sim.check() == 0
    ref = oracle_run(w, 40)
    _, u_ref = oracle.macros(ref["prm"], ref["f"], w.frames[39])
    e = rel_l2(interior(u.cpu().numpy().astype(np.float64), w), interior(u_ref, w))
    derr = np.abs(wr[:, 0] - ref["wrench"][:, 0]).max() / np.abs(ref["wrench"][:, 0]).max()
    say(f"sphere, all faces open: velocity rel L2 {e:.3e}, drag max rel err {derr:.3e}")
    assert e <= 1e-5 and derr <= 1e-4


def test_marker_range_guard_on_open_y_face():
    sw = I.sphere_workload(nsteps=1)
    w = dataclasses.replace(sw, markers=I.fibonacci_sphere(200, 3.0, (20.0, 4.5, 16.0)))  # reaches y = 1.5
    w.bc_y = (O, O)
    sim, _, _ = gpu_run(w, 1)
    assert sim.check() == lbm.ERR_MARKER_RANGE


def test_batched_environments_with_open_faces():
    """Environments with open y or z faces in a batch: the per-phase driver
    launches a collide specialised to their kind. Each agrees with its lone
    run (bit for bit as measured; the bound allows float32 rounding) and with
    the oracle."""
    n = 10
    envs = I.batch_workloads(count=2, seed=9, nsteps=n)
    envs[0].bc_y = (V, O)
    envs[1].bc_z = (O, O)
    b = lbm.Batch(envs, n)
    b.run(n, mode="phases", graph=False)
    assert b.check() == 0
    with torch.cuda.stream(b.stream):
        got = [s.read_populations() for s in b.sims]
        us = [s.macros(w.frames[n - 1])[1] for s, w in zip(b.sims, envs)]
    b.synchronize()
    for j, w in enumerate(envs):
        sim, _, _ = gpu_run(w, n, block=(128, 4))
        want = sim.read_populations()
        torch.cuda.synchronize()
        d = (got[j] - want).abs().max().item()
        ref = oracle_run(w, n)
        _, u_ref = oracle.macros(ref["prm"], ref["f"], w.frames[n - 1])
        e = rel_l2(interior(us[j].cpu().numpy().astype(np.float64), w), interior(u_ref, w))
        say(f"batched env {j} with open y/z faces: max |df| vs alone {d:.3e}, velocity rel L2 vs oracle {e:.3e}")
        assert d < 1e-6 and e <= 1e-5


def test_adjoint_refuses_open_y_or_z_faces():
    w = _box(16, 16, 16, ((V, O), (O, O), (P, P)), 1)
    sim = lbm.Simulation(16, 16, 16, 0.6, V, O, with_adjoint=True, bc_y=(O, O))
    s = sim.new_state()
    sim.save_state(s)
    lam = torch.zeros(sim.population_bytes // 4, device="cuda")
    with pytest.raises(lbm.LBMError) as ei:
        sim.adjoint_step(s, None, None, w.frames[0], [0, 0, 0, 0], lam, torch.zeros_like(lam), None)
    assert ei.value.code == lbm.ERR_UNSUPPORTED
