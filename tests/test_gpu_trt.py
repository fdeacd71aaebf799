"""Parity of the two-relaxation-time collision on the GPU with the FP64
oracle (same tolerances as the BGK step: one step from float32-exact inputs
keeps float32 rounding only, 1e-6 of the population scale; 100 sphere steps
hold the velocity to 1e-5 relative L2; 2-byte storage a few half-ulps of |h|)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import gpu_run, interior, oracle_run, random_state, rel_l2, say

pytestmark = pytest.mark.gpu


def _trt(w, lam=3.0 / 16.0):
    w.collision = lbm.COLLIDE_TRT
    w.trt_lambda = lam
    return w


def _one_step(w, seed, storage="f32", bound=None):
    f0 = random_state(w, seed)
    sim, dm, wr = gpu_run(w, nsteps=1, f0=f0, storage=storage)
    ref = oracle_run(w, nsteps=1, f0=f0)
    got = sim.read_populations().cpu().numpy().astype(np.float64)
    err = np.abs(interior(got, w) - interior(ref["f"], w)).max()
    say(f"{w.name} TRT (Lambda {w.trt_lambda:.4f}, {storage}): max |df| = {err:.3e}")
    assert sim.check() == 0
    if bound is None:
        assert err < 1e-6 * np.abs(ref["f"]).max()
    else:
        _, wts = oracle.lattice()
        h = np.abs(interior(ref["f"], w) - wts.reshape(27, 1, 1, 1)).max()
        assert err <= 4 * bound * h
    if dm is not None:
        np.testing.assert_allclose(wr[0, :7], ref["wrench"][0, :7], atol=2e-4 * np.abs(ref["wrench"][0, :7]).max())


@pytest.mark.parametrize("lam", [3.0 / 16.0, 1.0 / 12.0, 0.5])
def test_one_step_periodic_no_body(lam):
    w = _trt(I.sphere_workload(nsteps=1), lam)
    w.markers = None
    w.bc_lo = w.bc_hi = I.BC_PERIODIC
    _one_step(w, 31)


def test_one_step_open_faces_accelerating_rotating_frame_with_body():
    w = _trt(I.sphere_workload(nsteps=1))
    w.frames = I.make_frames(1, acc=(1e-4, -2e-4, 5e-5), omega=(0.002, -0.001, 0.003), alpha=(1e-5, 0, -2e-5),
                             origin=(30.5, 15.0, 16.5), u_lo=(0.04, 0.01, 0.0), u_hi=(0.05, 0, 0))
    _one_step(w, 32)


def test_one_step_open_faces_on_every_axis():
    w = _trt(I.sphere_workload(nsteps=1))
    w.bc_y = (I.BC_VELOCITY, I.BC_OUTFLOW)
    w.bc_z = (I.BC_OUTFLOW, I.BC_VELOCITY)
    w.frames = I.make_frames(1, acc=(1e-4, 0, 0), origin=(30.5, 15.0, 16.5), u_lo=(0.04, 0.01, 0.0),
                             u_hi=(0.05, 0, 0))
    _one_step(w, 33)


@pytest.mark.parametrize("storage,bound", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_one_step_two_byte_storage(storage, bound):
    _one_step(_trt(I.sphere_workload(nsteps=1)), 34, storage, bound)


def test_sphere_100_steps():
    w = _trt(I.sphere_workload())
    sim, dm, wr = gpu_run(w)
    assert sim.check() == 0
    ref = oracle_run(w)
    _, u_ref = oracle.macros(ref["prm"], ref["f"], w.frames[-1])
    _, u = sim.macros(w.frames[-1])
    e = rel_l2(interior(u.cpu().numpy().astype(np.float64), w), interior(u_ref, w))
    drag = np.abs(wr[:, 0] - ref["wrench"][:, 0]).max() / np.abs(ref["wrench"][:, 0]).max()
    say(f"TRT sphere 100 steps: velocity rel L2 {e:.3e}, drag series max rel err {drag:.3e}")
    assert e <= 1e-5
    assert drag <= 1e-4


def test_equal_rates_match_bgk():
    """Lambda = (tau - 1/2)^2 makes both rates 1/tau: one step of the TRT
    kernel gives the BGK kernel's result up to float rounding (the rates are
    rounded separately; over many steps such differences grow with the flow)."""
    w = I.sphere_workload(nsteps=1)
    f0 = random_state(w, 35)
    a, _, wa = gpu_run(w, f0=f0)
    b, _, wb = gpu_run(_trt(I.sphere_workload(nsteps=1), (w.tau - 0.5) ** 2), f0=f0)
    fa, fb = a.read_populations(), b.read_populations()
    d = (fa - fb).abs().max().item()
    say(f"TRT with equal rates vs BGK, one step: max |df| = {d:.3e}")
    assert d <= 1e-7


@pytest.mark.parametrize("mode", ["phases", "persistent"])
def test_batched_trt_environments(mode):
    """A batch mixing TRT (two values of Lambda) and BGK environments: the
    per-phase driver launches one collide per collision kind, the persistent
    kernel picks each environment's collision at run time. Each environment
    agrees with its lone single-lattice run (bit for bit as measured; the
    bound allows float32 rounding), and the TRT ones with the FP64 oracle."""
    n = 10
    envs = I.batch_workloads(count=3, seed=13, nsteps=n)
    _trt(envs[0])
    _trt(envs[1], 0.25)
    b = lbm.Batch(envs, n)
    b.run(n, mode=mode, graph=False)
    assert b.check() == 0
    with torch.cuda.stream(b.stream):
        got = [s.read_populations() for s in b.sims]
        us = [s.macros(w.frames[n - 1])[1] for s, w in zip(b.sims, envs)]
    b.synchronize()
    for j, w in enumerate(envs):
        sim, _, wr = gpu_run(w, n, block=(128, 4))
        want = sim.read_populations()
        torch.cuda.synchronize()
        d = (got[j] - want).abs().max().item()
        dw = np.abs(b.wrench[j].cpu().numpy() - wr).max()
        msg = f"{mode} env {j} collision {w.collision} lambda {w.trt_lambda}: max |df| vs alone {d:.3e}, wrench {dw:.3e}"
        if w.collision == lbm.COLLIDE_TRT:
            ref = oracle_run(w, n)
            _, u_ref = oracle.macros(ref["prm"], ref["f"], w.frames[n - 1])
            e = rel_l2(interior(us[j].cpu().numpy().astype(np.float64), w), interior(u_ref, w))
            msg += f", velocity rel L2 vs oracle {e:.3e}"
            assert e <= 1e-5
        say(msg)
        assert d < 1e-6 and dw < 1e-6


def test_adjoint_rejects_trt():
    w = _trt(I.sphere_workload(nsteps=4))
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=w.markers.n, max_bones=1,
                         u0=w.u0.astype(np.float32), with_adjoint=True, collision=lbm.COLLIDE_TRT)
    dm = lbm.DeviceMarkers(w.markers)
    pose = torch.as_tensor(w.poses[0].astype(np.float32), device="cuda")
    s = sim.new_state()
    sim.save_state(s)
    lam = torch.zeros(sim.population_bytes // 4, device="cuda")
    with pytest.raises(lbm.LBMError) as ei:
        sim.adjoint_step(s, dm, pose, w.frames[0], [1, 0, 0, 0], lam, torch.zeros_like(lam), torch.zeros_like(pose))
    assert ei.value.code == lbm.ERR_UNSUPPORTED
    sim.close()
