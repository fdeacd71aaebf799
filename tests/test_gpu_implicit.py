"""Parity of the implicit velocity correction (conjugate-gradient steps on
S G = (I + [omega]x)(U - U*)) on the GPU with the FP64 oracle.

Tolerances. Conjugate gradients amplify rounding by the conditioning of S
(markers closer than a cell make it nearly singular), so the float32 forces
drift from the FP64 ones with each step: about 1e-6 of their largest value
per step was measured (8e-6 after 4 steps on the 3000-marker fin), and the
bar is 5e-5; populations after one step stay within float32 rounding of
one direct-forcing step (2e-6 of their largest value). What the scheme is
for -- the slip at the markers -- is checked directly: the GPU forces, spread
and interpolated by the oracle, must leave no more slip than the oracle's own
forces plus float32 noise."""
import numpy as np
import pytest
import torch

import oracle
from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import gpu_run, interior, oracle_run, random_state, rel_l2, say

pytestmark = pytest.mark.gpu


def _rms_slip(prm, f0, frame, X, U, G, omega):
    rho, ustar = oracle.macros(prm, f0, frame)
    g = oracle.spread(prm, X, G) / (2.0 * rho)
    w = np.asarray(omega, dtype=np.float64).reshape(3, 1, 1, 1)
    corr = (g - np.cross(w, g, axis=0) + (w * g).sum(0, keepdims=True) * w) / (1.0 + (w * w).sum())
    r = oracle.interpolate(prm, ustar + corr, X) - U
    return float(np.sqrt((r * r).mean()))


def _one_step(w, seed, iters, omega=(0.0, 0.0, 0.0)):
    w.ib_scheme = lbm.IB_IMPLICIT
    f0 = random_state(w, seed)
    say(f"{w.name}: implicit, {iters} CG steps, {w.markers.n} markers")
    sim, dm, wr = gpu_run(w, nsteps=1, f0=f0, mdf_iters=iters)
    ref = oracle_run(w, nsteps=1, f0=f0, mdf_iters=iters)
    got = sim.read_populations().cpu().numpy().astype(np.float64)
    err_f = np.abs(interior(got, w) - interior(ref["f"], w)).max() / np.abs(ref["f"]).max()
    F = dm.F.cpu().numpy().astype(np.float64)
    err_F = np.abs(F - ref["F"]).max() / np.abs(ref["F"]).max()
    dv = w.markers.dv
    s_gpu = _rms_slip(ref["prm"], f0.astype(np.float64), w.frames[0], ref["X"], ref["U"], F * dv, omega)
    s_ref = _rms_slip(ref["prm"], f0.astype(np.float64), w.frames[0], ref["X"], ref["U"], ref["F"] * dv, omega)
    err_w = np.abs(wr[0, :7] - ref["wrench"][0, :7]).max() / np.abs(ref["wrench"][0, :7]).max()
    say(f"  populations {err_f:.2e}, forces {err_F:.2e}, wrench {err_w:.2e}; "
        f"rms slip gpu {s_gpu:.3e} oracle {s_ref:.3e}")
    assert sim.check() == 0
    assert err_f < 2e-6
    assert err_F < 5e-5
    assert err_w < 1e-5
    assert s_gpu <= 1.05 * s_ref + 1e-6
    return s_gpu


@pytest.mark.parametrize("iters", [1, 3, 6])
def test_one_step_sphere(iters):
    _one_step(I.sphere_workload(nsteps=1), 11, iters)


def test_one_step_rotating_frame():
    w = I.sphere_workload(nsteps=1)
    omega = (0.002, -0.001, 0.003)
    w.frames = I.make_frames(1, acc=(1e-4, 0, 0), omega=omega, origin=(30.5, 15.0, 16.5), u_lo=(0.04, 0, 0),
                             u_hi=(0.04, 0, 0))
    _one_step(w, 12, 4, omega)


def test_one_step_ragged_grid_wrapping_markers():
    nx, ny, nz = 37, 21, 13
    ms = I.fibonacci_sphere(300, 3.0, (0.4, 20.3, 12.6))
    ms.xrest[0] %= nx
    ms.xrest[1] %= ny
    ms.xrest[2] %= nz
    w = I.Workload("ragged", nx, ny, nz, 0.7, I.BC_PERIODIC, I.BC_PERIODIC, 1, np.zeros((3, nz, ny, nx)), ms,
                   I.identity_poses(1), I.make_frames(1, origin=(0.4, 20.3, 12.6)), np.array([-1.0, 0, 0]))
    _one_step(w, 13, 3)


def test_one_step_fish_mid_stroke():
    w = I.fin_workload(nsteps=160)
    w.poses = w.poses[157:158]
    w.frames = w.frames[157:158]
    w.nsteps = 1
    _one_step(w, 14, 4)


def test_sphere_100_steps():
    w = I.sphere_workload()
    w.ib_scheme = lbm.IB_IMPLICIT
    sim, dm, wr = gpu_run(w, mdf_iters=3)
    assert sim.check() == 0
    ref = oracle_run(w, mdf_iters=3)
    _, u_ref = oracle.macros(ref["prm"], ref["f"], w.frames[-1])
    _, u = sim.macros(w.frames[-1])
    u = u.cpu().numpy().astype(np.float64)
    e = rel_l2(interior(u, w), interior(u_ref, w))
    drag_err = np.abs(wr[:, 0] - ref["wrench"][:, 0]).max() / np.abs(ref["wrench"][:, 0]).max()
    say(f"implicit sphere 100 steps: velocity rel L2 {e:.3e}, drag series max rel err {drag_err:.3e}")
    assert e <= 1e-5
    assert drag_err <= 1e-5


def test_determinism_bitwise():
    w = I.sphere_workload(nsteps=20)
    w.ib_scheme = lbm.IB_IMPLICIT
    a, _, wa = gpu_run(w, mdf_iters=4)
    b, _, wb = gpu_run(w, mdf_iters=4)
    assert torch.equal(a.read_populations(), b.read_populations())
    assert np.array_equal(wa, wb)


@pytest.mark.parametrize("graph", [False, True])
def test_batched_implicit_environments_match_lone_runs(graph):
    """Three environments with the implicit correction (3 CG steps; one in a
    rotating frame, one with FP16 storage) batched by the per-phase driver:
    every environment equal to its lone single-lattice run, populations and
    wrench. The persistent driver refuses implicit batches."""
    n = 10
    envs = I.batch_workloads(count=3, seed=23, nsteps=n)
    for w in envs:
        w.ib_scheme = lbm.IB_IMPLICIT
        w.mdf_iters = 3
    w = envs[1]
    w.frames[:, 3:6] = (0.0, 0.0, 1e-3)
    w.frames[:, 9:12] = (w.nx / 2.0, w.ny / 2.0, w.nz / 2.0)
    formats = ["f32", "f32", "f16"]
    b = lbm.Batch(envs, n, storage=formats)
    b.run(n, mode="phases", graph=graph)
    assert b.check() == 0
    with torch.cuda.stream(b.stream):
        got = [s.read_populations() for s in b.sims]
    b.synchronize()
    for j, w in enumerate(envs):
        sim, _, wr = gpu_run(w, n, storage=formats[j], block=(128, 4))
        want = sim.read_populations()
        torch.cuda.synchronize()
        d = (got[j] - want).abs().max().item()
        dw = np.abs(b.wrench[j].cpu().numpy() - wr).max()
        say(f"graph={graph} implicit env {j} ({w.nx}x{w.ny}x{w.nz}, {formats[j]}): max |df| vs alone {d:.3e}, "
            f"wrench {dw:.3e}")
        assert d == 0.0 and dw == 0.0
    with pytest.raises(lbm.LBMError) as ei:
        b.run(n, mode="persistent", graph=graph)
    assert ei.value.code == lbm.ERR_UNSUPPORTED
    b.close()


def test_batch_mixing_schemes_and_adjoint_reject_the_implicit_scheme():
    w = I.sphere_workload(nsteps=4)
    w.ib_scheme = lbm.IB_IMPLICIT
    with pytest.raises(lbm.LBMError) as ei:
        lbm.Batch([w, I.sphere_workload(nsteps=4)], 4)
    assert ei.value.code == lbm.ERR_UNSUPPORTED
    sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=w.markers.n, max_bones=1,
                         u0=w.u0.astype(np.float32), with_adjoint=True, ib_scheme=lbm.IB_IMPLICIT)
    dm = lbm.DeviceMarkers(w.markers)
    pose = torch.as_tensor(w.poses[0].astype(np.float32), device="cuda")
    s = sim.new_state()
    sim.save_state(s)
    lam = torch.zeros(sim.population_bytes // 4, device="cuda")
    with pytest.raises(lbm.LBMError) as ei:
        sim.adjoint_step(s, dm, pose, w.frames[0], [1, 0, 0, 0], lam, torch.zeros_like(lam), torch.zeros_like(pose))
    assert ei.value.code == lbm.ERR_UNSUPPORTED
    sim.close()
