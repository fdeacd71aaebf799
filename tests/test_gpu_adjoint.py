"""Discrete adjoint of the coupled step (lbm_adjoint_step) and the
checkpointed reverse sweep: gradients with respect to the initial state
(dot-product test against central differences of the GPU forward), with
respect to the kinematics parameters (against the FP64 oracle's forward-mode
tangent), and invariance under the checkpoint interval."""
import numpy as np
import pytest
import torch

import oracle
from paper_2206_01683_amd import adjoint as AD
from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import say

pytestmark = pytest.mark.gpu

NSTEPS = 12
EVERY = 5  # segments of 5, 5 and 2 steps
GEOM = dict(nx=48, ny=32, nz=32, length=16.0, n=600, head=(12.0, 16.0, 16.0))


def _fin(nsteps=NSTEPS, params=I.C5_BASE):
    return I.fin_workload(params, nsteps=nsteps, **GEOM)


def _sim(w, with_markers=True, **kw):
    ms = w.markers if with_markers else None
    return lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=ms.n if ms else 0,
                          max_bones=ms.nbones if ms else 1, u0=w.u0.astype(np.float32), with_adjoint=True, **kw)


def _valid_mask(sim, ncell):
    """Stored-layout entries that hold populations (27 per cell; the rest of
    the buffer is padding)."""
    m = torch.zeros(sim.population_bytes // 4, dtype=torch.float32, device="cuda")
    sim.stored_view(m).fill_(1.0)
    return m != 0


def _smooth_perturbation(sim, w, state, seed, amp=1e-3):
    """delta_i(x) = amp * f_i(x) * (a_i + b_i sin(2 pi (x/nx + y/ny) + p_i)):
    smooth in space, random across directions, so it moves density and
    velocity coherently near the body. The stored layout holds h_i = f_i - w_i."""
    rng = np.random.default_rng(seed)
    a, b, p = rng.uniform(-1, 1, 27), rng.uniform(-1, 1, 27), rng.uniform(0, 2 * np.pi, 27)
    z, y, x = np.meshgrid(np.arange(w.nz), np.arange(w.ny), np.arange(w.nx), indexing="ij")
    ph = 2 * np.pi * (x / w.nx + y / w.ny)
    _, wts = oracle.lattice()
    f = sim.stored_view(state).cpu().numpy() + wts[:, None, None, None].astype(np.float32)
    d = np.zeros((27, w.nz, w.ny, w.nx), np.float32)
    for i in range(27):
        d[i] = amp * f[i] * (a[i] + b[i] * np.sin(ph + p[i]))
    out = torch.zeros(sim.population_bytes // 4, dtype=torch.float32, device="cuda")
    sim.stored_view(out).copy_(torch.as_tensor(d, device="cuda"))
    return out


def _run_J(sim, s0, dm, poses, frames, weights, c=None):
    sim.bind_own_buffers()
    sim.restore_state(s0, 0)
    J, tape = AD.forward(sim, dm, poses, frames, weights, every=len(frames))
    if c is not None:
        J += float(torch.dot(c.double(), tape.final.view(torch.float32).double()))
    return J


ACC = (2e-4, -1e-4, 5e-5)  # a uniform frame acceleration (Eq. (3) with no rotation)


def _accelerate(w):
    w.frames = w.frames.copy()
    w.frames[:, 0:3] = ACC
    return w


@pytest.mark.parametrize("case", ["fin", "fin-accelerating", "fin-periodic", "fluid-open", "fluid-periodic",
                                  "fluid-open-accelerating"])
def test_state_adjoint_matches_central_differences(case):
    """<dJ/ds0, delta> from the reverse sweep equals (J(s0 + delta) - J(s0 - delta)) / 2."""
    if case == "fin-periodic":  # the body straddles the periodic x seam
        w = I.fin_workload(I.C5_BASE, nsteps=NSTEPS, **dict(GEOM, head=(40.0, 16.0, 16.0)))
    else:
        w = _fin()
    if "periodic" in case:
        w.bc_lo = w.bc_hi = I.BC_PERIODIC
    if "accelerating" in case:
        _accelerate(w)
    markers = case.startswith("fin")
    sim = _sim(w, with_markers=markers)
    dm = lbm.DeviceMarkers(w.markers) if markers else None
    poses = torch.as_tensor(w.poses.astype(np.float32), device="cuda") if markers else None
    rng = np.random.default_rng(3)
    weights = rng.uniform(-1, 1, 4) if markers else np.zeros(4)
    mask = _valid_mask(sim, w.ncell)
    c = None
    if not markers:  # terminal functional <c, s_N> with c smooth in space
        c = _smooth_perturbation(sim, w, torch.ones(sim.population_bytes // 4, device="cuda").view(torch.uint8),
                                 seed=9, amp=1.0)
    s0 = sim.new_state()
    sim.save_state(s0)
    J0, tape = AD.forward(sim, dm, poses, w.frames, weights, every=EVERY)
    _, lam0 = AD.backward(sim, dm, poses, w.frames, tape, lam_final=c)
    torch.cuda.synchronize()
    delta = _smooth_perturbation(sim, w, s0, seed=5)
    adj = float(torch.dot(lam0[mask].double(), delta[mask].double()))
    sp = sim.new_state()
    sm = sim.new_state()
    sp.view(torch.float32).copy_(s0.view(torch.float32) + delta)
    sm.view(torch.float32).copy_(s0.view(torch.float32) - delta)
    Jp = _run_J(sim, sp, dm, poses, w.frames, weights, c)
    Jm = _run_J(sim, sm, dm, poses, w.frames, weights, c)
    fd = 0.5 * (Jp - Jm)
    err = abs(adj - fd) / abs(fd)
    say(f"{case}: <lam0, delta> = {adj:.8e}, central difference = {fd:.8e}, rel err {err:.2e}")
    assert np.isfinite(adj) and abs(fd) > 0
    assert err < 2e-3
    assert sim.check() == 0


def test_reverse_sweep_restores_forward_state():
    w = _fin()
    sim = _sim(w)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(w.poses.astype(np.float32), device="cuda")
    _, tape = AD.forward(sim, dm, poses, w.frames, [1, 0, 0, 0.5], every=EVERY)
    before = sim.read_populations().cpu().numpy()
    AD.backward(sim, dm, poses, w.frames, tape)
    after = sim.read_populations().cpu().numpy()
    assert np.array_equal(before, after)
    assert sim.step_count() == NSTEPS


def test_checkpoint_interval_does_not_change_gradient():
    """Recomputation is deterministic, so every interval gives the same bits."""
    w = _fin()
    sim = _sim(w)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(w.poses.astype(np.float32), device="cuda")
    s0 = sim.new_state()
    sim.save_state(s0)
    out = []
    for every in (1, EVERY, NSTEPS):
        sim.bind_own_buffers()
        sim.restore_state(s0, 0)
        _, tape = AD.forward(sim, dm, poses, w.frames, [-1, 0.3, 0, 2.0], every=every)
        pb, lam = AD.backward(sim, dm, poses, w.frames, tape)
        out.append((pb.cpu().numpy(), lam.cpu().numpy()))
    for pb, lam in out[1:]:
        assert np.array_equal(pb, out[0][0])
        assert np.array_equal(lam, out[0][1])


@pytest.mark.parametrize("every", [1, EVERY, NSTEPS])
def test_native_segment_sweep_matches_per_step_sweep(every):
    """lbm_adjoint_segment (recompute keeping each step's IB data, then the
    reverse passes) gives the same bits as recomputing by rebinding and
    calling lbm_adjoint_step per step."""
    w = _fin()
    sim = _sim(w)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(w.poses.astype(np.float32), device="cuda")
    s0 = sim.new_state()
    sim.save_state(s0)
    c = _smooth_perturbation(sim, w, s0, seed=2, amp=1.0)
    out = []
    for native in (True, False):
        sim.bind_own_buffers()
        sim.restore_state(s0, 0)
        _, tape = AD.forward(sim, dm, poses, w.frames, [-1, 0.3, 0.2, 2.0], every=every)
        pb, lam = AD.backward(sim, dm, poses, w.frames, tape, lam_final=c, native=native)
        out.append((pb.cpu().numpy(), lam.cpu().numpy(), sim.read_populations().cpu().numpy()))
        assert sim.check() == 0
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("accelerating", [False, True])
def test_parameter_gradient_against_fp64_oracle(accelerating):
    """dJ/dtheta (8 kinematics parameters) from the reverse sweep against the
    FP64 oracle's forward-mode tangent (the exact derivative of the discrete
    FP64 map, one dual-number run per parameter), J the time-averaged thrust
    plus a power term; inertial and uniformly accelerating frame."""
    weights = np.array([-1.0, 0.0, 0.0, 0.5])
    prob = AD.FinProblem(nsteps=NSTEPS, every=EVERY, weights=weights, **GEOM)
    if accelerating:
        _accelerate(prob.workload)
    theta = torch.tensor(I.C5_BASE, dtype=torch.float64, requires_grad=True)
    J = AD.FinObjective.apply(theta, prob)
    J.backward()
    g = theta.grad.numpy()
    w = prob.workload
    th = np.asarray(I.C5_BASE, dtype=np.float64)
    prm = oracle.params(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, 1, w.ib_alpha)
    f0 = oracle.equilibrium_field(np.ones((w.nz, w.ny, w.nx)), w.u0.astype(np.float32).astype(np.float64))
    poses = I.fin_poses(th, w.markers, np.arange(NSTEPS))
    jac = I.fin_pose_jacobian(th, w.markers, np.arange(NSTEPS))
    tan = np.zeros(8)
    for j in range(8):
        r = oracle.run_tangent(prm, f0.copy(), w.frames, w.markers, poses, jac[..., j], NSTEPS)
        tan[j] = AD.objective(r["wrench_d"], weights / NSTEPS)
    J64 = AD.objective(r["wrench"], weights / NSTEPS)
    say(f"J gpu {J.item():.8e} oracle {J64:.8e}")
    for j in range(8):
        say(f"  dJ/dtheta[{j}]: adjoint {g[j]: .6e}  oracle tangent {tan[j]: .6e}")
    err = np.abs(g - tan).max() / np.abs(tan).max()
    say(f"max |adjoint - tangent| / max |tangent| = {err:.2e}")
    assert abs(J.item() - J64) <= 1e-5 * abs(J64)
    assert err < 1e-4
    prob.close()


def test_adjoint_rejects_unsupported_configurations():
    w = _fin()
    dm = lbm.DeviceMarkers(w.markers)
    pose = torch.as_tensor(w.poses[0].astype(np.float32), device="cuda")
    for kw in (dict(with_adjoint=False), dict(storage="f16"), dict(mdf_iters=2)):
        args = dict(with_adjoint=True)
        args.update(kw)
        sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=w.markers.n,
                             max_bones=w.markers.nbones, u0=w.u0.astype(np.float32), **args)
        s = sim.new_state()
        sim.save_state(s)
        lam = torch.zeros(sim.population_bytes // 4, device="cuda")
        lam2 = torch.zeros_like(lam)
        pb = torch.zeros_like(pose)
        with pytest.raises(lbm.LBMError) as ei:
            sim.adjoint_step(s, dm, pose, w.frames[0], [1, 0, 0, 0], lam, lam2, pb)
        assert ei.value.code == lbm.ERR_UNSUPPORTED
        sim.close()


def test_recorded_forward_and_sweep_match_checkpointed_run():
    """Keeping every state (lbm_adjoint_record, then lbm_adjoint_sweep with
    no recompute) against checkpoints every 5 steps with the segment
    recompute: the same wrench rows, J, pose gradient, initial-state adjoint
    and final context state, bit for bit."""
    th = np.asarray(I.C5_BASE, dtype=np.float64)
    a = AD.FinProblem(nsteps=NSTEPS, every=EVERY, **GEOM)
    b = AD.FinProblem(nsteps=NSTEPS, every=EVERY, record=True, **GEOM)
    Ja, ta = a.value(th)
    Jb, tb = b.value(th)
    say(f"J checkpointed {Ja:.10e} recorded {Jb:.10e}")
    assert Ja == Jb
    assert torch.equal(ta.wrench, tb.wrench)
    assert torch.equal(a.sim.read_populations(), b.sim.read_populations())
    pa, la = AD.backward(a.sim, a.markers, ta.poses, a.workload.frames, ta)
    pb, lb = AD.backward(b.sim, b.markers, tb.poses, b.workload.frames, tb)
    torch.cuda.synchronize()
    say(f"pose gradient max |diff| {(pa - pb).abs().max().item():.3e}, lambda_0 max |diff| "
        f"{(la - lb).abs().max().item():.3e}")
    assert torch.equal(pa, pb) and torch.equal(la, lb)
    a.close()
    b.close()


def test_recorded_fluid_only_run_matches_checkpointed_run():
    """No body (zero wrench rows, a terminal functional <c, s_N>): the
    recorded forward and sweep give the checkpointed run's final state and
    initial-state adjoint bit for bit."""
    w = _fin()
    sim = _sim(w, with_markers=False)
    c = _smooth_perturbation(sim, w, torch.ones(sim.population_bytes // 4, device="cuda").view(torch.uint8),
                             seed=9, amp=1.0)
    s0 = sim.new_state()
    sim.save_state(s0)
    out = {}
    for record in (False, True):
        sim.bind_own_buffers()
        sim.restore_state(s0, 0)
        J, tape = AD.forward(sim, None, None, w.frames, np.zeros(4), every=EVERY, record=record)
        final = sim.read_populations()
        _, lam0 = AD.backward(sim, None, None, w.frames, tape, lam_final=c)
        torch.cuda.synchronize()
        out[record] = (J, tape.wrench.clone(), final, lam0.clone())
    assert out[False][0] == out[True][0] == 0.0
    assert torch.equal(out[False][1], out[True][1]) and not out[True][1].any()
    assert torch.equal(out[False][2], out[True][2])
    assert torch.equal(out[False][3], out[True][3])
    sim.close()


def test_record_and_sweep_reject_bad_arguments():
    """Host-side checks of lbm_adjoint_record / lbm_adjoint_sweep, before any
    launch: aliased ring entries, a ring entry that is the checkpoint, an
    unaligned IB ring, a rotating frame, and configurations the adjoint does
    not support."""
    w = _fin(nsteps=4)
    sim = _sim(w)
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(w.poses[:4].astype(np.float32), device="cuda")
    ck = sim.new_state()
    sim.save_state(ck)
    ring = [sim.new_state() for _ in range(4)]
    ib = sim.adjoint_ring(4)
    lam = torch.zeros(sim.population_bytes // 4, device="cuda")
    lam2 = torch.zeros_like(lam)
    pb = torch.zeros((4, w.markers.nbones, 24), device="cuda")
    bad = [
        (lambda: sim.adjoint_record(ck, [ring[0], ring[0], ring[2], ring[3]], dm, poses, w.frames[:4], ib),
         lbm.ERR_ARG),
        (lambda: sim.adjoint_record(ck, [ring[0], ck, ring[2], None], dm, poses, w.frames[:4], ib), lbm.ERR_ARG),
        (lambda: sim.adjoint_record(ck, [ring[0], ring[1], ring[2], None], dm, poses, w.frames[:4], ib[1:]),
         lbm.ERR_ARG),
        (lambda: sim.adjoint_segment(ck, [ring[0], ring[0], ring[2]], dm, poses, w.frames[:4], [1, 0, 0, 0], lam,
                                     lam2, pb, ib, sweep_only=True), lbm.ERR_ARG),
    ]
    spin = w.frames[:4].copy()
    spin[:, 3:6] = (0.0, 0.0, 1e-3)
    bad.append((lambda: sim.adjoint_record(ck, ring, dm, poses, spin, ib), lbm.ERR_UNSUPPORTED))
    bad.append((lambda: sim.adjoint_segment(ck, ring[:3], dm, poses, spin, [1, 0, 0, 0], lam, lam2, pb, ib,
                                            sweep_only=True), lbm.ERR_UNSUPPORTED))
    for j, (call, code) in enumerate(bad):
        with pytest.raises(lbm.LBMError) as ei:
            call()
        assert ei.value.code == code, j
    torch.cuda.synchronize()
    assert sim.check() == 0
    sim.close()
    f16 = _sim(w, storage="f16")
    s16 = f16.new_state()
    f16.save_state(s16)
    with pytest.raises(lbm.LBMError) as ei:
        f16.adjoint_record(s16, [f16.new_state() for _ in range(4)], dm, poses, w.frames[:4], f16.adjoint_ring(4))
    assert ei.value.code == lbm.ERR_UNSUPPORTED
    f16.close()
