"""Reverse-mode gradients of the coupled fluid-body steps.

The objective is a weighted sum over steps of the fluid force on the body and
the power the body delivers (the wrench each step reports; the external
generalized force of Eq. (1) and the coupled step of Sec. III-B):

    J = sum_n  w_F . F_n + w_P P_n  (+ <c, state_N> for a terminal term).

`forward` runs the steps on the GPU from the simulation's current state and
keeps a copy of the populations every `every` steps. `backward` walks the
segments from last to first: lbm_adjoint_segment recomputes a segment from
its checkpoint straight into a ring of states, keeping every step's forward
immersed-boundary data, then runs the adjoint passes in reverse, which carry
lambda = dJ/d(state) back one step at a time and accumulate each step's
dJ/d(bone pose). Memory: ceil(nsteps / every) checkpoints, every - 1 ring
states, the IB ring of `every` steps and two adjoint states.

With record=True, `forward` keeps every state of the horizon instead
(lbm_adjoint_record: nsteps states and the IB ring of nsteps steps, e.g.
400 x 56.6 MB for the 128x64x64 fin), and `backward` runs the reverse passes
alone (lbm_adjoint_sweep), with no recompute. The gradient is the same, bit
for bit.

`FinObjective` is a torch.autograd.Function from the 8 kinematics parameters
of the swimmer to J: each step's bone poses are an analytic function of the
parameters (inputs.fin_poses, the prescribed body motion of Sec. III-A), and
their Jacobian (inputs.fin_pose_jacobian) carries dJ/d(pose) to
dJ/d(parameters)."""
import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import inputs as I
from . import lbm


@dataclasses.dataclass
class Tape:
    """What `forward` keeps for `backward`."""
    start: int                      # step count of the context before the run
    nsteps: int
    every: int
    weights: np.ndarray             # (4,) per-step weights w_F (3), w_P
    checkpoints: List[torch.Tensor]  # state before step j * every
    final: torch.Tensor             # state after the last step
    wrench: torch.Tensor            # (nsteps, 8) float32, device
    ring: Optional[List[torch.Tensor]] = None  # record: state after step t, t < nsteps - 1
    ib_ring: Optional[torch.Tensor] = None     # record: every step's forward IB data


def objective(wrench, weights) -> float:
    """sum_n w_F . F_n + w_P P_n in float64 from the per-step wrench rows
    [force (3), torque (3), power, 0]."""
    wr = np.asarray(wrench, dtype=np.float64).reshape(-1, 8)
    w = np.asarray(weights, dtype=np.float64).reshape(4)
    return float((wr[:, :3] @ w[:3]).sum() + w[3] * wr[:, 6].sum())


def forward(sim: "lbm.Simulation", markers: Optional["lbm.DeviceMarkers"], poses: Optional[torch.Tensor],
            frames: np.ndarray, weights, every: int = 20, record: bool = False):
    """Run len(frames) steps with checkpoints (or, record=True, keeping
    every state); returns (J, tape)."""
    frames = np.asarray(frames, dtype=np.float64).reshape(-1, 18)
    n = frames.shape[0]
    if n < 1 or every < 1:
        raise ValueError("need at least one step and every >= 1")
    if markers is not None and (poses is None or poses.shape[0] < n):
        raise ValueError("poses must cover every step")
    start = sim.step_count()
    wr = torch.zeros((n, 8), dtype=torch.float32, device=sim.device)
    w4 = np.asarray(weights, dtype=np.float64).reshape(4)
    if record:
        ck = sim.new_state()
        sim.save_state(ck)
        ring = [sim.new_state() for _ in range(n)]
        ib_ring = sim.adjoint_ring(n)
        sim.adjoint_record(ck, ring, markers, None if markers is None else poses[:n].contiguous(), frames,
                           ib_ring, wr)
        sim.restore_state(ring[-1], start + n)  # the context ends after the run, as with checkpoints
        tape = Tape(start, n, n, w4, [ck], ring[-1], wr, ring=ring[:-1], ib_ring=ib_ring)
        return objective(wr.cpu().numpy(), tape.weights), tape
    cks = []
    for s in range(0, n, every):
        e = min(n, s + every)
        ck = sim.new_state()
        sim.save_state(ck)
        cks.append(ck)
        sim.step(frames[s:e], markers, None if markers is None else poses[s:e], wr[s:e])
    final = sim.new_state()
    sim.save_state(final)
    tape = Tape(start, n, every, w4, cks, final, wr)
    return objective(wr.cpu().numpy(), tape.weights), tape


def backward(sim: "lbm.Simulation", markers: Optional["lbm.DeviceMarkers"], poses: Optional[torch.Tensor],
             frames: np.ndarray, tape: Tape, lam_final: Optional[torch.Tensor] = None, native: bool = True):
    """Reverse sweep over the tape. Returns (pose_bar, lam0): dJ/d(pose of
    step n) as (nsteps, nbones, 24) float32 (None without markers) and
    dJ/d(initial state) in the stored layout (float32 view). The context ends
    at the state and step count `forward` left it in.

    native: each segment is one lbm_adjoint_segment call (recompute with the
    forward IB data of every step kept, then the reverse passes); otherwise a
    per-step loop here (recompute by rebinding the context's buffers, then
    lbm_adjoint_step per step, which recomputes the step's IB data). Both
    give the same bits."""
    frames = np.asarray(frames, dtype=np.float64).reshape(-1, 18)
    n, k = tape.nsteps, tape.every
    nfl = sim.population_bytes // 4
    dev = sim.device
    lam = torch.zeros(nfl, dtype=torch.float32, device=dev)
    if lam_final is not None:
        lam.copy_(lam_final.reshape(-1)[:nfl])
    lam2 = torch.zeros_like(lam)
    pose_bar = None
    if markers is not None:
        pose_bar = torch.zeros((n, markers.nbones, 24), dtype=torch.float32, device=dev)
    if tape.ring is not None:  # recorded: the reverse passes alone
        sim.adjoint_segment(tape.checkpoints[0], tape.ring, markers, None if markers is None else poses[:n],
                            frames[:n], tape.weights, lam, lam2, pose_bar, tape.ib_ring, sweep_only=True)
        return pose_bar, lam
    ring = [sim.new_state() for _ in range(min(k, n) - 1)]
    if native:
        ib_ring = sim.adjoint_ring(min(k, n))
        for j in reversed(range(len(tape.checkpoints))):
            s, e = j * k, min(n, (j + 1) * k)
            sim.adjoint_segment(tape.checkpoints[j], ring, markers, None if markers is None else poses[s:e],
                                frames[s:e], tape.weights, lam, lam2, None if pose_bar is None else pose_bar[s:e],
                                ib_ring)
        return pose_bar, lam
    scratch = torch.zeros((1, 8), dtype=torch.float32, device=dev)
    for j in reversed(range(len(tape.checkpoints))):
        s, e = j * k, min(n, (j + 1) * k)
        states = [tape.checkpoints[j]] + ring[:e - s - 1]
        for t in range(s, e - 1):  # recompute state t+1 from state t
            sim.bind_populations(states[t - s], states[t - s + 1])
            sim.step(frames[t:t + 1], markers, None if markers is None else poses[t:t + 1], scratch)
        for t in reversed(range(s, e)):
            sim.adjoint_step(states[t - s], markers, None if markers is None else poses[t], frames[t],
                             tape.weights, lam, lam2, None if pose_bar is None else pose_bar[t])
            lam, lam2 = lam2, lam
    sim.bind_own_buffers()
    sim.restore_state(tape.final, tape.start + n)
    return pose_bar, lam


class FinProblem:
    """The differentiation workload of inputs.fin_workload on the GPU with one
    reusable context: J(theta) = (1/N) sum_n w_F . F_n + w_P P_n over N steps
    from the inflow-velocity initial state, for kinematics parameters theta.
    The default weights (heading, 0) give the time-averaged thrust."""

    def __init__(self, nsteps: int = 400, every: int = 20, weights=None, device="cuda", max_active_tiles=256,
                 record: bool = False, **geometry):
        w = I.fin_workload(I.C5_BASE, nsteps=nsteps, **geometry)
        self.workload = w
        self.record = record  # keep every state (forward(record=True)) instead of checkpoints
        self.nsteps, self.every = nsteps, every
        if weights is None:
            weights = np.concatenate([w.heading, [0.0]])
        self.weights = np.asarray(weights, dtype=np.float64).reshape(4) / nsteps
        self.steps = np.arange(nsteps)
        ms = w.markers
        self.sim = lbm.Simulation(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, max_markers=ms.n,
                                  max_bones=ms.nbones, u0=w.u0.astype(np.float32), device=device,
                                  with_adjoint=True, max_active_tiles=max_active_tiles)
        self.s0 = self.sim.new_state()
        self.sim.save_state(self.s0)
        self.markers = lbm.DeviceMarkers(ms, device=device)

    def poses(self, theta) -> np.ndarray:
        return I.fin_poses(np.asarray(theta, dtype=np.float64), self.workload.markers, self.steps)

    def value(self, theta):
        """J(theta) and the tape for `gradient`."""
        self.sim.bind_own_buffers()
        self.sim.restore_state(self.s0, 0)
        poses = torch.as_tensor(self.poses(theta).astype(np.float32), device=self.sim.device)
        J, tape = forward(self.sim, self.markers, poses, self.workload.frames, self.weights, self.every,
                          record=self.record)
        tape.poses = poses
        return J, tape

    def pose_gradient(self, tape):
        """dJ/d(pose) per step, (nsteps, nbones, 24) float32."""
        pb, _ = backward(self.sim, self.markers, tape.poses, self.workload.frames, tape)
        return pb

    def gradient(self, theta, tape) -> np.ndarray:
        """dJ/dtheta (8,) float64."""
        pb = self.pose_gradient(tape).double().cpu().numpy()
        jac = I.fin_pose_jacobian(np.asarray(theta, dtype=np.float64), self.workload.markers, self.steps)
        return np.einsum('nbq,nbqj->j', pb, jac)

    def close(self):
        self.sim.close()


class FinObjective(torch.autograd.Function):
    """theta (8,) -> J as a float64 scalar; backward runs the reverse sweep."""

    @staticmethod
    def forward(ctx, theta: torch.Tensor, problem: FinProblem):
        th = theta.detach().cpu().double().numpy()
        J, tape = problem.value(th)
        ctx.problem, ctx.tape, ctx.theta = problem, tape, th
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.problem.gradient(ctx.theta, ctx.tape)
        ctx.tape = None
        return torch.as_tensor(g, dtype=torch.float64) * grad_out.cpu(), None
