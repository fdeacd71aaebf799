"""Single-lattice steps captured into a HIP graph (through torch) and
replayed: every replay reproduces the eager steps bit for bit. An even number
of steps is captured, so each replay starts from the same buffer; the
library clears its maps with fill kernels, not memset nodes."""
import numpy as np
import pytest
import torch

from paper_2206_01683_amd import inputs as I
from paper_2206_01683_amd import lbm
from gpu_helpers import gpu_sim, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ib_workgroups", [0, 32])
def test_captured_steps_replay_like_eager_steps(ib_workgroups):
    """ib_workgroups = 32: one launch per step with the chain beside the
    collide, whose barrier counts carry over from replay to replay."""
    w = I.sphere_workload(nsteps=2)  # fixed sphere, fixed frames: the same two steps repeat
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses[:2], np.float32), device="cuda")
    eager = gpu_sim(w, ib_workgroups=ib_workgroups)
    wr_e = torch.zeros((2, 8), device="cuda")
    for _ in range(5):
        eager.step(w.frames[:2], dm, poses, wr_e)
    torch.cuda.synchronize()

    sim = gpu_sim(w, ib_workgroups=ib_workgroups)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    sim.set_stream(side)
    wr_g = torch.zeros((2, 8), device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        sim.step(w.frames[:2], dm, poses, wr_g)
    scratch = torch.arange(4096, dtype=torch.float32, device="cuda")
    for r in range(5):
        g.replay()
        torch.cuda.synchronize()
        scratch.mul_(1.0001).add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
    with torch.cuda.stream(side):
        got = sim.read_populations()
    side.synchronize()
    want = eager.read_populations()
    torch.cuda.synchronize()
    d = (got - want).abs().max().item()
    say(f"graph replays vs eager: max |df| = {d:.3e}")
    assert d == 0.0
    assert torch.equal(wr_g, wr_e)
    assert sim.check() == 0
