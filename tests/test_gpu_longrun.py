"""Long run of the full fish workload (384x192x192, 12,000 markers, the
bench's configuration) with FP32, FP16 and BF16 population storage against
the FP64 oracle: relative L2 of the velocity at steps 100, 500 and the last,
and the error of the time-averaged thrust over the last 400 steps.

Opt-in (LBMIB_LONG=1): the oracle alone takes about 35 s per 50 steps on 16
host cores, so 1,000 steps (LBMIB_LONG_STEPS) take about 10 minutes. The
oracle runs in 50-step chunks and prints after each one."""
import os
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2206_01683_amd import inputs as I
from gpu_helpers import gpu_sim, interior, rel_l2, say

pytestmark = pytest.mark.gpu

STEPS = int(os.environ.get("LBMIB_LONG_STEPS", "1000"))
MARKS = sorted({100, 500, STEPS})
CHUNK = 50


def _thrust(wrench, heading):
    return np.asarray(wrench, dtype=np.float64)[:, :3] @ np.asarray(heading, dtype=np.float64)


def _gpu(w, storage):
    sim = gpu_sim(w, storage=storage)
    from paper_2206_01683_amd import lbm
    dm = lbm.DeviceMarkers(w.markers)
    poses = torch.as_tensor(np.ascontiguousarray(w.poses[:STEPS], np.float32), device="cuda")
    wr = torch.zeros((STEPS, 8), dtype=torch.float32, device="cuda")
    fields, done = {}, 0
    for m in MARKS:
        sim.step(w.frames[done:m], dm, poses[done:m], wr[done:m])
        done = m
        _, u = sim.macros(w.frames[min(m, STEPS - 1)])
        fields[m] = u.cpu().numpy().astype(np.float64)
    assert sim.check() == 0
    out = wr.cpu().numpy()
    sim.close()
    return fields, out


@pytest.mark.skipif(os.environ.get("LBMIB_LONG") != "1", reason="long run: about 10 minutes of FP64 oracle on the "
                    "host cores; set LBMIB_LONG=1")
@pytest.mark.timeout(3000)
def test_fish_long_run_precision_report():
    w = I.fish_workload(nsteps=STEPS)
    gpu = {st: _gpu(w, st) for st in ("f32", "f16", "bf16")}
    say(f"GPU runs done ({STEPS} steps each, FP32/FP16/BF16)")
    prm = oracle.params(w.nx, w.ny, w.nz, w.tau, w.bc_lo, w.bc_hi, w.mdf_iters, w.ib_alpha, w.bc_y, w.bc_z)
    f = oracle.equilibrium_field(np.ones((w.nz, w.ny, w.nx)), w.u0.astype(np.float32).astype(np.float64))
    ref_u, ref_w = {}, np.zeros((STEPS, 8))
    t0 = time.time()
    for s in range(0, STEPS, CHUNK):
        e = min(STEPS, s + CHUNK)
        res = oracle.run(prm, f, w.frames[s:e], w.markers, w.poses[s:e], e - s)
        f = res["f"]
        ref_w[s:e] = res["wrench"]
        say(f"oracle step {e}/{STEPS}, {time.time() - t0:.0f} s")
        if e in MARKS:
            _, u = oracle.macros(prm, f, w.frames[min(e, STEPS - 1)])
            ref_u[e] = u
    tail = slice(max(0, STEPS - 400), STEPS)
    t_ref = _thrust(ref_w[tail], w.heading).mean()
    report = {}
    for st, (fields, wr) in gpu.items():
        errs = [rel_l2(interior(fields[m], w), interior(ref_u[m], w)) for m in MARKS]
        t_err = abs(_thrust(wr[tail], w.heading).mean() - t_ref) / abs(t_ref)
        report[st] = (errs, t_err)
        say(f"{st}: velocity rel L2 at steps {MARKS}: " + ", ".join(f"{x:.2e}" for x in errs) +
            f"; mean thrust over the last 400 steps rel err {t_err:.2e} (oracle mean thrust {t_ref:.4e})")
    # measured on one MI355X, 1,000 steps: FP32 1.4e-6 / 5.6e-6 / 8.8e-6, mean thrust 3e-5
    assert max(report["f32"][0]) <= 2e-5 and report["f32"][1] <= 2e-4
    for j in range(len(MARKS)):
        assert report["f32"][0][j] < report["f16"][0][j] < report["bf16"][0][j]
