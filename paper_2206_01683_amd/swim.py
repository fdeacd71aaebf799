"""Free swimming: the fluid's force on the body drives its rigid motion, and
the local domain follows the body (Sec. III-A articulated body, Sec. III-B
localized fluid-structure interaction, the frame force of Eq. (3)).

The body's joint motion is prescribed (the travelling wave of the fish
workload); its floating base is free. Each step: the library's host dynamics
(lbm_swimmer_prepare) turns the body state and the step's shape into bone
poses and the step's frame, the GPU runs the coupled step (lbm_ib_step), and
the step's wrench comes back to advance the body (lbm_swimmer_advance). One
device-to-host copy of 8 floats per step couples the two."""
import ctypes

import numpy as np
import torch

from . import inputs as I
from . import lbm


class FreeSwimmer:
    """Host dynamics of a planar chain (lbm_swimmer_*) with the mass
    properties of the fish body of length `length` (inputs.fish_link_mass)
    at density rho_body, enclosing fluid of density rho_fluid; its mass centre
    sits at `origin` in the local domain. added_mass = 0 is explicit
    coupling, which needs rho_body somewhat above rho_fluid (1.5 and up with
    free yaw on the tests); an artificial added mass of order one (a multiple
    of the body's mass and inertia, on both sides of the update) keeps a
    neutrally buoyant body stable."""

    def __init__(self, markers, length, origin, rho_body=2.0, rho_fluid=1.0, free_yaw=True, added_mass=0.0):
        nb = markers.nbones
        mass, com, inertia, volume = I.fish_link_mass(length, nb, rho_body)
        self._arrays = [np.ascontiguousarray(a, dtype=np.float64) for a in
                        (mass, com, inertia, np.asarray(markers.joints_rest, dtype=np.float64).reshape(nb, 3))]
        ptr = [a.ctypes.data for a in self._arrays]
        self.s = lbm.Swimmer(nb, 1 if free_yaw else 0, length / nb, ptr[0], ptr[1], ptr[2], ptr[3],
                             rho_fluid / rho_body, (ctypes.c_double * 3)(*origin), float(added_mass))
        self.st = lbm.SwimmerState()
        self.nbones = nb
        self.mass = float(mass.sum())

    @staticmethod
    def _d(a):
        return np.ascontiguousarray(a, dtype=np.float64)

    def init(self, psi0, psid0, vel0=(0.0, 0.0), heading=0.0):
        v = self._d(vel0)
        p, d = self._d(psi0), self._d(psid0)
        lbm._check(lbm.lib().lbm_swimmer_init(ctypes.byref(self.s), ctypes.byref(self.st), v.ctypes.data,
                                              float(heading), p.ctypes.data, d.ctypes.data), "lbm_swimmer_init")

    def prepare(self, psi, psid):
        """(poses (nbones, 24) float32, frame (18,) float64) of the coming step."""
        poses = np.zeros((self.nbones, 24), dtype=np.float32)
        frame = lbm.Frame()
        p, d = self._d(psi), self._d(psid)
        lbm._check(lbm.lib().lbm_swimmer_prepare(ctypes.byref(self.s), ctypes.byref(self.st), p.ctypes.data,
                                                 d.ctypes.data, poses.ctypes.data, ctypes.byref(frame)),
                   "lbm_swimmer_prepare")
        return poses, np.frombuffer(frame, dtype=np.float64).copy()

    def advance(self, wrench, psi_next, psid_next):
        wr = np.ascontiguousarray(wrench, dtype=np.float32).reshape(8)
        p, d = self._d(psi_next), self._d(psid_next)
        lbm._check(lbm.lib().lbm_swimmer_advance(ctypes.byref(self.s), ctypes.byref(self.st), wr.ctypes.data,
                                                 p.ctypes.data, d.ctypes.data), "lbm_swimmer_advance")

    def state(self):
        st = self.st
        return {"vel": np.array(st.vel[:]), "acc": np.array(st.acc[:]), "heading": st.heading, "spin": st.spin,
                "ang_mom": st.ang_mom, "pos": np.array(st.pos[:])}


def swim(sim, markers_dev, swimmer: FreeSwimmer, psi, psid, nsteps):
    """Run nsteps coupled steps; psi, psid hold nsteps + 1 shapes. Returns the
    series of the body state before each step and the step wrenches."""
    dev = sim.device
    poses_dev = torch.empty((1, swimmer.nbones, 24), dtype=torch.float32, device=dev)
    pinned = torch.empty((swimmer.nbones, 24), dtype=torch.float32).pin_memory()
    wr_dev = torch.zeros((nsteps, 8), dtype=torch.float32, device=dev)
    wr_host = torch.empty(8, dtype=torch.float32).pin_memory()
    out = {"vel": [], "heading": [], "spin": [], "pos": [], "wrench": np.zeros((nsteps, 8)), "frames": []}
    for n in range(nsteps):
        st = swimmer.state()
        for k in ("vel", "heading", "spin", "pos"):
            out[k].append(st[k])
        poses, frame = swimmer.prepare(psi[n], psid[n])
        out["frames"].append(frame)
        pinned.numpy()[...] = poses
        poses_dev[0].copy_(pinned, non_blocking=True)
        sim.step(frame.reshape(1, 18), markers_dev, poses_dev, wr_dev[n:n + 1])
        wr_host.copy_(wr_dev[n], non_blocking=True)
        torch.cuda.current_stream(dev).synchronize()
        w = wr_host.numpy().copy()
        out["wrench"][n] = w
        swimmer.advance(w, psi[n + 1], psid[n + 1])
    for k in ("vel", "heading", "spin", "pos"):
        out[k] = np.array(out[k])
    out["frames"] = np.array(out["frames"])
    return out
