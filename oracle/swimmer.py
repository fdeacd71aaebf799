"""FP64 oracle of free swimming (TEST INFRASTRUCTURE ONLY: tests and the
smoke check use it; the product never does): the whole-body momentum balance
of a planar chain with prescribed joint motion, coupled step by step to the
FP64 fluid oracle (lbm_oracle.cpp).

Model (the articulated body of Sec. III-A with every joint prescribed, the
fluid force as the external generalized force of Eq. (1), the local domain of
Sec. III-B following the body's mass centre):
  M dV/dt = F,   d/dt (I_c theta' + L_s) = T   (about the mass centre),
stepped with r = rho_fluid / rho_body (the enclosed fluid's share) and an
artificial added mass k (a multiple of the body's mass and inertia, put on
both sides of the update; k = 0 is explicit coupling). Translation: the body
with the extra mass k M, driven by the step's force plus the extra mass times
the previous acceleration,
  (M + k M) a(n+1) = F(n) + (r M + k M) a(n),   V(n+1) = V(n) + a(n);
rotation: the angular momentum of the body and the extra inertia k I_c,
  L(n+1) + k I_c' (theta'(n+1) - theta'(n)) = L(n) + T(n) + (r I_c + k I_c') (theta'(n) - theta'(n-1)),
  L = I_c theta' + L_s (I_c' the next shape's), theta(n+1) = theta(n) + theta'(n+1);
with the yaw held, theta' = 0 and L = L_s.
Planar vectors are complex numbers here: rotation is multiplication by
exp(i theta) and the z cross product is Im(conj(a) b)."""
import numpy as np

from . import run as _fluid_run


class Body:
    def __init__(self, h, mass, com, inertia, joints_rest, fluid_ratio, origin, free_yaw=True, added_mass=0.0):
        self.h = float(h)
        self.mass = np.asarray(mass, dtype=np.float64)
        self.com = np.asarray(com, dtype=np.float64)
        self.inertia = np.asarray(inertia, dtype=np.float64)
        self.joints_rest = np.asarray(joints_rest, dtype=np.float64).reshape(-1, 3)
        self.fluid_ratio = float(fluid_ratio)
        self.origin = np.asarray(origin, dtype=np.float64)
        self.free_yaw = bool(free_yaw)
        self.added_mass = float(added_mass)
        self.M = float(self.mass.sum())


def shape(body, psi, psid):
    """Joint positions J and rates (complex, body frame, head joint at 0),
    mass centre rc, rcd, I_c and L_s of the chain with link headings psi."""
    e = np.exp(1j * np.asarray(psi, dtype=np.float64))
    ed = 1j * np.asarray(psid, dtype=np.float64) * e
    steps = body.h * e
    J = np.concatenate([[0.0 + 0.0j], np.cumsum(steps)[:-1]])
    Jd = np.concatenate([[0.0 + 0.0j], np.cumsum(body.h * ed)[:-1]])
    r = J + body.com * e
    rd = Jd + body.com * ed
    rc = (body.mass * r).sum() / body.M
    rcd = (body.mass * rd).sum() / body.M
    q, qd = r - rc, rd - rcd
    Ic = (body.inertia + body.mass * np.abs(q) ** 2).sum()
    Ls = (body.inertia * psid + body.mass * np.imag(np.conj(q) * qd)).sum()
    return J, Jd, rc, rcd, Ic, Ls


def init(body, psi0, psid0, vel0=(0.0, 0.0), heading=0.0):
    *_, Ic, Ls = shape(body, psi0, psid0)
    return {"vel": complex(vel0[0], vel0[1]), "acc": 0j, "heading": float(heading), "spin": 0.0, "spin_prev": 0.0,
            "ang_mom": Ls, "inertia": Ic, "pos": 0j}


def prepare(body, st, psi, psid):
    """Bone poses (nbones, 24) and the frame (18,) of the coming step."""
    J, Jd, rc, rcd, _, _ = shape(body, psi, psid)
    rot = np.exp(1j * st["heading"])
    d = rot * (J - rc)                                   # joints relative to the mass centre, in the frame
    dv = 1j * st["spin"] * d + rot * (Jd - rcd)          # their velocities relative to the frame
    nb = len(psi)
    poses = np.zeros((nb, 24))
    for j in range(nb):
        a = st["heading"] + psi[j]
        w = st["spin"] + psid[j]
        R = np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])
        Rd = w * np.array([[-np.sin(a), -np.cos(a), 0.0], [np.cos(a), -np.sin(a), 0.0], [0.0, 0.0, 0.0]])
        P = body.origin + np.array([d[j].real, d[j].imag, 0.0])
        Pd = np.array([dv[j].real, dv[j].imag, 0.0])
        Jr = body.joints_rest[j]
        poses[j, 0:9] = R.ravel()
        poses[j, 9:12] = P - R @ Jr
        poses[j, 12:21] = Rd.ravel()
        poses[j, 21:24] = Pd - Rd @ Jr
    v, a = st["vel"], st["acc"]
    frame = np.zeros(18)
    frame[0:3] = (a.real, a.imag, 0.0)
    frame[9:12] = body.origin
    frame[12:15] = (-v.real, -v.imag, 0.0)
    frame[15:18] = frame[12:15]
    return poses, frame


def advance(body, st, wrench, psi_next, psid_next):
    F = complex(wrench[0], wrench[1])
    r, k, M = body.fluid_ratio, body.added_mass, body.M
    a = st["acc"]
    st["vel"] = st["vel"] + a
    st["pos"] = st["pos"] + st["vel"]
    st["acc"] = (F + (r * M + k * M) * a) / (M + k * M)
    *_, Ic, Ls = shape(body, psi_next, psid_next)
    if body.free_yaw:
        # unknown w = theta'(n+1): Ic w + Ls + k Ic (w - theta'(n)) = L(n) + T(n) + (r I_c(n) + k Ic) theta''(n)
        dw = st["spin"] - st["spin_prev"]
        budget = st["ang_mom"] + float(wrench[5]) + (r * st["inertia"] + k * Ic) * dw
        w = (budget - Ls + k * Ic * st["spin"]) / (Ic + k * Ic)
        st["spin_prev"] = st["spin"]
        st["spin"] = w
        st["ang_mom"] = Ic * w + Ls
        st["heading"] = st["heading"] + w
    else:
        st["spin"] = st["spin_prev"] = 0.0
        st["ang_mom"] = Ls
    st["inertia"] = Ic
    return st


def coupled_run(prm, f, markers, body, psi, psid, nsteps, vel0=(0.0, 0.0), heading=0.0):
    """nsteps coupled steps with the fluid oracle; f is advanced in place.
    Returns the body-state series (before each step), the wrenches and f."""
    st = init(body, psi[0], psid[0], vel0, heading)
    out = {"vel": [], "heading": [], "spin": [], "pos": [], "wrench": np.zeros((nsteps, 8))}
    for n in range(nsteps):
        for k in ("vel", "heading", "spin", "pos"):
            out[k].append(st[k])
        poses, frame = prepare(body, st, psi[n], psid[n])
        res = _fluid_run(prm, f, frame.reshape(1, 18), markers, poses.reshape(1, -1, 24), 1)
        f = res["f"]
        out["wrench"][n] = res["wrench"][0]
        advance(body, st, res["wrench"][0], psi[n + 1], psid[n + 1])
    out["vel"] = np.array([[v.real, v.imag] for v in out["vel"]])
    out["pos"] = np.array([[p.real, p.imag] for p in out["pos"]])
    out["heading"] = np.array(out["heading"])
    out["spin"] = np.array(out["spin"])
    out["f"] = f
    return out
