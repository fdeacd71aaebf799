"""Seeded synthetic inputs for the immersed-boundary lattice Boltzmann step.

This module holds geometry, kinematics and random draws only. It contains no
lattice Boltzmann or immersed-boundary arithmetic, so it can feed both the HIP
path and the FP64 oracle without the two sharing any of the method.

Everything is in lattice units (cell spacing 1, time step 1). Arrays follow
the layouts of the library's C interface:
  * marker arrays are structure-of-arrays, shape (3, n) / (2, n) / (n,);
  * a bone pose is 24 numbers: R (3x3 row-major), t (3), dR/dt (3x3
    row-major), dt/dt (3), mapping rest-pose coordinates to the current pose
    (linear blend skinning, paper Sec. III-A);
  * a frame is 18 numbers: frame linear acceleration (3), angular velocity
    (3), angular acceleration (3), origin x0 (3), velocity prescribed on the
    x = 0 face (3) and on the x = nx-1 face (3) (paper Eq. (3)).

The paper's fish meshes, skeletons and policies are not available, so the
fish here is synthetic: an elliptic-section body on a serial chain of ten
revolute joints about z (paper Sec. III-A describes bones joined by joints
with a linear-blend-skinned surface; Fig. 2 shows several topologies).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

FRAME_FIELDS = 18
POSE_FIELDS = 24

BC_PERIODIC = 0
BC_VELOCITY = 1
BC_OUTFLOW = 2


# --------------------------------------------------------------------------
# frames (paper Eq. (3))
# --------------------------------------------------------------------------
def make_frames(nsteps: int, acc=None, omega=None, alpha=None, origin=None, u_lo=None, u_hi=None) -> np.ndarray:
    """Per-step frames, shape (nsteps, 18) float64. Each argument is either a
    3-vector (constant) or an (nsteps, 3) array; missing ones are zero."""
    fr = np.zeros((nsteps, FRAME_FIELDS), dtype=np.float64)
    for j, v in enumerate((acc, omega, alpha, origin, u_lo, u_hi)):
        if v is None:
            continue
        fr[:, 3 * j:3 * j + 3] = np.broadcast_to(np.asarray(v, dtype=np.float64), (nsteps, 3))
    return fr


def accelerating_frames(nsteps: int, a0: float, period: float, origin, start: int = 0) -> np.ndarray:
    """Frame accelerating along x with a(n) = a0 sin(2 pi n / period).

    The local domain moves with the body, so the far field, at rest in the
    lab, enters through the x faces with the frame's velocity reversed:
    u_face(n) = -V(n) e_x with V(n) = sum_{m<n} a(m) (paper Sec. III-B,
    localized moving domain). Both x faces get that velocity; which of them is
    a velocity face is the caller's boundary choice.
    """
    n = np.arange(start, start + nsteps, dtype=np.float64)
    a = a0 * np.sin(2.0 * math.pi * n / period)
    allsteps = a0 * np.sin(2.0 * math.pi * np.arange(0, start + nsteps, dtype=np.float64) / period)
    V = np.concatenate([[0.0], np.cumsum(allsteps)])[start:start + nsteps]
    acc = np.stack([a, np.zeros_like(a), np.zeros_like(a)], axis=1)
    u = np.stack([-V, np.zeros_like(V), np.zeros_like(V)], axis=1)
    return make_frames(nsteps, acc=acc, origin=origin, u_lo=u, u_hi=u)


# --------------------------------------------------------------------------
# random fields
# --------------------------------------------------------------------------
def perturbed_velocity(shape_zyx, u0, amp: float, seed: int) -> np.ndarray:
    """u0 + delta u with delta u ~ U[-amp, amp] per component per node,
    drawn with numpy's default_rng(seed) as one array of shape (3, nz, ny, nx)."""
    nz, ny, nx = shape_zyx
    rng = np.random.default_rng(seed)
    du = rng.uniform(-amp, amp, size=(3, nz, ny, nx)) if amp > 0 else np.zeros((3, nz, ny, nx))
    u = du + np.asarray(u0, dtype=np.float64).reshape(3, 1, 1, 1)
    return u


def random_density(shape_zyx, amp: float, seed: int) -> np.ndarray:
    """1 + delta rho, delta rho ~ U[-amp, amp]."""
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amp, amp, size=tuple(shape_zyx))


def random_offsets(shape, amp: float, seed: int) -> np.ndarray:
    """Uniform noise U[-amp, amp] of the given shape (used to add a
    non-equilibrium part to test populations)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=tuple(shape))


# --------------------------------------------------------------------------
# markers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class MarkerSet:
    """Lagrangian surface markers with their skin (paper Sec. III-B: the
    surface is uniformly sampled before simulation)."""
    xrest: np.ndarray   # (3, n) float64 rest-pose positions
    bone: np.ndarray    # (2, n) int32
    weight: np.ndarray  # (2, n) float64
    dv: np.ndarray      # (n,) float64
    nbones: int
    area: float
    joints_rest: Optional[np.ndarray] = None  # (nbones, 3) rest joint positions
    normals: Optional[np.ndarray] = None      # (3, n) rest-pose outward unit normals

    @property
    def n(self) -> int:
        return self.xrest.shape[1]


def fibonacci_sphere(n: int, radius: float, center) -> MarkerSet:
    """Fibonacci sphere: z_k = 1 - (2k+1)/n, rho_k = sqrt(1 - z_k^2),
    phi_k = k pi (3 - sqrt 5), X_k = c + R (rho_k cos phi_k, rho_k sin phi_k, z_k).
    One bone (identity pose keeps it fixed); dV = 4 pi R^2 / n."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    r = np.sqrt(1.0 - z * z)
    ph = k * math.pi * (3.0 - math.sqrt(5.0))
    c = np.asarray(center, dtype=np.float64)
    x = np.stack([c[0] + radius * r * np.cos(ph), c[1] + radius * r * np.sin(ph), c[2] + radius * z])
    area = 4.0 * math.pi * radius * radius
    normals = np.stack([r * np.cos(ph), r * np.sin(ph), z])
    return MarkerSet(xrest=x, bone=np.zeros((2, n), np.int32), weight=np.stack([np.ones(n), np.zeros(n)]),
                     dv=np.full(n, area / n), nbones=1, area=area, normals=normals)


def fish_half_width(xi: np.ndarray, length: float) -> np.ndarray:
    """b(xi) = 0.08 L sqrt(xi) (1 - xi) / 0.3849, maximal (0.08 L) at xi = 1/3."""
    peak = math.sqrt(1.0 / 3.0) * (2.0 / 3.0)
    return 0.08 * length * np.sqrt(np.clip(xi, 0.0, 1.0)) * (1.0 - xi) / peak


def fish_link_mass(length: float, nbones: int = 10, rho: float = 1.0, nq: int = 4000):
    """Mass properties of the fish body of fish_surface cut into nbones equal
    links (density rho): per link its mass, the distance of its mass centre
    from its proximal joint along the body axis, and its moment of inertia
    about z through that centre (axial spread plus the elliptic section's
    lateral spread b^2 / 4). Midpoint quadrature with nq points per link.
    Also returns the body volume."""
    h = length / nbones
    mass, com, inertia = np.zeros(nbones), np.zeros(nbones), np.zeros(nbones)
    for j in range(nbones):
        s = j * h + (np.arange(nq) + 0.5) * (h / nq)
        b = fish_half_width(s / length, length)
        area = math.pi * b * 1.5 * b
        dm = rho * area * (h / nq)
        mass[j] = dm.sum()
        com[j] = ((s - j * h) * dm).sum() / mass[j]
        inertia[j] = (((s - j * h - com[j]) ** 2 + b * b / 4.0) * dm).sum()
    return mass, com, inertia, float(mass.sum() / rho)


def _ellipse_perimeter(a, b):
    # Ramanujan's second approximation
    h = ((a - b) / np.maximum(a + b, 1e-300)) ** 2
    return math.pi * (a + b) * (1.0 + 3.0 * h / (10.0 + np.sqrt(4.0 - 3.0 * h)))


def fish_surface(n: int, length: float, head, nbones: int = 10) -> MarkerSet:
    """Synthetic fish: body along +x from the head (so it heads toward -x),
    elliptic cross-section with half-width b(xi) in y and half-height 1.5 b(xi)
    in z. Markers are placed area-uniformly: xi_k from the inverse of the
    cumulative surface area at (k + 1/2)/n, angle k times the golden angle;
    dV_k = A / n. Skeleton: nbones bones of length L/nbones, joints at
    s_j = j L / nbones. Skin: with u = s / (L/nbones) - 1/2, b0 = floor(u),
    t = u - b0, weight (1 - t) on bone b0 and t on bone b0 + 1, clamped at the
    ends."""
    head = np.asarray(head, dtype=np.float64)
    xi = np.linspace(0.0, 1.0, 200001)
    b = fish_half_width(xi, length)
    per = _ellipse_perimeter(b, 1.5 * b)
    ds = length * (xi[1] - xi[0])
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (per[1:] + per[:-1]) * ds)])
    area = float(cum[-1])
    k = np.arange(n, dtype=np.float64)
    xik = np.interp((k + 0.5) / n * area, cum, xi)
    ang = k * math.pi * (3.0 - math.sqrt(5.0))
    bk = fish_half_width(xik, length)
    x = np.stack([head[0] + xik * length, head[1] + bk * np.cos(ang), head[2] + 1.5 * bk * np.sin(ang)])
    h = length / nbones
    u = xik * length / h - 0.5
    b0 = np.floor(u).astype(np.int64)
    t = u - b0
    lo = b0 < 0
    hi = b0 >= nbones - 1
    b0c = np.clip(b0, 0, nbones - 1)
    b1c = np.clip(b0 + 1, 0, nbones - 1)
    w0 = np.where(lo | hi, 1.0, 1.0 - t)
    w1 = np.where(lo | hi, 0.0, t)
    bone = np.stack([b0c, b1c]).astype(np.int32)
    weight = np.stack([w0, w1])
    joints = np.stack([head + np.array([j * h, 0.0, 0.0]) for j in range(nbones)])
    # outward normal of S(xi, a) = (xi L, b cos a, 1.5 b sin a): along
    # dS/da x dS/dxi, proportional to (-1.5 b', 1.5 L cos a, L sin a), b' = db/dxi
    peak = math.sqrt(1.0 / 3.0) * (2.0 / 3.0)
    sq = np.sqrt(np.maximum(xik, 1e-300))
    db = 0.08 * length / peak * ((1.0 - xik) / (2.0 * sq) - sq)
    nv = np.stack([-1.5 * db, 1.5 * length * np.cos(ang), length * np.sin(ang)])
    nv /= np.linalg.norm(nv, axis=0, keepdims=True)
    return MarkerSet(xrest=x, bone=bone, weight=weight, dv=np.full(n, area / n), nbones=nbones, area=area,
                     joints_rest=joints, normals=nv)


# --------------------------------------------------------------------------
# skeleton kinematics (forward kinematics of the serial chain)
# --------------------------------------------------------------------------
def identity_poses(nsteps: int, nbones: int = 1) -> np.ndarray:
    p = np.zeros((nsteps, nbones, POSE_FIELDS))
    p[:, :, 0] = p[:, :, 4] = p[:, :, 8] = 1.0
    return p


def chain_poses(psi: np.ndarray, psidot: np.ndarray, joints_rest: np.ndarray) -> np.ndarray:
    """Bone poses of a planar serial chain whose root joint stays fixed.

    psi[n, j] is the heading of bone j about z (cumulative joint angle) and
    psidot its rate. Joint positions follow J_{j+1} = J_j + h (cos psi_j,
    sin psi_j, 0) from J_0 = rest root, h = rest bone length. Bone j maps a
    rest point xbar to R_j (xbar - Jbar_j) + J_j, with R_j the rotation by
    psi_j about z. Returns (nsteps, nbones, 24)."""
    nsteps, nb = psi.shape
    dt = np.result_type(psi, psidot, np.float64)  # complex when differentiating by complex step
    jr = np.asarray(joints_rest, dtype=np.float64)
    h = float(jr[1, 0] - jr[0, 0]) if nb > 1 else 1.0
    out = np.zeros((nsteps, nb, POSE_FIELDS), dtype=dt)
    J = np.repeat(jr[0][None, :], nsteps, axis=0).astype(dt)
    Jd = np.zeros((nsteps, 3), dtype=dt)
    for j in range(nb):
        c, s = np.cos(psi[:, j]), np.sin(psi[:, j])
        d = psidot[:, j]
        R = np.zeros((nsteps, 3, 3), dtype=dt)
        R[:, 0, 0], R[:, 0, 1], R[:, 1, 0], R[:, 1, 1], R[:, 2, 2] = c, -s, s, c, 1.0
        Rd = np.zeros((nsteps, 3, 3), dtype=dt)
        Rd[:, 0, 0], Rd[:, 0, 1], Rd[:, 1, 0], Rd[:, 1, 1] = -s * d, -c * d, c * d, -s * d
        t = J - np.einsum('nab,b->na', R, jr[j])
        td = Jd - np.einsum('nab,b->na', Rd, jr[j])
        out[:, j, 0:9] = R.reshape(nsteps, 9)
        out[:, j, 9:12] = t
        out[:, j, 12:21] = Rd.reshape(nsteps, 9)
        out[:, j, 21:24] = td
        J = J + h * np.stack([c, s, np.zeros_like(c)], axis=1)
        Jd = Jd + h * np.stack([-s * d, c * d, np.zeros_like(c)], axis=1)
    return out


def wave_headings(length: float, nbones: int, steps: np.ndarray, amp_frac: float = 0.1,
                  period: float = 400.0, wavelength_frac: float = 1.0):
    """Bone headings from a travelling body wave y(s, n) = amp_frac L (s/L)^2
    sin(2 pi (s/(wavelength_frac L) - n/period)): psi_j = atan2(y(s_{j+1}) -
    y(s_j), h) with its analytic rate."""
    h = length / nbones
    n = np.asarray(steps, dtype=np.float64)[:, None]
    s0 = np.arange(nbones)[None, :] * h
    s1 = s0 + h

    def y(s):
        return amp_frac * length * (s / length) ** 2 * np.sin(2 * math.pi * (s / (wavelength_frac * length) - n / period))

    def ydot(s):
        return amp_frac * length * (s / length) ** 2 * np.cos(
            2 * math.pi * (s / (wavelength_frac * length) - n / period)) * (-2 * math.pi / period)

    dy = y(s1) - y(s0)
    dyd = ydot(s1) - ydot(s0)
    psi = np.arctan2(dy, h)
    psid = h * dyd / (h * h + dy * dy)
    return psi, psid


C5_PARAM_NAMES = ("A1", "A2", "A3", "f", "phi2", "phi3", "At", "phit")
C5_BASE = np.array([0.15, 0.2, 0.3, 1.0, 0.0, 0.0, 0.4, 0.0])


def fin_joint_angles(params, steps: np.ndarray, nbones: int = 10, period: float = 400.0):
    """Joint angles of the differentiation workload from 8 kinematics
    parameters (A1, A2, A3, f, phi2, phi3, At, phit):
      theta_j(n) = A_seg(j) sin(2 pi f n / period - 2 pi j / 10 + phi_seg(j)),
      j = 0..8 with segments {0-2}, {3-5}, {6-8} (phi1 = 0), and the tail
      theta_9(n) = At sin(2 pi f n / period - 1.8 pi + phit).
    Returns (theta, thetadot), each (nsteps, nbones)."""
    A1, A2, A3, f, p2, p3, At, pt = list(np.asarray(params).ravel())
    n = np.asarray(steps, dtype=np.float64)[:, None]
    j = np.arange(nbones)[None, :]
    seg = np.minimum(j // 3, 2)
    dt = np.result_type(np.asarray(params), np.float64)
    A = np.choose(seg, [A1, A2, A3]).astype(dt)
    ph = np.choose(seg, [0.0, p2, p3]).astype(dt)
    w = 2 * math.pi * f / period
    arg = w * n - 2 * math.pi * j / 10.0 + ph
    th = A * np.sin(arg)
    thd = A * w * np.cos(arg)
    tail = nbones - 1
    arg_t = w * n[:, 0] - 1.8 * math.pi + pt
    th[:, tail] = At * np.sin(arg_t)
    thd[:, tail] = At * w * np.cos(arg_t)
    return th, thd


def fin_poses(params, ms: MarkerSet, steps, period: float = 400.0):
    """Bone poses of the differentiation workload for kinematics parameters."""
    th, thd = fin_joint_angles(params, steps, ms.nbones, period)
    psi, psid = headings_from_joint_angles(th, thd)
    return chain_poses(psi, psid, ms.joints_rest)


def fin_pose_jacobian(params, ms: MarkerSet, steps, period: float = 400.0, h: float = 1e-20):
    """d(bone poses)/d(params), shape (nsteps, nbones, 24, 8), by the complex
    step: the kinematics are analytic in the parameters, so Im(pose(p + i h
    e_j))/h is the derivative to machine precision."""
    p = np.asarray(params, dtype=np.float64)
    out = np.zeros((len(steps), ms.nbones, POSE_FIELDS, p.size))
    for j in range(p.size):
        pc = p.astype(np.complex128)
        pc[j] += 1j * h
        out[..., j] = np.imag(fin_poses(pc, ms, steps, period)) / h
    return out


def headings_from_joint_angles(theta, thetadot):
    return np.cumsum(theta, axis=1), np.cumsum(thetadot, axis=1)


def ramp_joint_angles(targets, steps, ramp: float = 50.0):
    """theta_j(n) = target_j (1 - cos(pi min(n/ramp, 1))) / 2 and its rate."""
    n = np.asarray(steps, dtype=np.float64)[:, None]
    s = np.minimum(n / ramp, 1.0)
    th = np.asarray(targets)[None, :] * 0.5 * (1.0 - np.cos(math.pi * s))
    thd = np.where(n < ramp, np.asarray(targets)[None, :] * 0.5 * math.pi / ramp * np.sin(math.pi * s), 0.0)
    return th, thd


def skin_positions(ms: MarkerSet, pose: np.ndarray) -> np.ndarray:
    """Marker positions of one pose (used only to check that a workload keeps
    its markers inside the domain)."""
    X = np.zeros((3, ms.n))
    for j in range(2):
        P = pose[ms.bone[j]]
        R = P[:, 0:9].reshape(-1, 3, 3)
        X += ms.weight[j] * (np.einsum('kab,bk->ak', R, ms.xrest) + P[:, 9:12].T)
    return X


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    tau: float
    bc_lo: int
    bc_hi: int
    nsteps: int
    u0: np.ndarray                 # (3, nz, ny, nx) initial velocity
    markers: Optional[MarkerSet]
    poses: np.ndarray              # (nsteps, nbones, 24)
    frames: np.ndarray             # (nsteps, 18)
    heading: np.ndarray            # unit vector the body swims toward
    mdf_iters: int = 1
    ib_alpha: float = 1.0
    meta: dict = dataclasses.field(default_factory=dict)
    bc_y: tuple = (BC_PERIODIC, BC_PERIODIC)  # y = 0, y = ny-1
    bc_z: tuple = (BC_PERIODIC, BC_PERIODIC)  # z = 0, z = nz-1
    ib_scheme: int = 0                        # 0 direct forcing, 1 implicit velocity correction
    collision: int = 0                        # 0 BGK, 1 two-relaxation-time
    trt_lambda: float = 3.0 / 16.0            # TRT: (tau - 1/2)(tau- - 1/2)
    wall_mode: int = 0                        # 0 no-slip, 1 slip (normal component only)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


def sphere_workload(nsteps: int = 100, seed: int = 0) -> Workload:
    """Plain method, small: 64x32x32, tau = 0.6, periodic y and z, velocity
    inlet u = (0.05, 0, 0) at x = 0 and zero-gradient outlet at x = 63, initial
    velocity u0 plus seeded U[-1e-3, 1e-3] noise, fixed sphere of radius 6 at
    (20, 16, 16) with 500 Fibonacci markers."""
    nx, ny, nz = 64, 32, 32
    u_in = np.array([0.05, 0.0, 0.0])
    u0 = perturbed_velocity((nz, ny, nx), u_in, 1e-3, seed)
    ms = fibonacci_sphere(500, 6.0, (20.0, 16.0, 16.0))
    frames = make_frames(nsteps, origin=(20.0, 16.0, 16.0), u_lo=u_in, u_hi=u_in)
    return Workload("sphere-64x32x32", nx, ny, nz, 0.6, BC_VELOCITY, BC_OUTFLOW, nsteps, u0, ms,
                    identity_poses(nsteps, 1), frames, heading=np.array([-1.0, 0.0, 0.0]))


def _fish_workload(name, nx, ny, nz, length, n, head, nsteps, psi, psid, frames, tau=0.6, u0=None,
                   bc=(BC_VELOCITY, BC_OUTFLOW)):
    ms = fish_surface(n, length, head)
    poses = chain_poses(psi, psid, ms.joints_rest)
    if u0 is None:
        u0 = np.zeros((3, nz, ny, nx))
    return Workload(name, nx, ny, nz, tau, bc[0], bc[1], nsteps, u0, ms, poses, frames,
                    heading=np.array([-1.0, 0.0, 0.0]))


def fish_workload(nsteps: int = 2000, start: int = 0, nx: int = 384, ny: int = 192, nz: int = 192,
                  length: float = 96.0, n: int = 12000, head=(112.0, 96.0, 96.0)) -> Workload:
    """Single fish in an accelerating local frame: 384x192x192, 12,000
    markers on a 10-joint chain of length 96, travelling wave of amplitude
    0.1 L (s/L)^2, period 400 steps, wavelength L; frame acceleration
    a(n) = 1e-5 sin(2 pi n / 400) along x; velocity inlet at x = 0,
    zero-gradient outlet at x = nx-1; fluid initially at rest."""
    steps = np.arange(start, start + nsteps)
    psi, psid = wave_headings(length, 10, steps)
    ms = fish_surface(n, length, head)
    origin = ms.xrest.mean(axis=1)
    frames = accelerating_frames(nsteps, 1e-5, 400.0, origin, start=start)
    w = _fish_workload(f"fish-{nx}x{ny}x{nz}", nx, ny, nz, length, n, head, nsteps, psi, psid, frames)
    w.meta.update(start=start)
    return w


def fin_workload(params=C5_BASE, nsteps: int = 400, nx: int = 128, ny: int = 64, nz: int = 64,
                 length: float = 48.0, n: int = 3000, head=(40.0, 32.0, 32.0)) -> Workload:
    """Differentiation workload: 128x64x64, 3,000-marker fish of length 48,
    joint angles from the 8 kinematics parameters (fin_joint_angles), inflow
    u = (0.05, 0, 0), zero-gradient outlet, fluid initially at the inflow
    velocity, 400 steps."""
    steps = np.arange(nsteps)
    th, thd = fin_joint_angles(params, steps)
    psi, psid = headings_from_joint_angles(th, thd)
    u_in = np.array([0.05, 0.0, 0.0])
    ms = fish_surface(n, length, head)
    frames = make_frames(nsteps, origin=ms.xrest.mean(axis=1), u_lo=u_in, u_hi=u_in)
    u0 = np.broadcast_to(u_in.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
    w = _fish_workload(f"fin-{nx}x{ny}x{nz}", nx, ny, nz, length, n, head, nsteps, psi, psid, frames, u0=u0)
    w.meta.update(params=np.asarray(params, dtype=np.float64))
    return w


def merge_marker_sets(sets) -> MarkerSet:
    """One marker set of several bodies: markers concatenated in order, bone
    indices of body j shifted by the bone counts of bodies 0 .. j-1."""
    off = np.cumsum([0] + [m.nbones for m in sets])
    joints = [m.joints_rest for m in sets]
    return MarkerSet(xrest=np.concatenate([m.xrest for m in sets], axis=1),
                     bone=np.concatenate([m.bone + off[j] for j, m in enumerate(sets)], axis=1).astype(np.int32),
                     weight=np.concatenate([m.weight for m in sets], axis=1),
                     dv=np.concatenate([m.dv for m in sets]), nbones=int(off[-1]),
                     area=float(sum(m.area for m in sets)),
                     joints_rest=None if any(j is None for j in joints) else np.concatenate(joints, axis=0),
                     normals=None if any(m.normals is None for m in sets) else
                     np.concatenate([m.normals for m in sets], axis=1))


def two_fish_workload(nsteps: int = 400, nx: int = 150, ny: int = 50, nz: int = 100, length: float = 40.0,
                      n: int = 2000, u_in: float = 0.04, lag: float = 0.25) -> Workload:
    """Two swimmers in one domain (the paper's two-fish domain, 150x50x100):
    fish of length 40 with 2,000 markers each, heads at (40, ny/2, nz/3) and
    (50, ny/2, 2 nz/3), both bending in the x-y plane with the travelling wave
    of fish_workload (period 400 steps), the second lagging by `lag` of a
    period. Inertial frame, inflow u = (u_in, 0, 0) at x = 0, zero-gradient
    outlet, fluid initially at the inflow velocity, tau = 0.6. One marker set
    of 20 bones: fish j owns bones 10 j .. 10 j + 9 and markers
    n j .. n j + n - 1 (meta['fish_bones'], meta['fish_markers'])."""
    steps = np.arange(nsteps)
    heads = [(40.0, ny / 2.0, nz / 3.0), (50.0, ny / 2.0, 2.0 * nz / 3.0)]
    sets, poses = [], []
    for j, head in enumerate(heads):
        ms = fish_surface(n, length, head)
        psi, psid = wave_headings(length, 10, steps - lag * 400.0 * j)
        poses.append(chain_poses(psi, psid, ms.joints_rest))
        sets.append(ms)
    ms = merge_marker_sets(sets)
    uv = np.array([u_in, 0.0, 0.0])
    frames = make_frames(nsteps, origin=ms.xrest.mean(axis=1), u_lo=uv, u_hi=uv)
    u0 = np.broadcast_to(uv.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
    w = Workload(f"two-fish-{nx}x{ny}x{nz}", nx, ny, nz, 0.6, BC_VELOCITY, BC_OUTFLOW, nsteps, u0, ms,
                 np.concatenate(poses, axis=1), frames, heading=np.array([-1.0, 0.0, 0.0]))
    w.meta.update(fish_bones=[(0, 10), (10, 20)], fish_markers=[(0, n), (n, 2 * n)])
    return w


def _max_marker_speed(ms: MarkerSet, pose: np.ndarray) -> float:
    """Largest skinned marker speed of one pose (rates included)."""
    U = np.zeros((3, ms.n))
    for j in range(2):
        P = pose[ms.bone[j]]
        Rd = P[:, 12:21].reshape(-1, 3, 3)
        U += ms.weight[j] * (np.einsum('kab,bk->ak', Rd, ms.xrest) + P[:, 21:24].T)
    return float(np.linalg.norm(U, axis=0).max())


BATCH_MAX_MARKER_SPEED = 0.08


def batch_workloads(count: int = 64, seed: int = 4, nsteps: int = 200):
    """Batched environments: sizes nx ~ U{64..192}, ny, nz ~ U{48..96}
    (independent integers), markers n ~ U{2000..6000}, joint-angle targets
    ~ U[-0.4, 0.4]^10, all drawn from numpy's default_rng(seed) in that order
    per environment. Fish of length round(0.4 nx) with its head at
    (0.25 nx, ny/2, nz/2); inflow (0.05, 0, 0) with a zero-gradient outlet,
    no noise. The joint angles approach their targets along a half-cosine
    ramp. Two deterministic adjustments keep the workload valid, both
    recorded in meta: targets are halved until every pose of the ramp keeps
    the markers 2 cells (3 on the high side) inside the domain, and the ramp
    is lengthened from 50 steps until the fastest marker moves at most
    BATCH_MAX_MARKER_SPEED lattice units per step (a lattice Boltzmann fluid
    must stay well below the lattice speed of sound, 0.577)."""
    rng = np.random.default_rng(seed)
    out = []
    u_in = np.array([0.05, 0.0, 0.0])
    for e in range(count):
        nx = int(rng.integers(64, 193))
        ny = int(rng.integers(48, 97))
        nz = int(rng.integers(48, 97))
        n = int(rng.integers(2000, 6001))
        targets = rng.uniform(-0.4, 0.4, size=10)
        length = float(round(0.4 * nx))
        head = (0.25 * nx, ny / 2.0, nz / 2.0)
        ms = fish_surface(n, length, head)
        halvings = 0
        probe = np.array([0.0, 12.5, 25.0, 37.5, 50.0])  # ramp fractions 0 .. 1 for a 50-step ramp
        while True:
            th, thd = ramp_joint_angles(targets, probe, ramp=50.0)
            psi, psid = headings_from_joint_angles(th, thd)
            poses = chain_poses(psi, psid, ms.joints_rest)
            ok = True
            for s in range(len(probe)):
                X = skin_positions(ms, poses[s])
                for a, m in enumerate((nx, ny, nz)):
                    if X[a].min() < 2.0 or X[a].max() >= m - 3.0:
                        ok = False
            if ok:
                break
            targets = targets * 0.5
            halvings += 1
        # marker speed scales as 1 / ramp length; the half-cosine rate peaks mid-ramp
        th, thd = ramp_joint_angles(targets, np.array([25.0]), ramp=50.0)
        psi, psid = headings_from_joint_angles(th, thd)
        v50 = _max_marker_speed(ms, chain_poses(psi, psid, ms.joints_rest)[0])
        ramp = float(math.ceil(50.0 * max(1.0, v50 / BATCH_MAX_MARKER_SPEED)))
        steps = np.arange(nsteps)
        th, thd = ramp_joint_angles(targets, steps, ramp=ramp)
        psi, psid = headings_from_joint_angles(th, thd)
        poses = chain_poses(psi, psid, ms.joints_rest)
        frames = make_frames(nsteps, origin=ms.xrest.mean(axis=1), u_lo=u_in, u_hi=u_in)
        u0 = np.broadcast_to(u_in.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
        w = Workload(f"env{e}-{nx}x{ny}x{nz}", nx, ny, nz, 0.6, BC_VELOCITY, BC_OUTFLOW, nsteps, u0, ms, poses,
                     frames, heading=np.array([-1.0, 0.0, 0.0]))
        w.meta.update(targets=targets, halvings=halvings, ramp=ramp)
        out.append(w)
    return out
