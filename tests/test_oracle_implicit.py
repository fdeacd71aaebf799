"""Pins of the oracle's implicit velocity correction (the implicit immersed
boundary the paper cites, Wu and Shu's velocity correction): the marker forces
are the solution of S G = (I + [omega]x)(U - U*), S = interp . 1/(2 rho) .
spread, taken by conjugate-gradient steps.

What fixes the result independently of the oracle's code:
  * one marker in a uniform state: S is the scalar (3/8)^3 / (2 rho) (the
    4-point kernel's squared weights sum to 3/8 along each axis), so one step
    gives G = 2 rho (8/3)^3 (U - u0) exactly, wherever the marker sits;
  * n markers: conjugate gradients end in at most n steps, after which the
    velocity with the spread force, interpolated back, equals the body
    velocity at every marker (no slip) -- also in a rotating frame, where the
    forced velocity comes from the Coriolis solve u + omega x u = b;
  * a body at rest in fluid at rest needs no force (and no 0/0 appears)."""
import numpy as np
import pytest

import oracle
from paper_2206_01683_amd import inputs as I


def _markers(pos, dv=0.7):
    pos = np.asarray(pos, dtype=np.float64).reshape(3, -1)
    n = pos.shape[1]
    return I.MarkerSet(xrest=pos.copy(), bone=np.zeros((2, n), np.int32),
                       weight=np.vstack([np.ones(n), np.zeros(n)]), dv=np.full(n, dv), nbones=1, area=dv * n)


def _moving_pose(vel):
    p = I.identity_poses(1)
    p[0, 0, 21:24] = vel  # translation rate: every marker moves with vel
    return p


def _coriolis_solve(v, omega):
    """u with u + omega x u = v, per node (v: (3, ...))."""
    w = np.asarray(omega, dtype=np.float64).reshape(3, *([1] * (v.ndim - 1)))
    wv = np.cross(w, v, axis=0)
    wd = (w * v).sum(0, keepdims=True)
    return (v - wv + wd * w) / (1.0 + (w * w).sum())


def _slip(prm, f0, frame, res, dv, omega=(0.0, 0.0, 0.0)):
    """Interpolated velocity with the step's IB force minus the body velocity."""
    rho, ustar = oracle.macros(prm, f0, frame)
    g = oracle.spread(prm, res["X"], res["F"] * dv)
    uf = ustar + _coriolis_solve(g / (2.0 * rho), omega)
    return oracle.interpolate(prm, uf, res["X"]) - res["U"], U_scale(res, prm, ustar)


def U_scale(res, prm, ustar):
    return np.abs(res["U"] - oracle.interpolate(prm, ustar, res["X"])).max()


@pytest.mark.parametrize("pos,rho0", [((6.3, 5.71, 6.02), 1.0), ((5.5, 6.0, 5.25), 1.3), ((6.0, 6.0, 6.0), 0.9)])
@pytest.mark.parametrize("iters", [1, 3])
def test_one_marker_closed_form(pos, rho0, iters):
    n = 12
    u0 = np.array([0.03, -0.02, 0.01])
    f0 = oracle.equilibrium_field(np.full((n, n, n), rho0), np.broadcast_to(u0.reshape(3, 1, 1, 1), (3, n, n, n)))
    ms = _markers(pos)
    U = np.array([0.05, 0.01, -0.02])
    prm = oracle.params(n, n, n, 0.7, mdf_iters=iters, ib_scheme=oracle.IB_IMPLICIT)
    res = oracle.run(prm, f0.copy(), I.make_frames(1), ms, _moving_pose(U))
    G = res["F"][:, 0] * ms.dv[0]
    np.testing.assert_allclose(G, 2.0 * rho0 * (8.0 / 3.0) ** 3 * (U - u0), rtol=1e-12, atol=1e-15)
    slip, _ = _slip(prm, f0, I.make_frames(1)[0], res, ms.dv)
    assert np.abs(slip).max() < 1e-14


def _cluster(center, n, seed, spacing=1.1):
    """n points near `center`, pairwise at least `spacing` apart (their
    kernel supports overlap, so S is far from diagonal)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        q = np.asarray(center) + rng.uniform(-1.8, 1.8, 3)
        if all(np.linalg.norm(q - p) >= spacing for p in pts):
            pts.append(q)
    return np.array(pts).T


@pytest.mark.parametrize("omega", [(0.0, 0.0, 0.0), (0.01, -0.02, 0.03)])
def test_n_markers_end_with_no_slip_after_n_steps(omega):
    n, nm = 14, 6
    shape = (n, n, n)
    rho = I.random_density(shape, 0.05, seed=3)
    u = I.perturbed_velocity(shape, np.array([0.02, 0.01, -0.01]), 0.02, seed=4)
    f0 = oracle.equilibrium_field(rho, u)
    ms = _markers(_cluster((7.0, 7.0, 7.0), nm, seed=5))
    U = np.array([-0.03, 0.02, 0.04])
    frame = I.make_frames(1, omega=omega, origin=(7.0, 7.0, 7.0))
    slips = []
    for iters in (1, nm):
        prm = oracle.params(n, n, n, 0.7, mdf_iters=iters, ib_scheme=oracle.IB_IMPLICIT)
        res = oracle.run(prm, f0.copy(), frame, ms, _moving_pose(U))
        slip, scale = _slip(prm, f0, frame[0], res, ms.dv, omega)
        slips.append(np.abs(slip).max() / scale)
    assert slips[0] > 1e-3, slips       # one step is not the solution here
    assert slips[1] < 1e-9, slips       # n steps are


def test_body_moving_with_the_fluid_needs_no_force():
    n = 12
    ms = _markers(_cluster((6.0, 6.0, 6.0), 4, seed=1))
    prm = oracle.params(n, n, n, 0.7, mdf_iters=5, ib_scheme=oracle.IB_IMPLICIT)
    # at rest in fluid at rest: the right-hand side is zero (some components
    # exactly, others to the rounding of the momentum sums); exact zeros give
    # 0/0 in alpha and beta unless guarded
    f0 = oracle.equilibrium_field(np.ones((n, n, n)), np.zeros((3, n, n, n)))
    res = oracle.run(prm, f0.copy(), I.make_frames(1), ms, _moving_pose(np.zeros(3)))
    assert np.all(np.isfinite(res["F"])) and np.abs(res["F"]).max() < 1e-12
    # moving with a uniform stream: zero up to the rounding of interpolation
    u0 = np.array([0.03, -0.02, 0.01])
    f0 = oracle.equilibrium_field(np.ones((n, n, n)), np.broadcast_to(u0.reshape(3, 1, 1, 1), (3, n, n, n)))
    res = oracle.run(prm, f0.copy(), I.make_frames(1), ms, _moving_pose(u0))
    assert np.all(np.isfinite(res["F"])) and np.abs(res["F"]).max() < 1e-12


def test_implicit_slip_below_multi_direct_forcing_on_the_sphere():
    """At an equal number of spread-and-interpolate passes, the implicit
    correction leaves far less slip than multi-direct forcing."""
    sw = I.sphere_workload(nsteps=1)
    f0 = oracle.equilibrium_field(np.ones((sw.nz, sw.ny, sw.nx)), sw.u0)
    rms = {}
    for scheme in (oracle.IB_DIRECT, oracle.IB_IMPLICIT):
        for k in (1, 2, 4):
            prm = oracle.params(sw.nx, sw.ny, sw.nz, sw.tau, sw.bc_lo, sw.bc_hi, k, 1.0, ib_scheme=scheme)
            res = oracle.run(prm, f0.copy(), sw.frames, sw.markers, sw.poses, 1)
            slip, _ = _slip(prm, f0, sw.frames[0], res, sw.markers.dv)
            rms[scheme, k] = np.sqrt((slip ** 2).mean())
    for k in (1, 2, 4):
        assert rms[oracle.IB_IMPLICIT, k] < 0.2 * rms[oracle.IB_DIRECT, k], rms
