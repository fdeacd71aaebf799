"""Checks of the seeded synthetic workload generators (geometry, kinematics,
frames). They hold no method arithmetic; these tests pin their definitions."""
import math

import numpy as np

from paper_2206_01683_amd import inputs as I


def test_fibonacci_sphere_on_radius():
    ms = I.fibonacci_sphere(500, 6.0, (20.0, 16.0, 16.0))
    r = np.linalg.norm(ms.xrest - np.array([[20.0], [16.0], [16.0]]), axis=0)
    np.testing.assert_allclose(r, 6.0, atol=1e-13)
    assert abs(ms.dv[0] - 4 * math.pi * 36 / 500) < 1e-15
    assert np.abs(ms.xrest.mean(1) - np.array([20, 16, 16])).max() < 0.05


def test_fish_surface_geometry():
    L = 96.0
    ms = I.fish_surface(12000, L, (112.0, 96.0, 96.0))
    assert ms.n == 12000
    # area of the elliptic-section body, about 4,000 lattice units^2
    assert 3800 < ms.area < 4300
    assert abs(ms.dv.sum() - ms.area) < 1e-9
    x = ms.xrest[0]
    assert x.min() >= 112.0 and x.max() <= 112.0 + L
    b = I.fish_half_width((x - 112.0) / L, L)
    ell = ((ms.xrest[1] - 96) / np.maximum(b, 1e-300)) ** 2 + ((ms.xrest[2] - 96) / np.maximum(1.5 * b, 1e-300)) ** 2
    np.testing.assert_allclose(ell[b > 1e-6], 1.0, atol=1e-9)
    np.testing.assert_allclose(ms.weight.sum(0), 1.0, atol=1e-15)
    assert ms.bone.min() >= 0 and ms.bone.max() <= 9
    assert abs(I.fish_half_width(np.array([1 / 3]), L)[0] - 0.08 * L) < 1e-12


def test_frames_velocity_is_running_sum_of_acceleration():
    fr = I.accelerating_frames(900, 1e-5, 400.0, (0, 0, 0))
    a = fr[:, 0]
    np.testing.assert_allclose(a, 1e-5 * np.sin(2 * np.pi * np.arange(900) / 400))
    V = -fr[:, 12]
    np.testing.assert_allclose(V[1:], np.cumsum(a)[:-1], atol=1e-18)
    assert V[0] == 0.0
    # a later window matches the same schedule
    fr2 = I.accelerating_frames(100, 1e-5, 400.0, (0, 0, 0), start=500)
    np.testing.assert_allclose(fr2, fr[500:600], atol=1e-18)


def test_wave_kinematics_speed_bound_and_head_fixed():
    w = I.fish_workload(nsteps=400)
    assert w.poses.shape == (400, 10, 24)
    X0 = I.skin_positions(w.markers, w.poses[0])
    assert X0[0].min() > 2 and X0[0].max() < w.nx - 3
    # the travelling wave's tail speed stays near 0.1 L 2 pi / 400 = 0.151
    X1 = I.skin_positions(w.markers, w.poses[1])
    assert np.abs(X1 - X0).max() < 0.2


def test_fin_parameters_and_batch_envs():
    th, thd = I.fin_joint_angles(I.C5_BASE, np.arange(400))
    assert th.shape == (400, 10)
    assert abs(np.abs(th[:, 9]).max() - 0.4) < 1e-3
    envs = I.batch_workloads(count=4, nsteps=60)
    for e in envs:
        assert 64 <= e.nx <= 192 and 48 <= e.ny <= 96 and 48 <= e.nz <= 96
        assert 2000 <= e.markers.n <= 6000
        for s in (0, 59):
            X = I.skin_positions(e.markers, e.poses[s])
            for a, m in enumerate((e.nx, e.ny, e.nz)):
                assert X[a].min() >= 2 and X[a].max() < m - 3
    # the draw is reproducible
    again = I.batch_workloads(count=4, nsteps=60)
    assert [(e.nx, e.ny, e.nz, e.markers.n) for e in envs] == [(e.nx, e.ny, e.nz, e.markers.n) for e in again]


def test_fin_pose_jacobian_matches_central_differences():
    """The complex-step Jacobian of the bone poses against central differences."""
    ms = I.fish_surface(300, 16.0, (12.0, 16.0, 16.0))
    steps = np.arange(7)
    p = np.asarray(I.C5_BASE, dtype=np.float64)
    J = I.fin_pose_jacobian(p, ms, steps)
    assert J.shape == (7, ms.nbones, 24, 8)
    np.testing.assert_array_equal(I.fin_poses(p, ms, steps), I.fin_workload(p, nsteps=7, nx=48, ny=32, nz=32,
                                                                            length=16.0, n=300,
                                                                            head=(12.0, 16.0, 16.0)).poses)
    h = 1e-6
    for j in range(8):
        e = np.zeros(8)
        e[j] = h
        fd = (I.fin_poses(p + e, ms, steps) - I.fin_poses(p - e, ms, steps)) / (2 * h)
        np.testing.assert_allclose(J[..., j], fd, atol=1e-7 * max(1.0, np.abs(J[..., j]).max()))


def test_two_fish_workload_structure():
    w = I.two_fish_workload(nsteps=40)
    ms = w.markers
    assert (w.nx, w.ny, w.nz) == (150, 50, 100) and ms.n == 4000 and ms.nbones == 20
    assert w.poses.shape == (40, 20, 24)
    (b0, b1), (c0, c1) = w.meta["fish_bones"][1], w.meta["fish_markers"][1]
    assert ms.bone[:, :c0].max() < b0 and ms.bone[:, c0:c1].min() >= b0 and ms.bone[:, c0:c1].max() < b1
    np.testing.assert_allclose(ms.weight.sum(0), 1.0, atol=1e-15)
    # each fish follows its own chain: the merged poses of fish 1 equal a lone fish's poses
    lone = I.fish_surface(2000, 40.0, (50.0, 25.0, 200.0 / 3.0))
    psi, psid = I.wave_headings(40.0, 10, np.arange(40) - 100.0)
    np.testing.assert_allclose(w.poses[:, 10:], I.chain_poses(psi, psid, lone.joints_rest), atol=1e-12)
    # the bodies stay apart and inside the open x faces
    for p in w.poses[::10]:
        X = I.skin_positions(ms, p)
        assert X[0].min() >= 2.0 and X[0].max() < w.nx - 3.0
        gap = np.linalg.norm(X[:, :2000, None] - X[:, None, 2000::11], axis=0).min()
        assert gap > 10.0


def test_surface_normals_are_outward_unit_and_normal_to_the_surface():
    """Sphere and fish rest normals: unit length, pointing away from the body
    axis, and orthogonal to the surface (the surface's own tangents, from
    nearby markers' positions projected on the tangent plane, are short)."""
    c = np.array([5.0, 6.0, 7.0])
    sp = I.fibonacci_sphere(300, 2.5, c)
    np.testing.assert_allclose(sp.normals, (sp.xrest - c[:, None]) / 2.5, rtol=0, atol=1e-14)
    L, head = 40.0, np.array([10.0, 20.0, 20.0])
    ms = I.fish_surface(3000, L, head)
    n = ms.normals
    np.testing.assert_allclose(np.linalg.norm(n, axis=0), 1.0, rtol=0, atol=1e-12)
    xi = (ms.xrest[0] - head[0]) / L
    mid = (xi > 0.05) & (xi < 0.95)
    radial = ms.xrest[1:] - head[1:, None]
    assert np.all((n[1:] * radial).sum(0)[mid] > 0)
    # the normal of a plane fitted to each marker's 12 nearest neighbours
    X = ms.xrest.T
    for k in np.flatnonzero(mid)[::50]:
        d = X - X[k]
        near = np.argsort((d * d).sum(1))[:13]
        P = X[near] - X[near].mean(0)
        fit = np.linalg.svd(P)[2][-1]
        assert abs(fit @ n[:, k]) > 0.98, (k, abs(fit @ n[:, k]))  # an x-sign error gives 0.69
