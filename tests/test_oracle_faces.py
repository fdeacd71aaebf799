"""Pins of the oracle's open faces on every axis (non-equilibrium
extrapolation on y and z faces, edges and corners extrapolating from the
diagonal inward neighbour): the rest state and a uniform stream are kept
exactly, Poiseuille flow between y or z velocity walls is exact at tau = 1,
markers near an open face are rejected, mixed axes are refused."""
import numpy as np
import pytest

import oracle
from paper_2206_01683_amd import inputs as I

V, O, P = oracle.BC_VELOCITY, oracle.BC_OUTFLOW, oracle.BC_PERIODIC


def _uniform(nz, ny, nx, u):
    return oracle.equilibrium_field(np.ones((nz, ny, nx)),
                                    np.broadcast_to(np.asarray(u, float).reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy())


@pytest.mark.parametrize("faces", [((V, O), (V, O), (V, O)), ((O, O), (O, O), (O, O)), ((P, P), (V, V), (O, O))])
def test_rest_state_with_open_faces(faces):
    nz, ny, nx = 6, 7, 8
    f = _uniform(nz, ny, nx, (0, 0, 0))
    prm = oracle.params(nx, ny, nz, 0.6, faces[0][0], faces[0][1], bc_y=faces[1], bc_z=faces[2])
    out = oracle.run(prm, f.copy(), I.make_frames(100))["f"]
    np.testing.assert_allclose(out[:, 1:-1, 1:-1, 1:-1], f[:, 1:-1, 1:-1, 1:-1], atol=1e-15, rtol=0)


@pytest.mark.parametrize("high", [V, O])
def test_uniform_stream_through_all_open_faces_is_kept(high):
    """The local moving domain at constant velocity: every face sees the same
    far field, so the uniform stream is a fixed point (edges and corners too)."""
    nz, ny, nx = 7, 8, 9
    u0 = np.array([0.03, -0.01, 0.02])
    f = _uniform(nz, ny, nx, u0)
    prm = oracle.params(nx, ny, nz, 0.7, V, high, bc_y=(V, high), bc_z=(V, high))
    fr = I.make_frames(60, u_lo=u0, u_hi=u0)
    out = oracle.run(prm, f.copy(), fr)["f"]
    _, u = oracle.macros(prm, out, fr[0])
    err = np.abs(u[:, 1:-1, 1:-1, 1:-1] - u0.reshape(3, 1, 1, 1)).max()
    assert err < 1e-15


def _poiseuille_walls(axis, n, tau, g=1e-6):
    """Walls (velocity faces at rest) normal to `axis` (1: y, 2: z), flow
    along x driven by a frame acceleration, the other axes periodic."""
    nu = (tau - 0.5) / 3
    H = n - 1
    steps = int(3 * H * H / nu)
    dims = {0: 4, 1: 4, 2: 4}
    dims[axis] = n
    nx, ny, nz = dims[0], dims[1], dims[2]
    prm = oracle.params(nx, ny, nz, tau, bc_y=(V, V) if axis == 1 else (P, P), bc_z=(V, V) if axis == 2 else (P, P))
    f = _uniform(nz, ny, nx, (0, 0, 0))
    fr = I.make_frames(steps, acc=(-g, 0, 0))  # a_ni = -acc = +g e_x
    f = oracle.run(prm, f, fr)["f"]
    _, u = oracle.macros(prm, f, fr[0])
    s = np.arange(n)
    ue = g * s * (H - s) / (2 * nu)
    ux = u[0, 0, :, 0] if axis == 1 else u[0, :, 0, 0]
    assert np.abs(u[1]).max() < 1e-14 and np.abs(u[2]).max() < 1e-14
    return np.linalg.norm(ux[1:-1] - ue[1:-1]) / np.linalg.norm(ue)


@pytest.mark.parametrize("axis", [1, 2])
def test_poiseuille_between_y_or_z_walls_exact_at_tau_one(axis):
    for n in (9, 17):
        assert _poiseuille_walls(axis, n, 1.0) < 1e-9


def test_poiseuille_between_z_walls_second_order():
    import math
    e9, e17 = _poiseuille_walls(2, 9, 0.6), _poiseuille_walls(2, 17, 0.6)
    assert 1.8 < math.log(e9 / e17) / math.log(2) < 2.3


def test_marker_near_open_y_face_rejected_and_mixed_axis_refused():
    sw = I.sphere_workload(nsteps=2)
    prm = oracle.params(sw.nx, sw.ny, sw.nz, sw.tau, sw.bc_lo, sw.bc_hi, bc_y=(O, O))
    near = I.fibonacci_sphere(200, 3.0, (20.0, 4.5, 16.0))  # reaches y = 1.5 < 2
    f = _uniform(sw.nz, sw.ny, sw.nx, (0.05, 0, 0))
    with pytest.raises(oracle.OracleError):
        oracle.run(prm, f.copy(), sw.frames, near, I.identity_poses(2), 2)
    far = I.fibonacci_sphere(200, 3.0, (20.0, 16.0, 16.0))
    oracle.run(prm, f.copy(), sw.frames, far, I.identity_poses(2), 2)
    bad = oracle.params(sw.nx, sw.ny, sw.nz, sw.tau, bc_y=(P, O))
    with pytest.raises(oracle.OracleError):
        oracle.run(bad, f.copy(), sw.frames, None, None, 1)
