"""Pins of the oracle's two-relaxation-time (TRT) collision, the smallest
member of the multiple-relaxation-time family: the parts of f even and odd in
c relax at omega+ = 1/tau (viscosity) and omega- with
(tau - 1/2)(1/omega- - 1/2) = Lambda.

What fixes it independently of the oracle's code:
  * equal rates (Lambda = (tau - 1/2)^2) reduce it to the textbook BGK
    collision, written separately in the oracle;
  * a pure even non-equilibrium part that carries no mass relaxes by exactly
    (1 - omega+), a pure odd one without momentum by exactly (1 - omega-);
  * a forced collision conserves mass and adds exactly F to the momentum;
  * the shear viscosity tends to (tau - 1/2)/3 at second order whatever
    Lambda: Taylor-Green decay;
  * Poiseuille flow between velocity walls is exact at tau = 1 for every
    Lambda, as for BGK."""
import math

import numpy as np
import pytest

import oracle
from paper_2206_01683_amd import inputs as I

C, W = oracle.lattice()


def _state(seed, rho=1.02, u=(0.03, -0.02, 0.01), noise=2e-4):
    rng = np.random.default_rng(seed)
    feq = oracle.equilibrium(rho, np.array(u))
    return feq + noise * rng.standard_normal(27) * W


FRAME = I.make_frames(1, acc=(1e-4, -2e-4, 5e-5), omega=(0.002, -0.001, 0.003), alpha=(1e-5, 0, -2e-5),
                      origin=(3.0, 2.0, 1.0))[0]
X = np.array([5.0, 4.0, 2.0])


@pytest.mark.parametrize("tau", [0.55, 0.6, 0.9, 1.4])
def test_equal_rates_are_bgk(tau):
    f = _state(1)
    g = np.array([1e-4, -3e-5, 2e-5])
    a, ua, Fa = oracle.collide_node(f, g, FRAME, X, tau)
    b, ub, Fb = oracle.collide_node(f, g, FRAME, X, tau, trt_lambda=(tau - 0.5) ** 2)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-16)
    np.testing.assert_array_equal(ua, ub)
    np.testing.assert_array_equal(Fa, Fb)


@pytest.mark.parametrize("tau,lam", [(0.6, 3 / 16), (0.8, 1 / 12), (1.2, 1 / 4)])
def test_even_and_odd_parts_relax_at_their_own_rates(tau, lam):
    rho, u = 1.03, np.array([0.02, 0.01, -0.015])
    feq = oracle.equilibrium(rho, u)
    wp, wm = 1.0 / tau, 1.0 / (0.5 + lam / (tau - 0.5))
    even = 1e-4 * W * (C[:, 0] ** 2 - 1.0 / 3.0)            # no mass, no momentum
    odd = 1e-4 * W * (C[:, 0] * C[:, 1] * C[:, 2])          # no mass, no momentum
    zero = np.zeros(3)
    still = I.make_frames(1)[0]
    for d, w in ((even, wp), (odd, wm)):
        out, _, _ = oracle.collide_node(feq + d, zero, still, X, tau, trt_lambda=lam)
        np.testing.assert_allclose(out - feq, (1.0 - w) * d, rtol=0, atol=2e-16)
    out, _, _ = oracle.collide_node(feq + even + odd, zero, still, X, tau, trt_lambda=lam)
    np.testing.assert_allclose(out - feq, (1.0 - wp) * even + (1.0 - wm) * odd, rtol=0, atol=2e-16)


@pytest.mark.parametrize("lam", [3 / 16, 1 / 12])
def test_forced_collision_conserves_mass_and_adds_the_force(lam):
    f = _state(2)
    g = np.array([2e-4, 1e-4, -3e-4])
    out, _, F = oracle.collide_node(f, g, FRAME, X, 0.7, trt_lambda=lam)
    assert abs(out.sum() - f.sum()) < 1e-15
    np.testing.assert_allclose(C.T @ out, C.T @ f + F, rtol=0, atol=1e-16)


def _taylor_green_rate(N, tau, lam, steps=200, every=20):
    nx = ny = N
    nz = 4
    k = 2 * math.pi / N
    Xg, Yg = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    u = np.zeros((3, nz, ny, nx))
    u[0] = (0.01 * np.sin(k * Xg) * np.cos(k * Yg))[None]
    u[1] = (-0.01 * np.cos(k * Xg) * np.sin(k * Yg))[None]
    f = oracle.equilibrium_field(np.ones((nz, ny, nx)), u)
    prm = oracle.params(nx, ny, nz, tau, collision=oracle.COLLIDE_TRT, trt_lambda=lam)
    fr = I.make_frames(every)
    E = []
    for _ in range(steps // every):
        _, uu = oracle.macros(prm, f, fr[0])
        E.append((uu ** 2).sum())
        f = oracle.run(prm, f, fr)["f"]
    t = np.arange(len(E)) * every
    rate = -np.polyfit(t[2:], np.log(E[2:]), 1)[0]
    return rate, 4 * (tau - 0.5) / 3 * k * k


@pytest.mark.parametrize("lam", [3 / 16, 1 / 4])
def test_taylor_green_viscosity_is_set_by_tau_plus(lam):
    """The decay rate tends to 4 nu k^2 with nu = (tau+ - 1/2)/3 at second
    order; Lambda only enters the O(k^2) error."""
    r32, t32 = _taylor_green_rate(32, 0.6, lam)
    r64, t64 = _taylor_green_rate(64, 0.6, lam)
    e32, e64 = abs(r32 / t32 - 1), abs(r64 / t64 - 1)
    assert e32 < 4e-3
    assert 1.8 < math.log(e32 / e64) / math.log(2) < 2.3


@pytest.mark.parametrize("lam", [3 / 16, 1 / 12, 1 / 4])
def test_poiseuille_exact_at_tau_one(lam):
    nx, tau, gy = 9, 1.0, 1e-6
    nu = (tau - 0.5) / 3
    H = nx - 1
    steps = int(3 * H * H / nu)
    prm = oracle.params(nx, 4, 4, tau, oracle.BC_VELOCITY, oracle.BC_VELOCITY, collision=oracle.COLLIDE_TRT,
                        trt_lambda=lam)
    f = oracle.equilibrium_field(np.ones((4, 4, nx)), np.zeros((3, 4, 4, nx)))
    fr = I.make_frames(steps, acc=(0, -gy, 0))
    f = oracle.run(prm, f, fr)["f"]
    _, u = oracle.macros(prm, f, fr[0])
    x = np.arange(nx)
    ue = gy * x * (H - x) / (2 * nu)
    err = np.linalg.norm(u[1, 0, 0, 1:-1] - ue[1:-1]) / np.linalg.norm(ue)
    assert err < 1e-9


def test_invalid_trt_parameters_are_rejected():
    f = oracle.equilibrium_field(np.ones((4, 4, 4)), np.zeros((3, 4, 4, 4)))
    for lam in (0.0, -0.1, float("nan")):
        prm = oracle.params(4, 4, 4, 0.7, collision=oracle.COLLIDE_TRT, trt_lambda=lam)
        with pytest.raises(oracle.OracleError):
            oracle.run(prm, f.copy(), I.make_frames(1))
