"""Pins of the oracle's lattice, equilibrium and collision against closed forms.

Each test checks the FP64 oracle against something other than itself: a
published table, an exact moment identity of the lattice, or a property the
definition of the collision fixes (mass, momentum, relaxation rate).
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_d3q27_weights_match_published_table():
    c, w = oracle.lattice()
    table = {}
    for line in open(os.path.join(GOLDEN, "d3q27_weights.txt")):
        if line.startswith("#") or not line.strip():
            continue
        s2, count, frac = line.split()
        table[int(s2)] = (int(count), float(Fraction(frac)))
    s2 = (c ** 2).sum(axis=1)
    for k, (count, wt) in table.items():
        assert (s2 == k).sum() == count
        np.testing.assert_allclose(w[s2 == k], wt, rtol=0, atol=1e-16)
    # velocity set is exactly {-1,0,1}^3 and the index convention holds
    assert {tuple(v) for v in c} == set(itertools.product((-1, 0, 1), repeat=3))
    for i in range(27):
        assert i == (c[i, 0] + 1) + 3 * (c[i, 1] + 1) + 9 * (c[i, 2] + 1)
        assert np.all(c[26 - i] == -c[i])
    assert np.all(c[13] == 0)


def test_lattice_isotropy_moments():
    c, w = oracle.lattice()
    c = c.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3.0, atol=1e-16)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-0.1, 0.1)
    u = rng.uniform(-0.15, 0.15, 3)
    c, _ = oracle.lattice()
    c = c.astype(float)
    feq = oracle.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-14
    np.testing.assert_allclose(feq @ c, rho * u, atol=1e-15)
    # second moment rho (u u + I/3) and third moment rho/3 (u_a d_bc + ...)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, c, c), rho * (np.outer(u, u) + np.eye(3) / 3.0),
                               atol=1e-15)
    d = np.eye(3)
    third = rho / 3.0 * (np.einsum("a,bc->abc", u, d) + np.einsum("b,ac->abc", u, d) + np.einsum("c,ab->abc", u, d))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", feq, c, c, c), third, atol=1e-15)
    # rest state is exactly the weight vector
    _, w = oracle.lattice()
    np.testing.assert_array_equal(oracle.equilibrium(1.0, np.zeros(3)), w)


def _frame(acc=(0, 0, 0), omega=(0, 0, 0), alpha=(0, 0, 0), origin=(0, 0, 0)):
    return np.concatenate([acc, omega, alpha, origin, np.zeros(6)]).astype(float)


def _nonequilibrium_direction(rng):
    """A population vector with zero mass and zero momentum."""
    c, _ = oracle.lattice()
    A = np.vstack([np.ones(27), c.T.astype(float)])  # 4 x 27
    h = rng.standard_normal(27)
    h -= A.T @ np.linalg.solve(A @ A.T, A @ h)
    return h


@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0, 1.7])
def test_bgk_relaxes_nonequilibrium_by_one_minus_inverse_tau(tau):
    rng = np.random.default_rng(1)
    rho, u = 1.03, np.array([0.04, -0.02, 0.01])
    h = 1e-3 * _nonequilibrium_direction(rng)
    f = oracle.equilibrium(rho, u) + h
    out, uo, F = oracle.collide_node(f, np.zeros(3), _frame(), np.zeros(3), tau)
    np.testing.assert_allclose(uo, u, atol=1e-16)
    np.testing.assert_allclose(F, 0.0, atol=0)
    np.testing.assert_allclose(out - oracle.equilibrium(rho, u), (1.0 - 1.0 / tau) * h, atol=1e-16)


@pytest.mark.parametrize("seed", range(4))
def test_forced_collision_conserves_mass_and_adds_force_to_momentum(seed):
    rng = np.random.default_rng(10 + seed)
    c, _ = oracle.lattice()
    c = c.astype(float)
    tau = 0.55 + rng.uniform(0, 1)
    f = oracle.equilibrium(1 + rng.uniform(-.05, .05), rng.uniform(-.1, .1, 3)) + 1e-3 * _nonequilibrium_direction(rng)
    g = rng.uniform(-1e-3, 1e-3, 3)
    fr = _frame(acc=rng.uniform(-1e-4, 1e-4, 3), omega=rng.uniform(-1e-2, 1e-2, 3),
                alpha=rng.uniform(-1e-4, 1e-4, 3), origin=rng.uniform(0, 10, 3))
    x = rng.uniform(0, 10, 3)
    out, u, F = oracle.collide_node(f, g, fr, x, tau)
    assert abs(out.sum() - f.sum()) < 1e-15
    np.testing.assert_allclose(out @ c - f @ c, F, atol=1e-16)


def _eq3(frame, x, u):
    """Eq. (3) of the paper written out: -p'' - r'' x x' - r' x (r' x x') - 2 r' x u."""
    acc, om, al, x0 = frame[0:3], frame[3:6], frame[6:9], frame[9:12]
    xp = np.asarray(x) - x0
    return -acc - np.cross(al, xp) - np.cross(om, np.cross(om, xp)) - 2.0 * np.cross(om, u)


@pytest.mark.parametrize("seed", range(6))
def test_node_velocity_satisfies_its_implicit_definition(seed):
    """u = (m + F/2)/rho with F = g + rho a_ni(x, u) and a_ni from Eq. (3)."""
    rng = np.random.default_rng(20 + seed)
    rho = 1 + rng.uniform(-.1, .1)
    m = rng.uniform(-.1, .1, 3)
    g = rng.uniform(-1e-2, 1e-2, 3)
    fr = _frame(acc=rng.uniform(-1e-3, 1e-3, 3), omega=rng.uniform(-0.3, 0.3, 3),
                alpha=rng.uniform(-1e-3, 1e-3, 3), origin=rng.uniform(0, 10, 3))
    x = rng.uniform(0, 10, 3)
    u, F = oracle.node_velocity(rho, m, g, fr, x)
    F_def = g + rho * _eq3(fr, x, u)
    np.testing.assert_allclose(F, F_def, atol=1e-15)
    np.testing.assert_allclose(u, (m + 0.5 * F_def) / rho, atol=1e-15)


def test_delta_kernel_golden_values():
    for line in open(os.path.join(GOLDEN, "peskin4_values.txt")):
        if line.startswith("#") or not line.strip():
            continue
        r, expr = line.split(None, 1)
        want = eval(expr.strip(), {"sqrt": math.sqrt})
        assert abs(oracle.phi(float(r)) - want) < 1e-15


def test_delta_kernel_identities():
    rng = np.random.default_rng(3)
    for r in np.concatenate([rng.uniform(0, 1, 200), [0.0, 0.5, 1e-12, 1 - 1e-12]]):
        j = np.arange(-3, 5)
        ph = np.array([oracle.phi(r - jj) for jj in j])
        assert abs(ph.sum() - 1.0) < 1e-14
        assert abs(((r - j) * ph).sum()) < 1e-14
        assert abs((ph ** 2).sum() - 3.0 / 8.0) < 1e-14
    # continuity and C^1 at |r| = 1 and 2, support [-2, 2], symmetry
    for a in (1.0, 2.0):
        e = 1e-7
        assert abs(oracle.phi(a - e) - oracle.phi(a + e)) < 1e-6
        dl = (oracle.phi(a - e) - oracle.phi(a - 2 * e)) / e
        dr = (oracle.phi(a + 2 * e) - oracle.phi(a + e)) / e
        assert abs(dl - dr) < 1e-5
    assert oracle.phi(2.0) == 0.0 and oracle.phi(-2.3) == 0.0
    for r in rng.uniform(0, 2, 50):
        assert oracle.phi(r) == oracle.phi(-r)
