"""Pins of the oracle's node-level operators against facts that the paper and
the mathematics fix independently of how the oracle writes them:

* cascaded collision = relaxation of the central moments of eq. (14)/(31)
  toward their Maxwellian values (text after eq. 15 and after eq. 32),
  computed here by brute force (moment matrix, relax, invert);
* the equilibria carry exactly the Maxwellian central moments and are
  fixed points of the collision;
* the split source changes exactly the zeroth and first moments by
  M^A, F (eq. 23, 25) and psi/phi by S (eq. 40, 41, 51), and collision alone
  conserves them (text before eq. 17, after eq. 34, after eq. 46).
"""
import numpy as np
import pytest

EX9 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
EY9 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
EX5 = np.array([0, 1, 0, -1, 0], float)
EY5 = np.array([0, 0, 1, 0, -1], float)
CS2 = 1.0 / 3.0
ORDERS9 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
ORDERS5 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2)]


def central_matrix(ex, ey, orders, ux, uy):
    """Rows: (e_x - u_x)^m (e_y - u_y)^n for each moment order (eq. 14)."""
    return np.array([(ex - ux) ** m * (ey - uy) ** n for (m, n) in orders])


def brute_collide_f(f, om):
    rho = f.sum()
    ux, uy = (f * EX9).sum() / rho, (f * EY9).sum() / rho
    T = central_matrix(EX9, EY9, ORDERS9, ux, uy)
    k = T @ f
    tr, dev = k[3] + k[4], k[3] - k[4]
    tr = (1 - om[3]) * tr + om[3] * 2 * CS2 * rho
    dev = (1 - om[4]) * dev
    post = k.copy()
    post[3], post[4] = 0.5 * (tr + dev), 0.5 * (tr - dev)
    post[5] = (1 - om[5]) * k[5]
    post[6] = (1 - om[6]) * k[6]
    post[7] = (1 - om[7]) * k[7]
    post[8] = (1 - om[8]) * k[8] + om[8] * CS2 * CS2 * rho
    return np.linalg.solve(T, post), rho, ux, uy


def brute_collide_adv(g, ux, uy, om):
    s = g.sum()
    T = central_matrix(EX5, EY5, ORDERS5, ux, uy)
    k = T @ g
    post = k.copy()
    post[1] = (1 - om[1]) * k[1]
    post[2] = (1 - om[2]) * k[2]
    tr, dev = k[3] + k[4], k[3] - k[4]
    tr = (1 - om[3]) * tr + om[3] * 2 * CS2 * s
    dev = (1 - om[4]) * dev
    post[3], post[4] = 0.5 * (tr + dev), 0.5 * (tr - dev)
    return np.linalg.solve(T, post), s


def random_f(rng):
    rho = 1 + 0.05 * rng.standard_normal()
    ux, uy = 0.1 * rng.standard_normal(2)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    feq = rho * w * (1 + 3 * (EX9 * ux + EY9 * uy) + 4.5 * (EX9 * ux + EY9 * uy) ** 2
                     - 1.5 * (ux * ux + uy * uy))
    return feq + 0.01 * rng.standard_normal(9) * w


def random_omegas(rng, n):
    return rng.uniform(0.3, 1.95, n)


@pytest.mark.parametrize("seed", range(20))
def test_cascaded_f_equals_central_moment_relaxation(orc, seed):
    rng = np.random.default_rng(seed)
    f = random_f(rng)
    om = np.zeros(9)
    om[3:] = random_omegas(rng, 6)
    expect, rho, ux, uy = brute_collide_f(f, om)
    got = orc.collide_f(f, rho, ux, uy, 0.0, 0.0, 0.0, om)
    np.testing.assert_allclose(got, expect, rtol=0, atol=2e-15)


@pytest.mark.parametrize("seed", range(20))
def test_cascaded_adv_equals_central_moment_relaxation(orc, seed):
    rng = np.random.default_rng(100 + seed)
    s = rng.uniform(-1, 1)
    ux, uy = 0.1 * rng.standard_normal(2)
    w = np.array([1 / 3] + [1 / 6] * 4)
    g = s * w + 0.02 * rng.standard_normal(5)
    om = np.zeros(5)
    om[1:] = random_omegas(rng, 4)
    expect, s_sum = brute_collide_adv(g, ux, uy, om)
    got = orc.collide_adv(g, s_sum, ux, uy, 0.0, om)
    np.testing.assert_allclose(got, expect, rtol=0, atol=2e-15)


@pytest.mark.parametrize("seed", range(10))
def test_equilibria_have_maxwellian_central_moments(orc, seed):
    rng = np.random.default_rng(200 + seed)
    rho = 1 + 0.1 * rng.standard_normal()
    ux, uy = 0.15 * rng.standard_normal(2)
    feq = orc.equilibrium_f(rho, ux, uy)
    k = central_matrix(EX9, EY9, ORDERS9, ux, uy) @ feq
    maxwell = np.array([rho, 0, 0, CS2 * rho, CS2 * rho, 0, 0, 0, CS2 * CS2 * rho])
    np.testing.assert_allclose(k, maxwell, rtol=0, atol=1e-15)
    s = rng.uniform(-1, 1)
    geq = orc.equilibrium_adv(s, ux, uy)
    k5 = central_matrix(EX5, EY5, ORDERS5, ux, uy) @ geq
    np.testing.assert_allclose(k5, [s, 0, 0, CS2 * s, CS2 * s], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(10))
def test_equilibria_are_collision_fixed_points(orc, seed):
    rng = np.random.default_rng(300 + seed)
    rho = 1 + 0.1 * rng.standard_normal()
    ux, uy = 0.15 * rng.standard_normal(2)
    om = np.zeros(9)
    om[3:] = random_omegas(rng, 6)
    feq = orc.equilibrium_f(rho, ux, uy)
    np.testing.assert_allclose(orc.collide_f(feq, rho, ux, uy, 0, 0, 0, om), feq,
                               rtol=0, atol=1e-15)
    s = rng.uniform(-1, 1)
    om5 = np.zeros(5)
    om5[1:] = random_omegas(rng, 4)
    geq = orc.equilibrium_adv(s, ux, uy)
    np.testing.assert_allclose(orc.collide_adv(geq, s, ux, uy, 0.0, om5), geq,
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(10))
def test_sources_change_exactly_the_conserved_moments(orc, seed):
    rng = np.random.default_rng(400 + seed)
    f = random_f(rng)
    rho_arg = 1 + 0.05 * rng.standard_normal()
    ux, uy = 0.1 * rng.standard_normal(2)
    MA, Fx, Fy = 1e-3 * rng.standard_normal(3)
    om = np.zeros(9)
    om[3:] = random_omegas(rng, 6)
    fp = orc.collide_f(f, rho_arg, ux, uy, MA, Fx, Fy, om)
    d = fp - f
    assert abs(d.sum() - MA) < 1e-15
    assert abs((d * EX9).sum() - Fx) < 1e-15
    assert abs((d * EY9).sum() - Fy) < 1e-15
    fp0 = orc.collide_f(f, rho_arg, ux, uy, 0.0, 0.0, 0.0, om)
    assert abs((fp0 - f).sum()) < 1e-15
    assert abs(((fp0 - f) * EX9).sum()) < 1e-15
    assert abs(((fp0 - f) * EY9).sum()) < 1e-15

    g = rng.uniform(-0.2, 0.2, 5)
    S = 1e-3 * rng.standard_normal()
    om5 = np.zeros(5)
    om5[1:] = random_omegas(rng, 4)
    gp = orc.collide_adv(g, rng.uniform(-1, 1), ux, uy, S, om5)
    assert abs((gp - g).sum() - S) < 1e-15
    gp0 = orc.collide_adv(g, rng.uniform(-1, 1), ux, uy, 0.0, om5)
    assert abs((gp0 - g).sum()) < 1e-15


def test_equilibrium_weights_at_rest(orc):
    """At rest the equilibria reduce to the lattice weights 4/9, 1/9, 1/36 and
    1/3, 1/6 (c_s^2 = 1/3)."""
    np.testing.assert_allclose(orc.equilibrium_f(1.0, 0.0, 0.0),
                               [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-16)
    np.testing.assert_allclose(orc.equilibrium_adv(1.0, 0.0, 0.0),
                               [1 / 3] + [1 / 6] * 4, atol=1e-16)
