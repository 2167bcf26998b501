"""Pins of the oracle's velocity set, product form and anomaly against what the
paper and the mathematics fix (Sec. 2.2, 2.3). No GPU.

Every expected value here is computed independently of the oracle's own code
path: moments are summed by brute force over the velocity list built here,
and compared with closed forms (Maxwell-Boltzmann tensors, the factorised
moments) or with textbook numbers.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def brute_velocities(D):
    return [tuple(v) for v in itertools.product((-1, 0, 1), repeat=D)]


@pytest.mark.parametrize("D", [2, 3])
def test_velocity_set_and_opposite(D):
    c = O.velocity_set(D)
    Q = 3 ** D
    assert c.shape == (Q, D)
    assert sorted(map(tuple, c.tolist())) == sorted(brute_velocities(D))
    # lexicographic order: i = sum_a (c_ia + 1) 3^a, so the opposite is Q-1-i
    for i in range(Q):
        assert i == sum((int(c[i, a]) + 1) * 3 ** a for a in range(D))
    np.testing.assert_array_equal(O.opposite(c), Q - 1 - np.arange(Q))


@pytest.mark.parametrize("D", [2, 3])
def test_second_order_truncation_is_polynomial_equilibrium(D):
    """At lam = 1, T = 1/3 the product-form equilibrium equals the textbook
    polynomial equilibrium w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u) up to
    O(u^3) (the conventional equilibrium is its second-order truncation, Sec. 3)."""
    tw = {2: [4 / 9, 1 / 9, 1 / 36], 3: [8 / 27, 2 / 27, 1 / 54, 1 / 216]}[D]
    vel = np.array(brute_velocities(D), dtype=float)
    # map brute velocities onto the oracle's order
    c = O.velocity_set(D)
    order = [brute_velocities(D).index(tuple(ci)) for ci in c.tolist()]
    vel = vel[order]
    w = np.array([tw[int(np.abs(v).sum())] for v in vel])
    direction = np.array([0.6, -0.48, 0.64][:D])
    errs = []
    for s in (0.04, 0.02, 0.01):
        u = s * direction
        poly = w * (1 + 3 * vel @ u + 4.5 * (vel @ u) ** 2 - 1.5 * u @ u)
        prod = O.equilibrium(np.array(1.0), u, 1.0 / 3.0, (1.0,) * D, c)
        errs.append(np.abs(prod - poly).max())
    # third-order remainder: halving u divides the difference by ~8
    assert 6.0 < errs[0] / errs[1] < 10.0
    assert 6.0 < errs[1] / errs[2] < 10.0


def brute_moment(f, vel, lam, powers):
    tot = 0.0
    for fi, v in zip(f, vel):
        term = fi
        for a, pw in enumerate(powers):
            term *= (lam[a] * v[a]) ** pw
        tot += term
    return tot


CASES = [
    (2, (1.0, 1.0), 1.0 / 3.0),
    (2, (2.0, 1.0), 1.0 / 3.0),
    (2, (1.4, 1.0), 0.5),
    (3, (1.0, 1.0, 1.0), 0.5),
    (3, (2.0, 1.0, 1.0), 0.5),
    (3, (1.4, 1.0, 2.0), 1.0 / 3.0),
]


@pytest.mark.parametrize("D,lam,T", CASES)
def test_factorised_moments(D, lam, T):
    """M_lmn = M_l00 M_0m0 M_00n with M_l00 = lam^(l-1) u (l odd), lam^(l-2) P (l even >= 2)
    (Sec. 2.2; the y and z rows read with m and n, the printed exponents repeat l)."""
    g = np.random.default_rng(11)
    c = O.velocity_set(D)
    vel = c.tolist()
    for _ in range(5):
        rho = g.uniform(0.8, 1.2)
        u = g.uniform(-0.2, 0.2, D)
        P = np.array([T + u[a] ** 2 + g.uniform(-0.02, 0.02) for a in range(D)])
        f = O.product_form(np.array(rho), u, P, lam, c)

        def m1(a, l):
            if l == 0:
                return 1.0
            return lam[a] ** (l - 1) * u[a] if l % 2 else lam[a] ** (l - 2) * P[a]

        for powers in itertools.product(range(5), repeat=D):
            want = rho
            for a in range(D):
                want *= m1(a, powers[a])
            got = brute_moment(f, vel, lam, powers)
            assert abs(got - want) < 1e-14 * max(1.0, abs(want)) * 10


@pytest.mark.parametrize("D,lam,T", CASES)
def test_equilibrium_tensors_and_anomaly(D, lam, T):
    """P^eq = p I + rho u u and Q^eq = Q^MB + Q~ with Q~ diagonal and equal to
    rho u_a (lam_a^2 - 3T) - rho u_a^3 (Sec. 2.3, eqs. Peq, Qeq, PMB, QMB, Deviation)."""
    g = np.random.default_rng(5)
    c = O.velocity_set(D)
    vel = c.tolist()
    for _ in range(5):
        rho = g.uniform(0.8, 1.2)
        u = g.uniform(-0.2, 0.2, D)
        f = O.equilibrium(np.array(rho), u, T, lam, c)
        p = rho * T
        Qt = O.anomaly(np.array(rho), rho * u, T, lam)
        for a, b in itertools.product(range(D), repeat=2):
            pw = [0] * D
            pw[a] += 1
            pw[b] += 1
            want = p * (a == b) + rho * u[a] * u[b]
            assert abs(brute_moment(f, vel, lam, pw) - want) < 1e-14
        for a, b, e in itertools.product(range(D), repeat=3):
            pw = [0] * D
            pw[a] += 1
            pw[b] += 1
            pw[e] += 1
            qmb = p * ((a == b) * u[e] + (a == e) * u[b] + (b == e) * u[a]) + rho * u[a] * u[b] * u[e]
            dev = brute_moment(f, vel, lam, pw) - qmb
            if a == b == e:
                assert abs(dev - Qt[a]) < 1e-14
                assert abs(dev - (rho * u[a] * (lam[a] ** 2 - 3 * T) - rho * u[a] ** 3)) < 1e-14
            else:
                assert abs(dev) < 1e-14


def test_lattice_temperature_cancels_linear_anomaly():
    """At lam = 1 the choice T = T_L = 1/3 removes the term linear in u (Sec. 2.3, eq. TL)."""
    rho = np.array([1.1, 0.9])
    j = np.array([[0.01, -0.02], [0.03, 0.0], [-0.05, 0.04]])
    Qt = O.anomaly(rho, j, 1.0 / 3.0, (1.0, 1.0, 1.0))
    np.testing.assert_allclose(Qt, -j ** 3 / rho ** 2, rtol=0, atol=1e-17)


@pytest.mark.parametrize("D", [2, 3])
def test_conservation_for_any_pressure(D):
    """The product form carries rho and rho u for any diagonal pressure, so the
    extended equilibrium conserves mass and momentum (Sec. 2.1, eqs. density, momentum)."""
    g = np.random.default_rng(3)
    c = O.velocity_set(D)
    lam = (2.0, 1.0, 1.4)[:D]
    for _ in range(10):
        rho = g.uniform(0.5, 1.5)
        u = g.uniform(-0.3, 0.3, D)
        P = g.uniform(0.2, 0.6, D)
        f = O.product_form(np.array(rho), u, P, lam, c)
        assert abs(f.sum() - rho) < 1e-14
        for a in range(D):
            assert abs((lam[a] * c[:, a] * f).sum() - rho * u[a]) < 1e-14
        for a in range(D):
            assert abs((lam[a] ** 2 * c[:, a] ** 2 * f).sum() - rho * P[a]) < 1e-14
