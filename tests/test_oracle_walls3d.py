"""Pins of the D3Q27 Grad-wall oracle (oracle/elbm_walls3d.py): properties
the rule must have, checked without the GPU."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import elbm_faces as OF
from oracle import elbm_walls3d as OW


@pytest.mark.parametrize("lam,T", [((1.0, 1.0, 1.0), 1 / 3), ((1.4, 1.0, 2.0), 0.55)])
def test_grad_populations_carry_the_moments_they_are_built_from(lam, T):
    g = np.random.default_rng(12)
    c = O.velocity_set(3)
    v = c * np.array(lam)[None, :]
    for _ in range(4):
        rho = 1.0 + 0.1 * g.standard_normal()
        u = 0.05 * g.standard_normal(3)
        A = 1e-3 * g.standard_normal((3, 3))
        Pi = A + A.T
        f = OW.grad_populations_3d(rho, u, Pi, T, lam, c)
        assert f.sum() == pytest.approx(rho, abs=1e-14)
        for a in range(3):
            assert (v[:, a] * f).sum() == pytest.approx(rho * u[a], abs=1e-14)
        for a, b in itertools.product(range(3), range(3)):
            want = rho * ((T if a == b else 0.0) + u[a] * u[b]) + Pi[a, b]
            assert (v[:, a] * v[:, b] * f).sum() == pytest.approx(want, abs=1e-14), (a, b)


def _uniform(n, lam, T, u0):
    nx, ny, nz = n
    rho = np.ones((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    for a in range(3):
        u[a] = u0[a]
    return O.equilibrium(rho, u, T, lam, O.velocity_set(3))


@pytest.mark.parametrize("lam,T", [((1.0, 1.0, 1.0), 1 / 3), ((2.0, 1.0, 1.0), 0.5)])
def test_a_stream_moving_with_both_walls_stays_uniform(lam, T):
    """Both walls moving at U along x over a fluid moving at U: the uniform
    stream is a steady state of the rule (and of the anomaly's odd ghost,
    since j_y = 0), to 1e-14."""
    n = (4, 6, 3)
    U = 0.04
    p = O.Params(n=n, lam=lam, T=T, omega=1.6, walls=(False, True, False))
    f0 = _uniform(n, lam, T, (U, 0.0, 0.0))
    f = OW.run(f0, p, 20, wall_u=(U, U))
    assert np.abs(f - f0).max() < 1e-14


@pytest.mark.parametrize("omega,rates,lam,T", [
    (1.6, None, (1.0, 1.0, 1.0), 1 / 3),
    (1.0, None, (2.0, 1.0, 1.0), 0.5),
    (1.6, (1.6, 1.2), (2.0, 1.0, 1.0), 0.5),
])
def test_grad_walls_hold_couette_flow_linear(omega, rates, lam, T):
    """Plane Couette flow between a resting low wall and a high wall moving
    at u_w along x: the steady profile is the straight line through the two
    halfway walls, to 1e-8 of u_w, with no normal or spanwise velocity (LBGK,
    and the MRT collision with omega_bulk = omega)."""
    n, uw = (3, 6, 3), 0.01
    p = O.Params(n=n, lam=lam, T=T, omega=omega, walls=(False, True, False))
    f = OW.run(_uniform(n, lam, T, (0.0, 0.0, 0.0)), p, 2600, wall_u=(0.0, uw), rates=rates)
    _, u = O.velocity(f, p)
    y = np.arange(n[1]) + 0.5
    assert np.abs(u[0][1, :, 1] - uw * y / n[1]).max() < 1e-8 * uw
    assert np.abs(u[1]).max() < 1e-13 and np.abs(u[2]).max() < 1e-13


def test_z_uniform_flow_is_the_d2q9_grad_wall():
    """A flow that does not depend on z and has no z velocity: summed over
    c_z, the D3Q27 populations evolve exactly as the D2Q9 ones under the D2Q9
    Grad walls of elbm_faces (the product form's z triplets sum to one, and
    every xz, yz and zz term of the wall vanishes), to 1e-13 over 12 steps of
    a forced channel with a moving wall, on a stretched lattice."""
    nx, ny, nz = 6, 7, 3
    lam3, lam2, T, omega = (2.0, 1.0, 1.0), (2.0, 1.0), 0.5, 1.7
    g = np.random.default_rng(4)
    rho = 1.0 + 0.01 * g.standard_normal((ny, nx))
    u2 = 0.03 * g.standard_normal((2, ny, nx))
    c3, c2 = O.velocity_set(3), O.velocity_set(2)
    rho3 = np.broadcast_to(rho, (nz, ny, nx))
    u3 = np.zeros((3, nz, ny, nx))
    u3[0], u3[1] = u2[0], u2[1]
    f3 = O.equilibrium(rho3, u3, T, lam3, c3) * (1.0 + 0.002 * np.broadcast_to(g.standard_normal((27, 1, ny, nx)),
                                                                                (27, nz, ny, nx)))
    force = (2e-5, 0.0)
    p3 = O.Params(n=(nx, ny, nz), lam=lam3, T=T, omega=omega, walls=(False, True, False), force=force + (0.0,))
    p2 = O.Params(n=(nx, ny), lam=lam2, T=T, omega=omega, force=force)
    fc = OF.Faces((nx, ny), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL], wall_velocity=(0.0, 0.0, 0.0, 0.02))

    def marginal(f):
        out = np.zeros((9, ny, nx))
        for i in range(27):
            k = int(np.where((c2 == c3[i, :2]).all(axis=1))[0][0])
            out[k] += f[i, 0]
        return out

    f2 = marginal(f3)
    for _ in range(12):
        f3 = OW.step(f3, p3, wall_u=(0.0, 0.02))
        f2 = OF.step_open(f2, p2, fc)
        assert np.abs(marginal(f3) - f2).max() < 1e-13
