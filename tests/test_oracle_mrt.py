"""Pins of the multi-relaxation-time collision oracle (oracle/elbm_mrt.py)."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import elbm_mrt as OM
from test_oracle_linear import step_matrix


def _state(p, seed):
    g = np.random.default_rng(seed)
    grid = tuple(reversed(p.n))
    rho = 1.0 + 0.02 * g.standard_normal(grid)
    u = 0.04 * g.standard_normal((p.D,) + grid)
    f = O.equilibrium(rho, u, p.T, p.lam, p.c)
    return f * (1.0 + 0.01 * g.standard_normal(f.shape))


@pytest.mark.parametrize("n,lam,T", [((10, 8), (2.0, 1.0), 0.5), ((6, 5, 4), (1.4, 1.0, 1.0), 0.55)])
def test_equal_rates_are_lbgk(n, lam, T):
    p = O.Params(n=n, lam=lam, T=T, omega=1.7, force=(1e-4,) + (0.0,) * (len(n) - 1))
    f = _state(p, 1)
    assert np.abs(OM.collide(f, p, 1.7, 1.7) - O.collide(f, p)).max() < 1e-15


@pytest.mark.parametrize("D,lam,T", [(2, (2.0, 1.0), 0.5), (3, (1.4, 1.0, 2.0), 0.55)])
def test_grad_map_carries_exactly_its_stress(D, lam, T):
    """G(Pi) has no mass, no momentum and second moments Pi (brute force)."""
    c = O.velocity_set(D)
    g = np.random.default_rng(2)
    u = 0.05 * g.standard_normal(D)
    P = [T + u[a] ** 2 + 0.01 * g.standard_normal() for a in range(D)]
    A = 1e-3 * g.standard_normal((D, D))
    Pi = A + A.T
    G = OM.grad_map(Pi, u, P, lam, c)
    v = c * np.array(lam)[None, :]
    assert abs(G.sum()) < 1e-17
    for a in range(D):
        assert abs((v[:, a] * G).sum()) < 1e-17
    for a, b in itertools.product(range(D), range(D)):
        assert (v[:, a] * v[:, b] * G).sum() == pytest.approx(Pi[a, b], abs=1e-17)


def test_conservation_with_three_rates():
    p = O.Params(n=(9, 7), lam=(2.0, 1.0), T=0.5, omega=1.6, force=(2e-4, -1e-4))
    f = _state(p, 3)
    r0, j0 = O.moments(f, p.c, p.lam)
    f1 = OM.step(f, p, 1.1, 1.3)
    r1, j1 = O.moments(f1, p.c, p.lam)
    assert r1.sum() == pytest.approx(r0.sum(), rel=1e-14)
    for a in range(2):
        assert j1[a].sum() - j0[a].sum() == pytest.approx(p.force[a] * r0.sum(), rel=1e-9)


def mrt_step_matrix(k, U, T, omega, lam, omega_bulk, omega_ghost):
    """The linearised multi-relaxation-time step for one Fourier mode, from the
    LBGK one of test_oracle_linear: its collision part is I + omega (J - I),
    which gives the equilibrium Jacobian J; the non-equilibrium is (I - J)
    delta, its stress M2 (I - J) delta, split into trace and deviator and
    mapped back by the linear Grad map at the base state."""
    c = O.velocity_set(2)
    Q = c.shape[0]
    shift = np.diag([np.exp(-1j * (k[0] * c[i, 0] * lam[0] + k[1] * c[i, 1] * lam[1])) for i in range(Q)])
    coll = step_matrix(k, U, T, omega, lam, omega_bulk=omega_bulk) @ np.linalg.inv(shift)
    J = (coll - np.eye(Q)) / omega + np.eye(Q)
    v = [lam[a] * c[:, a] for a in range(2)]
    M2 = np.array([v[0] * v[0], v[1] * v[1], v[0] * v[1]])
    Pb = [T + U[a] ** 2 for a in range(2)]
    Gdev = np.zeros((Q, 3))
    Giso = np.zeros((Q, 3))
    for col, (xx, yy, xy) in enumerate(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0))):
        tr = 0.5 * (xx + yy)
        Giso[:, col] = OM.grad_map([[tr, 0.0], [0.0, tr]], U, Pb, lam, c)
        Gdev[:, col] = OM.grad_map([[xx - tr, xy], [xy, yy - tr]], U, Pb, lam, c)
    N = np.eye(Q) - J
    C = (J + (1.0 - omega_ghost) * N + (omega_ghost - omega) * Gdev @ M2 @ N
         + (omega_ghost - omega_bulk) * Giso @ M2 @ N)
    return C @ shift


def test_oracle_step_is_the_linear_map():
    """A small perturbation of all populations at one wave vector on a
    stretched box evolves under the oracle's MRT step by the linear map, to
    1e-6."""
    lam, T, omega, ob, og = (2.0, 1.0), 0.5, 1.6, 1.1, 1.3
    nx, ny = 12, 24
    p = O.Params(n=(nx, ny), lam=lam, T=T, omega=omega)
    L = nx * lam[0]
    k = (2.0 * math.pi / L, 2.0 * math.pi / L)
    X = (np.arange(nx) * lam[0])[None, :]
    Y = (np.arange(ny) * lam[1])[:, None]
    ph = k[0] * X + k[1] * Y
    g = np.random.default_rng(4)
    F = O.equilibrium(np.ones((ny, nx)), np.zeros((2, ny, nx)), T, lam, p.c)
    amp = 1e-8 * (g.standard_normal(9) + 1j * g.standard_normal(9))
    f = F + np.real(amp[:, None, None] * np.exp(1j * ph)[None])
    M = mrt_step_matrix(k, (0.0, 0.0), T, omega, lam, ob, og)

    def delta(f):
        return ((f - F) * np.exp(-1j * ph)[None]).sum(axis=(1, 2)) / (nx * ny) * 2.0

    for _ in range(5):
        d0 = delta(f)
        f = OM.step(f, p, ob, og)
        assert np.abs(delta(f) - M @ d0).max() < 1e-6 * np.abs(d0).max()


@pytest.mark.parametrize("lam,T", [((1.0, 1.0), 1 / 3), ((2.0, 1.0), 0.5)])
@pytest.mark.parametrize("ob,og", [(1.2, 1.0), (0.8, 1.9), (1.6, 1.6)])
def test_long_waves_shear_and_sound(lam, T, ob, og):
    """At long waves (2048 nodes): the shear mode decays by nu k^2 with
    nu = (1/omega - 1/2) T whatever the other two rates (1e-4); the sound
    modes travel at sqrt(T) and decay by (nu + nu_b) k^2 / 2 with
    nu_b = (1/omega_bulk - 1/2) T (1e-4)."""
    omega = 1.6
    nu = (1.0 / omega - 0.5) * T
    nub = (1.0 / ob - 0.5) * T
    N = 2048
    k = (2.0 * math.pi / (N * lam[0]), 0.0)
    M = mrt_step_matrix(k, (0.0, 0.0), T, omega, lam, ob, og)
    w, V = np.linalg.eig(M)
    c = O.velocity_set(2)
    # shear: largest transverse momentum among the near-unit eigenvalues
    cand = np.argsort(-np.abs(w))[:4]
    shear = max(cand, key=lambda m: abs((lam[1] * c[:, 1] * V[:, m]).sum()) / np.abs(V[:, m]).sum())
    assert -math.log(abs(w[shear])) / (nu * k[0] ** 2) == pytest.approx(1.0, abs=1e-4)
    cs = math.sqrt(T)
    sound = [m for m in cand if abs(abs(np.angle(w[m])) / (cs * k[0]) - 1.0) < 1e-3]
    assert len(sound) == 2
    for m in sound:
        assert -math.log(abs(w[m])) / (0.5 * (nu + nub) * k[0] ** 2) == pytest.approx(1.0, abs=1e-4)


def _max_growth_at_rest(T, omega, lam, ob, og, nk=25):
    worst = 0.0
    for kx in np.linspace(0.0, math.pi / lam[0], nk):
        for ky in np.linspace(-math.pi / lam[1], math.pi / lam[1], 2 * nk - 1):
            M = mrt_step_matrix((kx, ky), (0.0, 0.0), T, omega, lam, ob, og)
            worst = max(worst, float(np.abs(np.linalg.eigvals(M)).max()))
    return worst


def test_linear_stability_at_rest():
    """The linearised MRT step at rest: no growing mode at the rates of the
    GPU parity cases on the stretched lattice (omega = 1.6), nor at omega =
    1.9745 on the regular lattice; but on lambda = (2, 1) at omega = 1.9745
    with omega_bulk = 1.2, omega_ghost = 1.5 a mode grows by 0.37% per step
    (k = (pi/2, +-1.37)): the stretching, not the rates alone, makes it."""
    assert _max_growth_at_rest(0.5, 1.6, (2.0, 1.0), 1.1, 1.3) < 1.0 + 1e-9
    assert _max_growth_at_rest(1 / 3, 1.9745, (1.0, 1.0), 1.2, 1.5) < 1.0 + 1e-9
    assert _max_growth_at_rest(1 / 3, 1.9745, (2.0, 1.0), 1.2, 1.5) > 1.003


def _d3_wave(ob, og, kind, N=256):
    """Per-step ratio of a long plane wave's Fourier amplitude (k along x, N
    nodes) run by the D3Q27 MRT oracle on lambda = (2, 1, 1), T = 1/2,
    omega = 1.4, after 40 steps of transients: kind 'shear' (u_z = A sin kx,
    amplitude of u_z) or 'sound' (the right-going wave rho = 1 + A sin kx,
    u_x = c_s A sin kx, amplitude of its invariant c_s drho + j_x)."""
    lam, T, omega = (2.0, 1.0, 1.0), 0.5, 1.4
    p = O.Params(n=(N, 3, 3), lam=lam, T=T, omega=omega)
    k = 2.0 * math.pi / (N * lam[0])
    x = np.arange(N) * lam[0]
    cs = math.sqrt(T)
    A = 1e-6
    wave = np.sin(k * x)[None, None, :] * np.ones((3, 3, 1))
    rho = np.ones((3, 3, N))
    u = np.zeros((3, 3, 3, N))
    if kind == "shear":
        u[2] = A * wave
    else:
        rho = rho + A * wave
        u[0] = A * cs * wave
    f = OM.run(O.equilibrium(rho, u, T, lam, p.c), p, 40, ob, og)
    amps = []
    for _ in range(12):
        f = OM.step(f, p, ob, og)
        r, j = O.moments(f, p.c, p.lam)
        field = j[2] / r if kind == "shear" else cs * (r - 1.0) + j[0]
        amps.append((field[0, 0] * np.exp(-1j * k * x)).sum() / N)
    return np.array(amps[1:]) / np.array(amps[:-1]), k, (1.0 / omega - 0.5) * T, cs


@pytest.mark.parametrize("ob,og", [(0.8, 1.2), (1.6, 1.2)])
def test_d3q27_long_waves(ob, og):
    """D3Q27 (256 nodes along x of a stretched lattice): the shear wave
    decays per step by nu k^2 (5e-4) whatever the other rates; the sound wave
    travels at sqrt(T) (1e-4) and decays by (2 nu + nu_b) k^2 / 3, the
    Navier-Stokes attenuation with shear viscosity nu and a trace relaxed at
    omega_bulk, nu_b = (1/omega_bulk - 1/2) T (2e-3; 1.0 - 1.3e-3 measured,
    the rest is the wave's finite k). A trace taken over two axes, or the
    whole pressure correction at the shear rate's factor, misses by far more."""
    rat, k, nu, cs = _d3_wave(ob, og, "shear")
    assert -math.log(abs(rat[-1])) / (nu * k * k) == pytest.approx(1.0, abs=5e-4)
    rat, k, nu, cs = _d3_wave(ob, og, "sound")
    nub = (1.0 / ob - 0.5) * 0.5
    assert -np.angle(rat[-1]) / (cs * k) == pytest.approx(1.0, abs=1e-4)
    assert -math.log(abs(rat[-1])) / ((2.0 * nu + nub) * k * k / 3.0) == pytest.approx(1.0, abs=2e-3)


@pytest.mark.parametrize("T,rates,unstable", [
    (0.5, None, True), (0.5, (1.0, 1.0), False), (0.5, (1.0, 1.5), False),
    (1 / 3, None, False), (1 / 3, (1.0, 1.0), True), (1 / 3, (1.0, 1.5), False),
])
def test_linear_stability_of_the_shear_layer_stream(T, rates, unstable):
    """The double shear layer's stream (u = 0.1 along x) at the viscosity of
    Re = 3e4 on 256 nodes (omega = 1.99), cubic D2Q9, linearised about the
    uniform state (wave vectors on a 17 x 33 grid of the Brillouin zone):
    at T = 1/2 LBGK has modes growing by about 2% per step and the MRT
    collision with omega_bulk = 1 (omega_ghost = 1 or 1.5) none; at T = 1/3
    LBGK is stable and omega_ghost = 1 is not (0.9% per step), omega_ghost =
    1.5 is. The GPU runs of the shear layer follow this (tests/test_gpu_study.py)."""
    lam, omega, U = (1.0, 1.0), 1.99, (0.1, 0.0)
    worst = 0.0
    for kx in np.linspace(0.0, math.pi, 17):
        for ky in np.linspace(-math.pi, math.pi, 33):
            if rates is None:
                M = step_matrix((kx, ky), U, T, omega, lam)
            else:
                M = mrt_step_matrix((kx, ky), U, T, omega, lam, *rates)
            worst = max(worst, float(np.abs(np.linalg.eigvals(M)).max()))
    if unstable:
        assert worst > 1.005
    else:
        assert worst < 1.0 + 1e-9
