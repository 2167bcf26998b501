"""Pins of the open-boundary oracle (oracle/elbm_faces.py): properties its
rules must have whatever the reading, checked without the GPU."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle import elbm_faces as OF
from oracle import elbm_mrt as OM


@pytest.mark.parametrize("lam", [(1.0, 1.0), (2.0, 1.0), (1.0, 1.4)])
def test_grad_populations_carry_the_moments_they_are_built_from(lam):
    g = np.random.default_rng(11)
    c = O.velocity_set(2)
    T = 1 / 3 if lam == (1.0, 1.0) else 0.5
    for _ in range(5):
        rho = 1.0 + 0.1 * g.standard_normal()
        u = 0.05 * g.standard_normal(2)
        A = 1e-3 * g.standard_normal((2, 2))
        Pi = A + A.T
        f = OF.grad_populations(rho, u, Pi, T, lam, c)
        v = c * np.array(lam)[None, :]
        assert f.sum() == pytest.approx(rho, abs=1e-14)
        for a in range(2):
            assert (v[:, a] * f).sum() == pytest.approx(rho * u[a], abs=1e-14)
        for a, b in itertools.product(range(2), range(2)):
            want = rho * ((T if a == b else 0.0) + u[a] * u[b]) + Pi[a, b]
            assert (v[:, a] * v[:, b] * f).sum() == pytest.approx(want, abs=1e-14), (a, b)


def _uniform(n, lam, T, u0):
    nx, ny = n
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = u0[0]
    u[1] = u0[1]
    return O.equilibrium(rho, u, T, lam, O.velocity_set(2))


@pytest.mark.parametrize("lam", [(1.0, 1.0), (2.0, 1.0)])
def test_uniform_stream_through_inlet_and_outlet_stays_uniform(lam):
    """Inlet (x-), outlet (x+), symmetry planes (y-, y+): the uniform stream
    at the inlet velocity is a steady state of every rule, including the
    anomaly ghosts (on lambda_x = 2 the anomaly Q~_x is nonzero but uniform,
    so its ghost must be even at inlet and outlet)."""
    n = (12, 7)
    T = 1 / 3
    u0 = (0.05, 0.0)
    p = O.Params(n=n, lam=lam, T=T, omega=1.7)
    fc = OF.Faces(n, [OF.INLET, OF.OUTLET, OF.SYMMETRY, OF.SYMMETRY], inlet_velocity=(u0, u0, u0, u0))
    f0 = _uniform(n, lam, T, u0)
    f = OF.run_open(f0, p, fc, 40)
    assert np.abs(f - f0).max() < 1e-14


def _mirror_y(f, c):
    """Populations of the mirror image about the plane between rows."""
    Q = c.shape[0]
    out = np.empty_like(f)
    for i in range(Q):
        cm = c[i].copy()
        cm[1] = -cm[1]
        k = int(np.where((c == cm).all(axis=1))[0][0])
        out[k] = f[i][::-1, :]
    return out


@pytest.mark.parametrize("lam", [(1.0, 1.0), (2.0, 1.0)])
def test_symmetry_plane_reproduces_the_mirrored_walled_channel(lam):
    """A channel between Grad walls (y- and y+) whose state is mirror
    symmetric about its centre plane equals, in its lower half, the half
    channel with a wall at y- and a symmetry plane at y+: checks the specular
    rule, the odd anomaly ghost and that the wall rule of a high face is the
    mirror of the low face's."""
    c = O.velocity_set(2)
    nx, m = 6, 5
    T = 0.5 if lam[0] == 2.0 else 1 / 3
    g = np.random.default_rng(3)
    p_full = O.Params(n=(nx, 2 * m), lam=lam, T=T, omega=1.6, force=(2e-5, 0.0))
    p_half = O.Params(n=(nx, m), lam=lam, T=T, omega=1.6, force=(2e-5, 0.0))
    rho = 1.0 + 0.01 * g.standard_normal((m, nx))
    u = 0.02 * g.standard_normal((2, m, nx))
    fh = O.equilibrium(rho, u, T, lam, c) * (1.0 + 0.002 * g.standard_normal((9, m, nx)))
    ff = np.concatenate([fh, _mirror_y(fh, c)], axis=1)
    full = OF.Faces((nx, 2 * m), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL])
    half = OF.Faces((nx, m), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.SYMMETRY])
    for _ in range(15):
        ff = OF.step_open(ff, p_full, full)
        fh = OF.step_open(fh, p_half, half)
    assert np.abs(ff[:, :m, :] - fh).max() < 1e-14
    assert np.abs(ff - _mirror_y(ff, c)).max() < 1e-14


def _poiseuille_error(ny, lam_x=1.0):
    T, omega, g = 1 / 3, 1.0, 1e-6
    nx = 3
    lam = (lam_x, 1.0)
    p = O.Params(n=(nx, ny), lam=lam, T=T, omega=omega, force=(g, 0.0))
    fc = OF.Faces((nx, ny), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL])
    f = _uniform((nx, ny), lam, T, (0.0, 0.0))
    prev = None
    for it in range(400):
        f = OF.run_open(f, p, fc, 50)
        _, u = O.velocity(f, p)
        prof = u[0][:, 0]
        if prev is not None and np.abs(prof - prev).max() < 1e-12 * np.abs(prof).max():
            break
        prev = prof
    y = (np.arange(ny) + 0.5)  # distance from the wall at -1/2
    H = float(ny)
    exact = g / (2.0 * p.nu) * y * (H - y)
    return float(np.sqrt(np.mean((prof - exact) ** 2)) / np.sqrt(np.mean(exact ** 2)))


def test_grad_walls_converge_to_the_poiseuille_parabola_at_second_order():
    """Force-driven channel between Grad walls (periodic x): the steady
    velocity profile approaches the Navier-Stokes parabola through the
    halfway walls, and halving the node spacing cuts the error by about 4."""
    # (measured: 9.5e-2 at 6 rows, 2.38e-2 at 12, 5.9e-3 at 24: the straight
    # line from the wall through the inward neighbour misses the parabola's
    # curvature over one and a half node spacings)
    e6 = _poiseuille_error(6)
    e12 = _poiseuille_error(12)
    assert e12 < 3e-2
    assert 3.6 < e6 / e12 < 4.4, (e6, e12)


@pytest.mark.parametrize("omega", [1.0, 1.6])
@pytest.mark.parametrize("lam,T", [((1.0, 1.0), 1 / 3), ((2.0, 1.0), 0.5)])
def test_grad_walls_hold_couette_flow_linear(omega, lam, T):
    """Plane Couette flow between a resting Grad wall (y-) and one moving at
    u_w (y+): the steady profile is the straight line from 0 to u_w through
    the two halfway walls, to 1e-8 of u_w. The wall's non-equilibrium
    stress decides it: with its sign reversed the profile misses by 24%, and
    without it by 8%."""
    ny, nx, uw = 8, 3, 0.01
    p = O.Params(n=(nx, ny), lam=lam, T=T, omega=omega)
    fc = OF.Faces((nx, ny), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL], wall_velocity=(0.0, 0.0, 0.0, uw))
    f = OF.run_open(_uniform((nx, ny), lam, T, (0.0, 0.0)), p, fc, 3000)
    _, u = O.velocity(f, p)
    y = np.arange(ny) + 0.5
    assert np.abs(u[0][:, 0] - uw * y / ny).max() < 1e-8 * uw
    assert np.abs(u[1]).max() < 1e-14


def test_resting_inlet_is_halfway_bounce_back():
    """An inlet with zero velocity is a resting halfway bounce-back wall: with
    the anomaly correction off (its ghost parities differ), a box with such
    inlets on both x faces steps exactly as the bounce-back lattice of
    elbm_oracle (walls on x, periodic y) does."""
    c = O.velocity_set(2)
    n, lam, T = (7, 6), (2.0, 1.0), 0.5
    g = np.random.default_rng(9)
    rho = 1.0 + 0.01 * g.standard_normal((n[1], n[0]))
    u = 0.03 * g.standard_normal((2, n[1], n[0]))
    f = O.equilibrium(rho, u, T, lam, c) * (1.0 + 0.002 * g.standard_normal((9, n[1], n[0])))
    pb = O.Params(n=n, lam=lam, T=T, omega=1.7, walls=(True, False), extended=False)
    po = O.Params(n=n, lam=lam, T=T, omega=1.7, extended=False)
    fc = OF.Faces(n, [OF.INLET, OF.INLET, OF.PERIODIC, OF.PERIODIC])
    fb = fo = f
    for _ in range(12):
        fb = O.step(fb, pb)
        fo = OF.step_open(fo, po, fc)
    assert np.abs(fb - fo).max() < 1e-15


# ---- the multi-relaxation-time collision under open faces ----

def _plate_faces(n, lam, T):
    nx, ny = n
    kinds = [OF.INLET, OF.OUTLET, [OF.SYMMETRY] * (nx // 3) + [OF.WALL] * (nx - nx // 3), OF.SYMMETRY]
    return OF.Faces(n, kinds, inlet_velocity=((0.05, 0.0),) * 4)


def _noisy(n, lam, T, seed):
    g = np.random.default_rng(seed)
    nx, ny = n
    rho = 1.0 + 0.01 * g.standard_normal((ny, nx))
    u = 0.04 * g.standard_normal((2, ny, nx))
    f = O.equilibrium(rho, u, T, lam, O.velocity_set(2))
    return f * (1.0 + 0.002 * g.standard_normal(f.shape))


@pytest.mark.parametrize("lam,T", [((1.0, 1.0), 1 / 3), ((2.0, 1.0), 0.5)])
def test_mrt_faces_with_equal_rates_are_the_lbgk_faces(lam, T):
    """Every face kind at once (inlet, outlet, a bottom face half symmetry
    and half Grad wall, a symmetry top): with omega_bulk = omega_ghost =
    omega the multi-relaxation-time step is the LBGK step, to 1e-14."""
    n = (12, 9)
    p = O.Params(n=n, lam=lam, T=T, omega=1.7)
    fc = _plate_faces(n, lam, T)
    f = _noisy(n, lam, T, 3)
    a = OF.run_open(f, p, fc, 6)
    b = OF.run_open(f, p, fc, 6, rates=(1.7, 1.7))
    assert np.abs(a - b).max() < 1e-14


@pytest.mark.parametrize("rates", [(1.6, 1.3), (1.6, 0.8), (1.0, 1.3), (1.9, 0.8)])
@pytest.mark.parametrize("lam,T", [((1.0, 1.0), 1 / 3), ((2.0, 1.0), 0.5)])
def test_mrt_grad_walls_on_couette_flow(rates, lam, T):
    """Plane Couette flow between Grad walls with the MRT collision (omega =
    1.6). With omega_bulk = omega the higher-order rate leaves the steady
    profile the straight line through the halfway walls to 1e-8 of the wall
    velocity, and mass is conserved to rounding. With omega_bulk != omega the
    bulk's second-order normal stresses, which the first-order Grad stress
    does not carry, leave the profile within 2e-5 of the line and the walls
    exchanging mass with the flow at under 2e-7 of it per step (measured
    2-9e-8)."""
    ny, nx, uw = 8, 3, 0.01
    p = O.Params(n=(nx, ny), lam=lam, T=T, omega=1.6)
    fc = OF.Faces((nx, ny), [OF.PERIODIC, OF.PERIODIC, OF.WALL, OF.WALL], wall_velocity=(0.0, 0.0, 0.0, uw))
    f = OF.run_open(_uniform((nx, ny), lam, T, (0.0, 0.0)), p, fc, 3000, rates=rates)
    m0 = O.moments(f, p.c, p.lam)[0].sum()
    f = OF.run_open(f, p, fc, 500, rates=rates)
    r, u = O.velocity(f, p)
    y = np.arange(ny) + 0.5
    err = np.abs(u[0][:, 0] - uw * y / ny).max() / uw
    drift = abs(r.sum() / m0 - 1.0) / 500
    if rates[0] == p.omega:
        assert err < 1e-8
        assert np.abs(u[1]).max() < 1e-14
        assert drift < 1e-15
    else:
        assert err < 2e-5
        assert drift < 2e-7


@pytest.mark.parametrize("rates", [(1.0, 1.3), (1.9, 1.2)])
def test_mrt_bulk_stress_has_the_split_the_grad_wall_uses(rates):
    """The reading behind the Grad wall's stress under the MRT collision: in
    the bulk, the pre-collision non-equilibrium normal stress of a sound wave
    (cubic lattice, T = 1/3, omega = 1.6) is -rho T (S_dev / omega +
    S_iso / omega_bulk), S = grad u + grad u^T split into its deviator and
    trace parts, to 2%; the LBGK form -rho T S / omega misses it by more
    than 5%."""
    ob, og = rates
    nx, ny, lam, T, omega = 64, 8, (1.0, 1.0), 1 / 3, 1.6
    p = O.Params(n=(nx, ny), lam=lam, T=T, omega=omega)
    k = 2.0 * np.pi / nx
    x = np.arange(nx)
    rho = 1.0 + 1e-4 * np.sin(k * x)[None, :] * np.ones((ny, 1))
    f = OM.run(O.equilibrium(rho, np.zeros((2, ny, nx)), T, lam, p.c), p, 37, ob, og)
    fs = O.stream(f, p.c, p.walls)
    r, j = O.moments(fs, p.c, p.lam)
    u = j / r
    pxx = np.tensordot(p.c[:, 0] ** 2, fs, axes=(0, 0)) - r * (T + u[0] ** 2)
    S = 2.0 * (np.roll(u[0], -1, axis=1) - np.roll(u[0], 1, axis=1)) / 2.0
    iso = 0.5 * S
    split = -r * T * ((S - iso) / omega + iso / ob)
    lbgk = -r * T * S / omega
    sel = np.abs(split) > 0.3 * np.abs(split).max()
    assert np.median(pxx[sel] / split[sel]) == pytest.approx(1.0, abs=0.02)
    assert abs(np.median(pxx[sel] / lbgk[sel]) - 1.0) > 0.05
