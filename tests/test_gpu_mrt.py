"""GPU parity of the multi-relaxation-time collision (the extension that the
paper's conclusion, Sec. 4, names) on D2Q9 and D3Q27 lattices: the HIP path
through the C ABI against the FP64 oracle of oracle/elbm_mrt.py on the same
seeded states.

Tolerances are those of the LBGK parity (FP32 arithmetic on deviations):
one step max |f_gpu - f_oracle| <= 2e-7 and deviation rel-L2 <= 2e-6, ten
steps deviation rel-L2 <= 1e-5; FP16 deviation storage (11 significand
bits, relative quantum 2^-11 of a deviation) one step deviation rel-L2 <= 1e-3.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import elbm_mrt as OM
from gpu_helpers import dev_rel_l2, lib, random_state, rel_l2
from test_oracle_mrt import mrt_step_matrix

pytestmark = pytest.mark.gpu

CASES = {
    "stretched_periodic_ragged": (dict(n=(300, 77), lam=(2.0, 1.0), T=0.5, omega=1.6), 1.1, 1.3),
    "cubic_walls_y_force": (dict(n=(70, 33), T=1 / 3, omega=1.2, walls=(False, True), force=(1e-4, 0.0)), 0.8, 1.9),
    "stretched_walls_x": (dict(n=(40, 50), lam=(1.4, 1.0), T=0.4, omega=1.5, walls=(True, False)), 1.7, 1.0),
    "control_no_correction": (dict(n=(64, 64), T=0.5, omega=1.8, extended=False), 1.2, 1.5),
    "stretched_force_high_omega": (dict(n=(96, 40), lam=(2.0, 1.0), T=0.5, omega=1.9, force=(5e-5, -2e-5)),
                                   1.95, 0.7),
    "d3_periodic_ragged": (dict(n=(70, 37, 21), lam=(1.4, 1.0, 2.0), T=0.4, omega=1.6), 1.1, 1.3),
    "d3_channel_walls_y_force": (dict(n=(48, 24, 24), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9,
                                      walls=(False, True, False), force=(1e-5, 0.0, 0.0)), 1.2, 1.0),
    "d3_walls_xz": (dict(n=(20, 30, 18), T=1 / 3, omega=1.0, walls=(True, False, True)), 1.7, 1.5),
    "d3_force_periodic": (dict(n=(64, 16, 20), T=0.5, omega=1.3, force=(1e-4, -2e-4, 5e-5)), 0.9, 1.8),
    "d3_control_no_correction": (dict(n=(32, 40, 24), lam=(2.0, 1.0, 1.0), T=1 / 3, omega=1.7, extended=False),
                                 1.4, 1.2),
}


def _lattice(E, p, ob, og, storage="f32"):
    return E.Lattice(E.make_params(p.n, lam=p.lam, T=p.T, omega=p.omega, force=p.force, walls=p.walls,
                                   storage=storage, extended=p.extended, omega_bulk=ob, omega_ghost=og))


@pytest.mark.parametrize("case", sorted(CASES))
def test_mrt_one_and_ten_steps(case):
    E = lib()
    kw, ob, og = CASES[case]
    p = O.Params(**kw)
    f0 = random_state(p, seed=sum(map(ord, case)) % 997)
    lat = _lattice(E, p, ob, og)
    lat.set_populations(f0)
    g0 = lat.populations()
    lat.step(1)
    g1 = lat.populations()
    o1 = OM.step(g0, p, ob, og)
    assert np.abs(g1 - o1).max() <= 2e-7, case
    assert dev_rel_l2(g1, o1, p) <= 2e-6, case
    lat.step(9)
    g10 = lat.populations()
    o10 = OM.run(o1, p, 9, ob, og)
    assert dev_rel_l2(g10, o10, p) <= 1e-5, case
    # the collision conserves mass and (force aside) momentum
    r0, j0 = O.moments(g0, p.c, p.lam)
    r10, j10 = O.moments(g10, p.c, p.lam)
    assert abs(r10.sum() / r0.sum() - 1.0) < 1e-6
    lat.close()


@pytest.mark.parametrize("case,storage,gate", [
    ("stretched_periodic_ragged", "f16", 1e-3),
    ("d3_channel_walls_y_force", "f16", 1e-3),
    ("d3_periodic_ragged", "bf16", 1e-2),
])
def test_mrt_16bit_storage(case, storage, gate):
    """One step from an arbitrary state with 16-bit deviation storage: FP16
    (11 significand bits) within 1e-3 deviation rel-L2, BF16 (8 bits) within
    1e-2."""
    E = lib()
    kw, ob, og = CASES[case]
    p = O.Params(**kw)
    f0 = random_state(p, seed=11)
    lat = _lattice(E, p, ob, og, storage=storage)
    lat.set_populations(f0)
    g0 = lat.populations()
    lat.step(1)
    assert dev_rel_l2(lat.populations(), OM.step(g0, p, ob, og), p) <= gate
    lat.close()


@pytest.mark.parametrize("n,lam,walls,force", [
    ((128, 48), (2.0, 1.0), (False, True), (1e-4, 0.0)),
    ((64, 32, 16), (2.0, 1.0, 1.0), (False, True, False), (1e-4, 0.0, 0.0)),
])
def test_equal_rates_reproduce_the_lbgk_kernel(n, lam, walls, force):
    """omega_bulk = omega_ghost = omega is the LBGK step: the two GPU
    collisions agree to FP32 rounding over ten steps."""
    E = lib()
    p = O.Params(n=n, lam=lam, T=0.5, omega=1.7, walls=walls, force=force)
    f0 = random_state(p, seed=5)
    a = _lattice(E, p, p.omega, p.omega)
    b = E.Lattice(E.make_params(p.n, lam=p.lam, T=p.T, omega=p.omega, force=p.force, walls=p.walls))
    for L in (a, b):
        L.set_populations(f0)
        L.step(10)
    assert dev_rel_l2(a.populations(), b.populations(), p) <= 2e-6
    a.close()
    b.close()


def test_d3q27_mrt_kernel_choice_and_sample_steps():
    """A 16-bit D3Q27 lattice that the LDS-staged kernel would take runs the
    MRT collision on the register-pull kernel. With sample steps (the step
    kernel's diagnostics variant) an FP32 MRT lattice steps as without them,
    and its folded record agrees with a separate pass over the stored state
    (mass 1e-8, kinetic energy 1e-6, enstrophy 1e-5 relative)."""
    E = lib()
    p = O.Params(n=(64, 32, 16), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.8)
    kw = dict(lam=p.lam, T=p.T, omega=p.omega)
    lat16 = E.Lattice(E.make_params(p.n, storage="f16", omega_bulk=1.3, omega_ghost=1.1, **kw))
    assert lat16.kernel_info()["kernel"] == "register"
    lbgk = E.Lattice(E.make_params(p.n, storage="f16", **kw))
    assert lbgk.kernel_info()["kernel"] == "staged"
    lat16.close()
    lbgk.close()
    f0 = random_state(p, seed=21)
    lat = E.Lattice(E.make_params(p.n, omega_bulk=1.3, omega_ghost=1.1, diag_every=2, diag_capacity=4, **kw))
    ref = E.Lattice(E.make_params(p.n, omega_bulk=1.3, omega_ghost=1.1, **kw))
    for L in (lat, ref):
        L.set_populations(f0)
        L.step(2)
    assert dev_rel_l2(lat.populations(), ref.populations(), p) <= 1e-7
    d_fold = lat.diag_history()[-1]
    d_sep = lat.diag()
    assert d_sep["step"] == d_fold["step"] == 2
    assert abs(d_sep["mass"] / d_fold["mass"] - 1) <= 1e-8
    assert abs(d_sep["ke"] / d_fold["ke"] - 1) <= 1e-6
    assert abs(d_sep["enstrophy"] / d_fold["enstrophy"] - 1) <= 1e-5
    lat.close()
    ref.close()


@pytest.mark.parametrize("ob,og", [(1.2, 1.0), (0.8, 1.9)])
def test_shear_wave_follows_the_linear_eigenvalue(ob, og):
    """A shear wave of amplitude 1e-4 on a stretched lattice (lambda = (2, 1),
    T = 1/2, 64 nodes along x): its Fourier amplitude changes per step by the
    shear eigenvalue of the linearised MRT step (built from the paper's
    equations in tests/test_oracle_mrt.py), to 1e-5 relative once the other
    modes have decayed -- the shear rate set by omega alone."""
    E = lib()
    lam, T, omega, N = (2.0, 1.0), 0.5, 1.6, 64
    p = O.Params(n=(N, 4), lam=lam, T=T, omega=omega)
    k = (2.0 * math.pi / (N * lam[0]), 0.0)
    x = np.arange(N) * lam[0]
    rho = np.ones((4, N))
    u = np.zeros((2, 4, N))
    u[1] = 1e-4 * np.sin(k[0] * x)[None, :]
    lat = _lattice(E, p, ob, og)
    lat.set_populations(O.equilibrium(rho, u, T, lam, p.c))
    lat.step(200)  # the ghost modes decay by |1 - omega_ghost| per step
    amps = []
    for _ in range(20):
        lat.step(1)
        _, v = lat.fields()
        amps.append((v[1][0] * np.exp(-1j * k[0] * x)).sum() / N)
    ratios = np.array(amps[1:]) / np.array(amps[:-1])
    M = mrt_step_matrix(k, (0.0, 0.0), T, omega, lam, ob, og)
    w, V = np.linalg.eig(M)
    c = O.velocity_set(2)
    cand = np.argsort(-np.abs(w))[:4]
    mu = w[max(cand, key=lambda m: abs((lam[1] * c[:, 1] * V[:, m]).sum()) / np.abs(V[:, m]).sum())]
    assert np.abs(ratios / mu - 1.0).max() < 1e-5, (ratios[-1], mu)
    lat.close()


@pytest.mark.parametrize("ob,og", [(1.2, 1.0), (0.8, 1.9), (1.9, 1.9)])
def test_d3q27_shear_wave_viscosity(ob, og):
    """Sec. 3.1 on D3Q27 with the MRT collision: a shear wave u_z = A sin(k x)
    on the stretched lattice lambda = (2, 1, 1), T = 1/2, omega = 1.4 (128
    nodes along x) decays at nu k^2 with nu = (1/omega - 1/2) T, whatever the
    bulk and higher-order rates, to 1% (the fitted rate of the Fourier
    amplitude over steps 100-400)."""
    E = lib()
    lam, T, omega, N = (2.0, 1.0, 1.0), 0.5, 1.4, 128
    n = (N, 4, 4)
    p = O.Params(n=n, lam=lam, T=T, omega=omega)
    k = 2.0 * math.pi / (N * lam[0])
    x = np.arange(N) * lam[0]
    rho = np.ones((4, 4, N))
    u = np.zeros((3, 4, 4, N))
    u[2] = 1e-4 * np.sin(k * x)[None, None, :]
    lat = E.Lattice(E.make_params(n, lam=lam, T=T, omega=omega, omega_bulk=ob, omega_ghost=og))
    lat.set_populations(O.equilibrium(rho, u, T, lam, p.c))
    lat.step(100)
    t, a = [], []
    for s in range(7):
        _, v = lat.fields()
        t.append(100 + 50 * s)
        a.append(abs((v[2][0, 0] * np.exp(-1j * k * x)).sum()) / N)
        lat.step(50)
    rate = -np.polyfit(t, np.log(a), 1)[0]
    nu = (1.0 / omega - 0.5) * T
    assert rate / (nu * k * k) == pytest.approx(1.0, abs=1e-2)
    lat.close()


@pytest.mark.parametrize("mode", ["batch", "batch_graph", "static"])
def test_mrt_lattices_in_batched_launches(mode):
    """MRT lattices batched with LBGK lattices of the same shapes (their own
    kernel classes: the D3Q27 MRT variant, the D2Q9 kernel's runtime branch)
    advance bitwise as alone, through the batch object with and without
    HIP-graph replay and through the allocation-free entry point."""
    E = lib()
    specs = [
        ((48, 24, 24), (2.0, 1.0, 1.0), (False, True, False), (1e-5, 0.0, 0.0), "f32", (1.2, 1.0)),
        ((48, 24, 24), (2.0, 1.0, 1.0), (False, True, False), (1e-5, 0.0, 0.0), "f32", None),
        ((64, 32, 16), (1.0, 1.0, 1.0), (False, False, False), None, "f16", (0.9, 1.6)),
        ((64, 32, 16), (1.0, 1.0, 1.0), (False, False, False), None, "f16", None),
        ((96, 40), (2.0, 1.0), (False, True), (5e-5, 0.0), "f32", (1.3, 1.1)),
        ((96, 40), (2.0, 1.0), (False, True), (5e-5, 0.0), "f32", None),
        ((70, 37, 21), (1.4, 1.0, 2.0), (False, False, False), None, "bf16", (1.1, 1.3)),
    ]
    steps = [6, 9, 4, 7, 11, 3, 5]

    def make():
        out = []
        for k, (n, lam, walls, force, st, rates) in enumerate(specs):
            p = O.Params(n=n, lam=lam, T=0.5, omega=1.7, walls=walls, force=force)
            kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
            lat = E.Lattice(E.make_params(n, lam=lam, T=0.5, omega=1.7, walls=walls, force=force, storage=st,
                                          **kw))
            lat.set_populations(random_state(p, seed=40 + k))
            out.append(lat)
        return out

    alone = make()
    for lat, k in zip(alone, steps):
        lat.step(k)
    ref = [lat.populations() for lat in alone]
    batched = make()
    if mode == "static":
        E.batch_run_static(batched, steps)
    else:
        b = E.Batch(len(batched))
        b.run(batched, steps, use_graph=mode == "batch_graph")
        b.close()
    for lat, k, r in zip(batched, steps, ref):
        assert lat.step_count == k
        assert np.array_equal(lat.populations(), r)
    for lat in alone + batched:
        lat.close()


def test_mrt_checkpoint_resumes_bitwise_and_checks_the_rates():
    """elbm_save / elbm_load of an MRT lattice: a resumed run is bitwise the
    uninterrupted one; a checkpoint does not load into a lattice with other
    rates or the LBGK collision."""
    E = lib()
    p = O.Params(n=(48, 24, 24), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, walls=(False, True, False),
                 force=(1e-5, 0.0, 0.0))
    kw = dict(lam=p.lam, T=p.T, omega=p.omega, walls=p.walls, force=p.force)
    lat = E.Lattice(E.make_params(p.n, omega_bulk=1.2, omega_ghost=1.0, **kw))
    lat.set_populations(random_state(p, seed=8))
    lat.step(5)
    ck = lat.save()
    lat.step(7)
    want = lat.populations()
    other = E.Lattice(E.make_params(p.n, omega_bulk=1.2, omega_ghost=1.0, **kw))
    other.load(ck)
    other.step(7)
    assert np.array_equal(other.populations(), want)
    for bad in (E.make_params(p.n, omega_bulk=1.3, omega_ghost=1.0, **kw), E.make_params(p.n, **kw)):
        L = E.Lattice(bad)
        with pytest.raises(E.ElbmError):
            L.load(ck)
        L.close()
    lat.close()
    other.close()


@pytest.mark.parametrize("n,lam,T,u_adv", [
    ((96, 40), (2.0, 1.0), 0.5, (0.06, -0.02)),
    ((48, 24, 20), (1.4, 1.0, 2.0), 0.55, (0.05, 0.02, -0.03)),
])
def test_mrt_with_an_advected_reference(n, lam, T, u_adv):
    """Deviations stored from the advected reference w(u_adv) (periodic
    lattices): the MRT step from an arbitrary state around u_adv matches the
    oracle to the LBGK bounds (one step 2e-7 max, ten steps 1e-5 deviation
    rel-L2, deviations taken from w(u_adv))."""
    E = lib()
    p = O.Params(n=n, lam=lam, T=T, omega=1.7)
    g = np.random.default_rng(17)
    grid = tuple(reversed(n))
    rho = 1.0 + 0.02 * g.standard_normal(grid)
    u = 0.03 * g.standard_normal((p.D,) + grid) + np.array(u_adv).reshape((p.D,) + (1,) * p.D)
    f0 = O.equilibrium(rho, u, T, lam, p.c) * (1.0 + 0.01 * g.standard_normal((p.c.shape[0],) + grid))
    lat = E.Lattice(E.make_params(n, lam=lam, T=T, omega=p.omega, u_adv=u_adv, omega_bulk=1.3, omega_ghost=1.1))
    lat.set_populations(f0)
    g0 = lat.populations()
    lat.step(1)
    o1 = OM.step(g0, p, 1.3, 1.1)
    assert np.abs(lat.populations() - o1).max() <= 2e-7
    lat.step(9)
    o10 = OM.run(o1, p, 9, 1.3, 1.1)
    assert dev_rel_l2(lat.populations(), o10, p, u_ref=u_adv) <= 1e-5
    lat.close()


def test_d2q9_mrt_sample_steps():
    """D2Q9 MRT (the runtime branch of the D2Q9 kernel) with walls, force and
    sample steps: the state is that of the run without samples, and the
    folded record agrees with a separate pass over the stored state."""
    E = lib()
    p = O.Params(n=(96, 40), lam=(2.0, 1.0), T=0.5, omega=1.8, walls=(False, True), force=(1e-5, 0.0))
    kw = dict(lam=p.lam, T=p.T, omega=p.omega, walls=p.walls, force=p.force, omega_bulk=1.1, omega_ghost=1.4)
    f0 = random_state(p, seed=23)
    lat = E.Lattice(E.make_params(p.n, diag_every=3, diag_capacity=4, **kw))
    ref = E.Lattice(E.make_params(p.n, **kw))
    for L in (lat, ref):
        L.set_populations(f0)
        L.step(6)
    assert dev_rel_l2(lat.populations(), ref.populations(), p) <= 1e-7
    d_fold = lat.diag_history()[-1]
    d_sep = lat.diag()
    assert d_sep["step"] == d_fold["step"] == 6
    assert abs(d_sep["mass"] / d_fold["mass"] - 1) <= 1e-8
    assert abs(d_sep["ke"] / d_fold["ke"] - 1) <= 1e-6
    assert abs(d_sep["enstrophy"] / d_fold["enstrophy"] - 1) <= 1e-5
    lat.close()
    ref.close()
