"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs, element by element.

Tolerances (FP32 arithmetic on deviations, FP64 oracle):
* one step from an arbitrary state: max |f_gpu - f_oracle| <= 2e-7 and the
  rel-L2 of the deviations f - w <= 2e-6;
* ten steps: rel-L2 of the deviations <= 1e-5;
* workload fields after 100 steps: rel-L2 of every velocity component
  <= 1e-5 with FP32 storage, <= 1e-3 with FP16 deviation storage and
  <= 1e-2 with BF16 (8 significand bits) -- unless the storage format alone
  causes more: tests/golden/storage_floors.txt holds, per case, format and
  component, the error of the FP64 oracle whose state is rounded to the
  format after every step. Where that floor times 1.5 exceeds the target,
  the bound is 1.5 times the floor (gpu_helpers.bound): the FP16 channel's
  transverse components (floors 2.3e-3 and 3.6e-3 at 96 x 48 x 48: a
  perturbation of rms 4e-3 riding on a mean flow of 0.075 whose deviations
  the 11-bit format rounds) and the BF16 channel. Every measured error is
  recorded with its floor, target and bound ($ELBM_PARITY_JSON).
"""
import math

import numpy as np
import pytest

import inputs as I
import oracle as O
from gpu_helpers import (MEASURED, check_fields, dev_rel_l2, lattice_from_field, lib, oracle_init, params_for,
                         random_state, rel_l2)

pytestmark = pytest.mark.gpu

ARBITRARY = {
    "d2_periodic_ragged": dict(n=(300, 77), lam=(2.0, 1.0), T=0.45, omega=1.7),
    "d2_walls_y_force": dict(n=(70, 33), T=1 / 3, omega=1.2, walls=(False, True), force=(1e-4, 0.0)),
    "d2_walls_x_stretched": dict(n=(40, 50), lam=(1.4, 1.0), T=0.4, omega=1.5, walls=(True, False)),
    "d2_control": dict(n=(64, 64), T=0.5, omega=1.8, extended=False),
    "d3_periodic_ragged": dict(n=(70, 37, 21), lam=(1.4, 1.0, 2.0), T=0.4, omega=1.6),
    "d3_channel": dict(n=(48, 24, 24), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, walls=(False, True, False),
                       force=(1e-5, 0.0, 0.0)),
    "d3_walls_xz": dict(n=(20, 30, 18), T=1 / 3, omega=1.0, walls=(True, False, True)),
    "d3_force_periodic": dict(n=(64, 16, 20), T=0.5, omega=1.3, force=(1e-4, -2e-4, 5e-5)),
    "d3_min_periodic": dict(n=(3, 3, 3), T=0.3, omega=1.1),
    "d3_min_walls": dict(n=(5, 2, 4), T=0.5, omega=1.4, walls=(False, True, False)),
    "d3_control_stretched": dict(n=(32, 40, 24), lam=(2.0, 1.0, 1.0), T=1 / 3, omega=1.7, extended=False),
    # an even number of chunks along the marched axis (eight of 4 rows; two of
    # 16 planes): the last chunk marches down from the wall
    "d2_walls_y_even_chunks": dict(n=(70, 32), T=0.4, omega=1.6, walls=(False, True), force=(5e-5, 0.0)),
    "d3_walls_yz_two_chunks": dict(n=(20, 8, 32), T=0.4, omega=1.5, walls=(False, True, True),
                                   force=(1e-4, 0.0, 0.0)),
}


@pytest.mark.parametrize("case", sorted(ARBITRARY))
def test_arbitrary_state_one_and_ten_steps(case):
    E = lib()
    p = O.Params(**ARBITRARY[case])
    f0 = random_state(p, seed=hash(case) % 1000)
    lat = E.Lattice(params_for(p))
    lat.set_populations(f0)
    g0 = lat.populations()  # the GPU's (FP32-rounded) initial state
    assert np.abs(g0 - f0).max() < 1e-8
    lat.step(1)
    g1 = lat.populations()
    o1 = O.step(g0, p)
    assert np.abs(g1 - o1).max() <= 2e-7, case
    assert dev_rel_l2(g1, o1, p) <= 2e-6, case
    lat.step(9)
    g10 = lat.populations()
    o10 = O.run(o1, p, 9)
    assert dev_rel_l2(g10, o10, p) <= 1e-5, case
    # macroscopic fields agree with the oracle's moments of the same state
    rho, u = lat.fields()
    ro, uo = O.velocity(o10, p)
    assert np.abs(rho - ro).max() < 1e-6
    assert np.abs(u - uo).max() < 1e-6


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_init_matches_equilibrium(storage):
    """f'(0) = f^eq(rho, u + u_adv) (Sec. 2.3, eq. 27eq), rounded once to the storage format."""
    p = O.Params(n=(40, 24, 10), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.5)
    g = I.rng(77)
    fld = I.Field(1.0 + 0.01 * g.standard_normal((10, 24, 40)), 0.05 * g.standard_normal((3, 10, 24, 40)),
                  p.n, p.lam)
    uadv = (0.03, -0.01, 0.02)
    lat = lattice_from_field(p, fld, storage, u_adv=uadv)
    fo = oracle_init(p, fld, u_adv=uadv)
    w = O.reference_weights(p, uadv).reshape((-1, 1, 1, 1))
    h = fo - w
    tol = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}[storage]
    err = np.abs(lat.populations() - fo)
    assert (err <= tol * np.abs(h) + 1e-12).all()


def _cfg1(T, storage, via_uadv):
    """GPU and oracle velocities after 100 steps, and the floor-table case name."""
    fld = I.shear_wave_axis((64, 64), U0=0.0 if via_uadv else 0.1, A=0.01)
    uadv = (0.1, 0.0) if via_uadv else None
    p = O.Params(n=(64, 64), T=T, omega=1.8)
    lat = lattice_from_field(p, fld, storage, u_adv=uadv)
    fo = oracle_init(p, fld, u_adv=uadv)
    lat.step(100)
    fo = O.run(fo, p, 100)
    rho, u = lat.fields()
    _, uo = O.velocity(fo, p)
    case = f"cfg1_T{0.5 if T == 0.5 else 0.33}_{'uadv' if via_uadv else 'rest'}"
    return u, uo, case


@pytest.mark.parametrize("T", [1 / 3, 0.5])
@pytest.mark.parametrize("via_uadv", [True, False])
def test_cfg1_shear_wave_fp32(T, via_uadv):
    """D2Q9 64x64, U0 = 0.1, A = 0.01, omega = 1.8, 100 steps: rel-L2 of u_x and
    u_y <= 1e-5, and u_x = U0 (dormant anomaly: exact in exact arithmetic) to 1e-6."""
    u, uo, case = _cfg1(T, "f32", via_uadv)
    check_fields("cfg1", case, "f32", u, uo, (1e-5, 1e-5))
    ux = np.abs(u[0] - 0.1).max()
    MEASURED.append(dict(test="cfg1", case=case, storage="f32", component="ux_dev", measured=float(ux), target=1e-6,
                         bound=1e-6))
    assert ux <= 1e-6


@pytest.mark.parametrize("T", [1 / 3, 0.5])
def test_cfg1_shear_wave_fp16(T):
    u, uo, case = _cfg1(T, "f16", True)
    check_fields("cfg1", case, "f16", u, uo, (1e-3, 1e-3))
    assert np.abs(u[0] - 0.1).max() <= 1e-4


def test_cfg1_shear_wave_bf16():
    u, uo, case = _cfg1(1 / 3, "bf16", True)
    check_fields("cfg1", case, "bf16", u, uo, (1e-2, 1e-2))


_hit_cache = {}


def _hit_oracle():
    if "fo" not in _hit_cache:
        fld = I.hit_field(64, k0=4.0, urms=0.05)
        p = O.Params(n=(64, 64, 64), T=0.5, omega=1.892885)
        fo = O.run(oracle_init(p, fld), p, 100)
        _hit_cache.update(fld=fld, p=p, fo=fo)
    return _hit_cache["fld"], _hit_cache["p"], _hit_cache["fo"]


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16", 1e-3), ("bf16", 1e-2)])
def test_hit_64_cube(storage, tol):
    """D3Q27 decaying turbulence, 64^3, T = 0.5, u_rms = 0.05, 100 steps."""
    fld, p, fo = _hit_oracle()
    lat = lattice_from_field(p, fld, storage)
    lat.step(100)
    _, u = lat.fields()
    _, uo = O.velocity(fo, p)
    check_fields("hit", "hit64", storage, u, uo, (tol, tol, tol))


_chan_cache = {}


def _channel(n=(96, 48, 48)):
    """Sec. 3.5 channel (lambda = (2, 1, 1), walls in y, Re_tau = 180 force) and
    its oracle state after 100 steps."""
    if n not in _chan_cache:
        lam = (2.0, 1.0, 1.0)
        H = 0.5 * n[1] * lam[1]
        omega = 1.976785
        nu = (1 / omega - 0.5) * 0.5
        g = 180.0 ** 2 * nu ** 2 / H ** 3
        fld = I.channel_field(n, lam)
        p = O.Params(n=n, lam=lam, T=0.5, omega=omega, walls=(False, True, False), force=(g, 0.0, 0.0))
        fo = O.run(oracle_init(p, fld), p, 100)
        _chan_cache[n] = (fld, p, fo)
    return _chan_cache[n]


@pytest.mark.parametrize("storage,gate", [("f32", 1e-5), ("f16", 1e-3), ("bf16", 1e-2)])
def test_channel_stretched_walls_force(storage, gate):
    """D3Q27 lam = (2,1,1), bounce-back in y, body force, 96x48x48, 100 steps
    (n_x % 64 != 0: the register-pull kernel for every storage)."""
    fld, p, fo = _channel()
    lat = lattice_from_field(p, fld, storage)
    assert lat.kernel_info()["kernel"] == "register"
    lat.step(100)
    _, u = lat.fields()
    _, uo = O.velocity(fo, p)
    check_fields("channel", "channel96", storage, u, uo, (gate, gate, gate))


@pytest.mark.parametrize("storage,gate", [("f32", 1e-5), ("f16", 1e-3), ("bf16", 1e-2)])
def test_channel_staged_size_100_steps(storage, gate):
    """The same channel at 128 x 48 x 32 (n_x % 64 == 0, n_y % 16 == 0): FP16 and
    BF16 take the LDS-staged kernel with y walls and force, the kernel of the
    full-size channel, for 100 steps against the oracle."""
    fld, p, fo = _channel((128, 48, 32))
    lat = lattice_from_field(p, fld, storage)
    assert lat.kernel_info()["kernel"] == ("register" if storage == "f32" else "staged")
    lat.step(100)
    _, u = lat.fields()
    _, uo = O.velocity(fo, p)
    check_fields("channel_staged", "channel128x48x32", storage, u, uo, (gate, gate, gate))


@pytest.mark.parametrize("storage,gate", [("f32", 1e-5), ("f16", 1e-3)])
def test_double_shear_layer_256(storage, gate):
    """D2Q9 double shear layer (Re = 30000 scaled to L = 256 at constant nu,
    omega = 1.973), 100 steps. FP16's floor on u_y (1.1e-2: the layer's
    transverse perturbation is 5% of the stream speed the deviations carry)
    sets its bound."""
    fld = I.double_shear_layer((256, 256))
    p = O.Params(n=(256, 256), T=0.5, omega=1.973061)
    lat = lattice_from_field(p, fld, storage)
    lat.step(100)
    fo = O.run(oracle_init(p, fld), p, 100)
    _, u = lat.fields()
    _, uo = O.velocity(fo, p)
    check_fields("dsl", "dsl256", storage, u, uo, (gate, gate))


def test_diagnostics_match_oracle():
    """FP64 reductions on the GPU against the oracle's, same state."""
    fld = I.shear_wave_rotated((32, 64), (2.0, 1.0), U0=0.05, a0=1e-3)
    p = O.Params(n=(32, 64), lam=(2.0, 1.0), T=1 / 3, omega=1.8)
    lat = lattice_from_field(p, fld)
    lat.step(37)
    d = lat.diag()
    f = lat.populations()
    do = O.diagnostics(f, p, fld.mode_k, fld.mode_dir)
    assert d["step"] == 37
    assert abs(d["mass"] - do.mass) <= 1e-12 * do.mass
    for a in range(2):
        assert abs(d["mom"][a] - do.mom[a]) <= 1e-10
    assert abs(d["ke"] / do.ke - 1) <= 1e-6
    assert abs(d["enstrophy"] / do.enstrophy - 1) <= 1e-5
    assert abs(d["mode"] - do.mode) <= 1e-6 * abs(do.mode)
    assert abs(d["max_uperp"] / do.max_uperp - 1) <= 1e-6
    assert abs(d["min_rho"] - do.min_rho) <= 1e-7
    assert d["nan_count"] == 0


def test_diagnostics_3d_walls_force():
    fld = I.channel_field((48, 24, 24), (2.0, 1.0, 1.0))
    p = O.Params(n=(48, 24, 24), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, walls=(False, True, False),
                 force=(1e-5, 0.0, 0.0))
    lat = lattice_from_field(p, fld)
    lat.step(5)
    d = lat.diag()
    do = O.diagnostics(lat.populations(), p)
    assert abs(d["mass"] / do.mass - 1) <= 1e-12
    for a in range(3):
        assert abs(d["mom"][a] - do.mom[a]) <= 1e-9
    assert abs(d["ke"] / do.ke - 1) <= 1e-6
    assert abs(d["enstrophy"] / do.enstrophy - 1) <= 1e-5


def _gpu_viscosity(n, lam, T, U0, storage, extended=True, steps=500, every=5, a0=1e-3, rotated=True):
    if rotated:
        fld = I.shear_wave_rotated(n, lam, U0=0.0, a0=a0)
        s2 = math.sqrt(0.5)
        uadv = (U0 * s2, U0 * s2)
    else:
        fld = I.shear_wave_axis(n, U0=0.0, A=a0)
        uadv = (U0, 0.0)
    p = O.Params(n=n, lam=lam, T=T, omega=1.8, extended=extended)
    lat = lattice_from_field(p, fld, storage, u_adv=uadv, diag_every=every, diag_capacity=steps // every)
    lat.step(steps)
    hist = lat.diag_history()
    t = [h["step"] for h in hist]
    amp = [abs(h["mode"]) for h in hist]
    k2 = sum(k * k for k in fld.mode_k)
    return O.fit_decay_rate(t, amp, 50) / k2 / p.nu


@pytest.mark.parametrize("T", [1 / 3, 0.5])
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_viscosity_cfg1_on_gpu(T, storage):
    """Sec. 3.1: fitted decay of the axis-aligned wave gives nu = (1/omega - 1/2) T
    within 1%, over the workload's 500 steps. With FP16 storage the fit is
    only resolved to about 1%: the viscous decrement per step (nu k^2 = 1.8e-4
    of the amplitude at T = 1/3) is 0.37 of FP16's unit roundoff, and the
    fitted rate depends on the exact rounding sequence. The oracle with its
    state rounded to FP16 after every step fits 0.9933 (T = 1/3) and 1.0073
    (T = 1/2) (tests/golden/storage_floors.txt); float32 models of the
    kernel's arithmetic with different operation orders land between 0.997
    and 1.010 at T = 1/3, and the FP32-storage variant of the collision
    (relaxation of the non-equilibrium part) ran at 1.0125 on the GPU. The
    16-bit kernels therefore keep the plain relaxation order."""
    r = _gpu_viscosity((64, 64), (1.0, 1.0), T, 0.1, storage, rotated=False, a0=0.01)
    MEASURED.append(dict(test="viscosity_cfg1", case=f"T={T:.3f} 500 steps", storage=storage,
                         component="nu_fit/nu", measured=float(r - 1), target=1e-2, bound=1e-2))
    assert abs(r - 1) < 1e-2


@pytest.mark.parametrize("U0", [0.0, 0.173])
def test_galilean_invariance_on_gpu(U0):
    r = _gpu_viscosity((64, 64), (1.0, 1.0), 1 / 3, U0, "f32")
    assert abs(r - 1) < 1e-2


def test_isotropy_stretched_on_gpu_and_control():
    """Extended model recovers nu on lam = (2,1); the uncorrected control shows the
    predicted hyper-viscosity 1 + (lam_x^2 - 3T)/(4T) = 3.25."""
    r = _gpu_viscosity((64, 128), (2.0, 1.0), 1 / 3, 0.1, "f32", steps=600)
    assert abs(r - 1) < 1e-2
    rc = _gpu_viscosity((32, 64), (2.0, 1.0), 1 / 3, 0.0, "f32", extended=False)
    assert abs(rc / 3.25 - 1) < 0.1


@pytest.mark.parametrize("T,U0,predicted", [
    (0.5, 0.0, 0.50),      # temperature away from T_L (Sec. 3.1: temperature dependence)
    (1 / 3, 0.173, 0.933),  # advected rotated wave (Sec. 3.1: Galilean invariance lost)
])
def test_uncorrected_control_trends_on_gpu(T, U0, predicted):
    """Negative control on the GPU kernels: the uncorrected product form's
    viscosity follows the linearised limit without the counter term,
    nu_eff / nu = 1 + (c_x + c_y) / (4T), c_a = lambda_a^2 - 3T - 3 U_a^2 (the
    oracle pins the same law), while the extended model stays within 1%."""
    rc = _gpu_viscosity((64, 64), (1.0, 1.0), T, U0, "f32", extended=False)
    assert abs(rc / predicted - 1) < 0.1
    assert abs(rc - 1) > 0.05
    r = _gpu_viscosity((64, 64), (1.0, 1.0), T, U0, "f32")
    assert abs(r - 1) < 1e-2


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_runs_are_deterministic_and_checkpoint_resumes_bitwise(storage):
    E = lib()
    fld = I.hit_field(32, k0=4.0, urms=0.05, seed_offset=9)
    p = O.Params(n=(32, 32, 32), T=0.5, omega=1.7)
    a = lattice_from_field(p, fld, storage)
    b = lattice_from_field(p, fld, storage)
    a.step(40)
    b.step(20)
    ck = b.save()
    c = E.Lattice(params_for(p, storage))
    c.load(ck)
    assert c.step_count == 20
    c.step(20)
    b.step(20)
    fa, fb, fc = a.populations(), b.populations(), c.populations()
    assert np.array_equal(fa, fb)
    assert np.array_equal(fa, fc)


def test_error_paths():
    E = lib()
    import torch

    p = O.Params(n=(64, 64), T=1 / 3, omega=1.5)
    ep = params_for(p)
    small = torch.empty(E.query_bytes(ep) - 4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(E.ElbmError) as ei:
        E.Lattice(ep, buffer=small)
    assert ei.value.status == E.ENOMEM
    big = torch.empty(E.query_bytes(ep) + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(E.ElbmError) as ei:
        E.Lattice(ep, buffer=big[4:])
    assert ei.value.status == E.EINVAL
    lat = E.Lattice(ep)
    f = O.init_state(np.ones((64, 64)), np.zeros((2, 64, 64)), p)
    f[3, 10, 10] = np.nan
    lat.set_populations(f)
    with pytest.raises(E.ElbmError) as ei:
        lat.diag()
    assert ei.value.status == E.EUNSTABLE
    d = lat.diag(check=False)
    assert d["nan_count"] == 1
    other = E.Lattice(params_for(O.Params(n=(64, 32), T=1 / 3, omega=1.5)))
    with pytest.raises(E.ElbmError):
        other.load(lat.save())


@pytest.mark.parametrize("chunk", [1, 2, 3])
def test_short_chunks_match_oracle(chunk, monkeypatch):
    """Tiles of 1, 2 or 3 planes (forced): the prologue, the ring planes at
    both chunk ends, the downward march of odd chunks and the skipped fetches
    of unused planes all act on nearly every plane. Walls on z put chunk ends
    next to the wall ghosts; one and ten steps from an arbitrary state against
    the oracle, as for the other lattices."""
    monkeypatch.setenv("ELBM_CHUNK", str(chunk))
    E = lib()
    p = O.Params(n=(20, 16, 9), lam=(1.0, 1.5, 1.0), T=0.45, omega=1.5, walls=(False, False, True),
                 force=(5e-5, 0.0, -3e-5))
    f0 = random_state(p, seed=91 + chunk)
    lat = E.Lattice(params_for(p))
    assert lat.kernel_info()["tile"][2] == chunk
    lat.set_populations(f0)
    g0 = lat.populations()
    lat.step(1)
    o1 = O.step(g0, p)
    assert np.abs(lat.populations() - o1).max() <= 2e-7
    lat.step(9)
    assert dev_rel_l2(lat.populations(), O.run(o1, p, 9), p) <= 1e-5


@pytest.mark.parametrize("D,storage,n", [(2, "f32", (64, 8)), (3, "f32", (40, 8, 6))])
def test_poiseuille_exact_at_magic_relaxation_on_gpu(D, storage, n):
    """The GPU's walls, force and reported velocity (j + rho g/2)/rho against the
    Navier-Stokes parabola u = g/(2 nu) y (2H - y), which LBGK with halfway
    bounce-back reproduces without wall slip at tau = 1/2 + sqrt(3)/4 (the
    oracle meets it to 1e-10). Without the half-force shift the profile would
    be off by g/2 everywhere: 0.9% of the centreline value at 8 rows. FP32
    storage, within 1e-5 of the centreline value. (FP16 storage cannot resolve
    this steady state: at 64 x 16 x 4 the staged kernel's profile sits 3e-3
    off, more than the g/2 shift, from rounding the small deviations of a
    low-speed flow to 11 bits; the staged kernel's walls and force are checked
    against the oracle over 100 steps instead.)"""
    tau = 0.5 + math.sqrt(3.0) / 4.0
    g = 1e-5
    ny = n[1]
    walls = (False, True) + ((False,) if D == 3 else ())
    p = O.Params(n=n, T=1.0 / 3.0, omega=1.0 / tau, walls=walls, force=(g,) + (0.0,) * (D - 1))
    grid = tuple(reversed(n))
    y = np.arange(ny) + 0.5
    exact = g / (2.0 * p.nu) * y * (ny - y)
    u0 = np.zeros((D,) + grid)
    shape = [1] * D
    shape[D - 2] = ny
    u0[0] = exact.reshape(shape)
    fld = I.Field(np.ones(grid), u0, n, (1.0,) * D)
    lat = lattice_from_field(p, fld, storage)
    lat.step(1500)
    _, u = lat.fields()
    ux = np.moveaxis(u[0], D - 2, 0).reshape(ny, -1)
    err = np.abs(ux - exact[:, None]).max() / exact.max()
    tol = 1e-5
    MEASURED.append(dict(test="poiseuille_magic_tau", case=f"D{D} {n}", storage=storage, component="u0",
                         measured=float(err), target=tol, bound=tol))
    assert err <= tol
    assert 0.5 * g / exact.max() > 2 * tol  # the unshifted velocity would fail


@pytest.mark.parametrize("walls", [False, True])
def test_enstrophy_3d_closed_form_on_gpu(walls):
    """GPU enstrophy of a state initialised with a velocity field whose
    central-difference curl is known node by node (all three components
    nonzero, unequal spacings; with walls, the no-slip ghost on y): against the
    closed form directly, not only against the oracle."""
    import importlib
    import sys as _sys

    _sys.path.insert(0, __file__.rsplit("/", 1)[0])
    tod = importlib.import_module("test_oracle_dynamics")
    p, u, exact = tod._vorticity_closed_form_case(walls)
    fld = I.Field(np.ones(u.shape[1:]), u, p.n, p.lam)
    lat = lattice_from_field(p, fld, "f32")
    d = lat.diag()
    e = abs(d["enstrophy"] / exact.mean() - 1)
    MEASURED.append(dict(test="enstrophy_closed_form", case=f"walls={walls}", storage="f32", component="enstrophy",
                         measured=float(e), target=1e-5, bound=1e-5))
    assert e <= 1e-5


def test_empty_and_zero_step_requests():
    """Degenerate requests: zero steps leave a lattice bitwise unchanged (step
    count 0), negative steps are rejected, an empty batch and a batch whose
    step counts are all zero are no-ops (also through the allocation-free
    entry point), and zero face steps change nothing."""
    E = lib()
    p = O.Params(n=(32, 16, 8), T=0.5, omega=1.6)
    lat = E.Lattice(params_for(p))
    lat.set_populations(random_state(p, seed=31))
    f0 = lat.populations()
    lat.step(0)
    assert lat.step_count == 0
    assert np.array_equal(lat.populations(), f0)
    with pytest.raises(E.ElbmError) as ei:
        lat.step(-1)
    assert ei.value.status == E.EINVAL
    b = E.Batch(4)
    b.run([], [])
    b.run([lat], [0])
    E.batch_run_static([], [])
    E.batch_run_static([lat], [0])
    assert lat.step_count == 0
    assert np.array_equal(lat.populations(), f0)
    b.close()
    lat.close()
    lat2 = E.Lattice(E.make_params((8, 10), T=1 / 3, omega=1.2))
    lat2.set_populations(random_state(O.Params(n=(8, 10), T=1 / 3, omega=1.2), seed=32))
    faces = E.Faces(lat2, ["periodic", "periodic", "wall", "wall"])
    g0 = lat2.populations()
    faces.step(0)
    assert np.array_equal(lat2.populations(), g0)
    faces.close()
    lat2.close()
