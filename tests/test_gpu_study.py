"""GPU studies of stretched lattices against regular ones: the periodic double
shear layer of Sec. 3.3, and (further down) the laminar flat plate of Sec. 3.4
with Grad's-approximation walls, the temperature independence of decaying
turbulence, the channel driver, and (at the end) two flows whose parameters
LBGK cannot run and the multi-relaxation-time collision can.

Double shear layer: on the cubic lattice and on the lattice stretched to
lambda = (2, 1) with half the x nodes.

Setup as in the paper: L = 1024, u0 = 0.1, kappa = 80, delta = 0.05,
Re = u0 L / nu = 1e4, T = 1/3, run to t* = t u0 / L = 1 (10240 steps), FP32
storage. Kinetic energy and enstrophy (FP64 diagnostics: node averages of
|u|^2 / 2 and |curl u|^2 with spacings lambda_a) are compared at t* = 0, 0.1,
..., 1.

The paper shows both lattices giving the same flow; with the extended
equilibrium the stretched lattice should reproduce the cubic one up to the
truncation error of its coarser x spacing, while the uncorrected product form
on the stretched lattice carries the anomaly's extra viscosity (Sec. 3.1) and
loses energy and enstrophy faster.

Measured on one MI355X: stretched vs cubic |dKE/KE| <= 2.4e-5 and
|dZ/Z| <= 2.6e-3 over the run; the uncorrected stretched lattice ends 0.97%
low in KE and 13.2% low in enstrophy. The bounds below sit about four times
above the measured agreement and well inside the control's gap, so a broken
correction on stretched lattices (sign, spacing, prefactor) fails them.
This is a property of the method at this resolution, not a parity bound.
"""
import math

import numpy as np
import pytest

import inputs as I
from gpu_helpers import MEASURED, lib

pytestmark = pytest.mark.gpu

L, U, T = 1024, 0.1, 1.0 / 3.0
RE = 1.0e4
NU = U * L / RE
OMEGA = 1.0 / (NU / T + 0.5)
STEPS = int(round(L / U))
RECORDS = 10


def _history(n, lam, extended):
    E = lib()
    fld = I.double_shear_layer(n, lam=lam, U=U)
    lat = E.Lattice(E.make_params(n, lam=lam, T=T, omega=OMEGA, storage="f32", extended=extended))
    lat.init(fld.rho, fld.u)
    ke, z = [], []
    for k in range(RECORDS + 1):
        d = lat.diag()
        ke.append(d["ke"])
        z.append(d["enstrophy"])
        if k < RECORDS:
            lat.step(STEPS // RECORDS)
    lat.close()
    return np.array(ke), np.array(z)


@pytest.fixture(scope="module")
def runs():
    return {
        "cubic": _history((L, L), (1.0, 1.0), True),
        "stretched": _history((L // 2, L), (2.0, 1.0), True),
        "control": _history((L // 2, L), (2.0, 1.0), False),
    }


def test_stretched_lattice_reproduces_cubic(runs):
    kc, zc = runs["cubic"]
    ks, zs = runs["stretched"]
    assert kc[-1] < kc[0] and zc[-1] < zc[0]  # viscous decay over the run
    assert np.abs(ks / kc - 1).max() <= 1e-4
    assert np.abs(zs / zc - 1).max() <= 1e-2


def test_uncorrected_stretched_lattice_is_more_dissipative(runs):
    kc, zc = runs["cubic"]
    ks, zs = runs["stretched"]
    kn, zn = runs["control"]
    # the control loses enstrophy faster than the cubic reference ...
    assert zn[-1] < 0.95 * zc[-1]
    assert kn[-1] < kc[-1] * (1 - 3e-3)
    # ... by far more than the corrected stretched lattice deviates
    assert abs(zn[-1] / zc[-1] - 1) > 10 * abs(zs[-1] / zc[-1] - 1)


@pytest.fixture(scope="module")
def plates():
    """The Sec. 3.4 flat plate (Re = 4000, Ma = 0.1, T = 1/3) on the regular
    and the lambda_x = 2 lattice at 4x the printed resolution (800 x 800 in
    units of the y spacing: omega = 1.901; at the printed 200 x 200 the
    lambda_x = 2 lattice is unstable at this viscosity, see
    tests/test_oracle_dynamics.py), 240 000 steps, fields averaged over the
    second half."""
    from paper_2101_04550_amd import flat_plate as FP

    out = {}
    for lam_x in (1.0, 2.0):
        res, _ = FP.run(lam_x, 240000, check_every=4000, scale=4)
        out[lam_x] = res
    return out


def test_flat_plate_matches_blasius(plates):
    """Both lattices reproduce Blasius' profile (with the local edge velocity)
    to 0.03 of it and C_f = 0.664/sqrt(Re_x) to 5% rms over 20-90% of the
    plate (measured: profile 0.010 / 0.018, C_f 2.1% / 3.3% rms, regular /
    stretched; C_f runs above Blasius as the stream accelerates by 3-4%
    along the plate)."""
    for lam_x, r in plates.items():
        assert r["profile_edge_max_dev"] < 0.03, (lam_x, r["profile_edge_max_dev"])
        assert r["cf_edge_rms_rel_dev"] < 0.05, (lam_x, r["cf_edge_rms_rel_dev"])
        assert r["last_vs_mean"] < 0.05


def test_stretched_plate_reproduces_regular(plates):
    """Half the nodes (lambda_x = 2) give the regular lattice's profile to
    0.015 of the edge velocity and its skin friction to 5% (measured 0.0077
    and 3.2%, the largest near the outlet)."""
    a, b = plates[2.0], plates[1.0]
    ua = np.array(a["profile_edge_u"])
    ub = np.interp(a["profile_edge_eta"], b["profile_edge_eta"], b["profile_edge_u"])
    assert np.abs(ua - ub).max() < 0.015
    ca = np.array(a["cf_edge"])
    cb = np.interp(a["cf_x"], b["cf_x"], b["cf_edge"])
    assert np.abs(ca / cb - 1).max() < 0.05


def _hit_run(T, N=256, k0=8.0, ma_t=0.1, re_lambda=72.0, tstar_end=3.0, every=None, rates=None):
    """Decaying turbulence of Sec. 3.2 at temperature T: Ma_t = sqrt(<u.u>)/sqrt(T)
    and Re_lambda fixed, kappa_0 = 2 pi k0 / L = 16 pi / L. Returns t* and the
    FP64 records (KE, enstrophy) of the sample steps."""
    E = lib()
    urms = ma_t * math.sqrt(T) / math.sqrt(3.0)
    fld = I.hit_field(N, k0=k0, urms=urms, seed_offset=5)
    lam_T = 2.0 / (2.0 * math.pi * k0 / N)  # Taylor microscale of the k^4 exp(-2 (k/k0)^2) spectrum (R16)
    nu = urms * lam_T / re_lambda
    omega = 1.0 / (nu / T + 0.5)
    L_I = math.sqrt(2.0 * math.pi) / (2.0 * math.pi * k0 / N)
    tau = L_I / urms
    steps = int(round(tstar_end * tau))
    every = every or max(1, int(round(0.05 * tau)))
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    lat = E.Lattice(E.make_params((N, N, N), T=T, omega=omega, diag_every=every,
                                  diag_capacity=steps // every + 1, **kw))
    lat.init(fld.rho, fld.u)
    lat.step(steps)
    hist = lat.diag_history()
    lat.close()
    t = np.array([h["step"] / tau for h in hist])
    ke = np.array([h["ke"] for h in hist])
    Z = np.array([h["enstrophy"] for h in hist])
    # u_rms^2 = 2 KE / 3; isotropy: <(d_x u_x)^2> = <|curl u|^2> / 15
    u2 = 2.0 * ke / 3.0
    re_l = u2 * np.sqrt(15.0 / Z) / nu
    ke0 = 1.5 * urms ** 2
    return dict(t=t, ke=ke / ke0, re_lambda=re_l, steps=steps, omega=omega)


@pytest.fixture(scope="module")
def hit_temperatures():
    return {T: _hit_run(T) for T in (1.0 / 3.0, 0.55)}


def test_hit_temperature_independence(hit_temperatures):
    """Sec. 3.2: decaying turbulence at Ma_t = 0.1, Re_lambda = 72 gives the
    same kinetic-energy and Re_lambda histories in eddy-turnover time at
    T = 1/3 and T = 0.55, the higher temperature in sqrt(0.55 / (1/3)) = 1.28x
    fewer steps."""
    a, b = hit_temperatures[1.0 / 3.0], hit_temperatures[0.55]
    assert a["steps"] / b["steps"] == pytest.approx(math.sqrt(0.55 * 3.0), rel=5e-3)
    t = np.linspace(0.2, 2.8, 27)
    ka, kb = np.interp(t, a["t"], a["ke"]), np.interp(t, b["t"], b["ke"])
    ra, rb = np.interp(t, a["t"], a["re_lambda"]), np.interp(t, b["t"], b["re_lambda"])
    dk, dr = float(np.abs(ka / kb - 1).max()), float(np.abs(ra / rb - 1).max())
    MEASURED.append(dict(test="hit_temperature", case="256^3 Ma_t 0.1 Re_lambda 72, t* 0.2-2.8", storage="f32",
                         component="KE / Re_lambda max rel diff", measured=[dk, dr, float(ka[-1]), float(ra[0])],
                         target=None, bound=[0.02, 0.03]))
    assert ka[-1] < 0.6  # the turbulence decays over the run
    assert dk < 0.02, dk
    assert dr < 0.03, dr


def test_hit_with_the_mrt_collision(hit_temperatures):
    """The same decaying turbulence (T = 0.55) with the D3Q27 MRT collision
    (omega_bulk = 1.2, omega_ghost = 1.0; the shear rate omega unchanged):
    kinetic-energy history within 1% and Re_lambda within 2% of LBGK's
    (measured on one MI355X: 0.26% and 0.81%) -- the extra rates act on the
    nearly incompressible flow's acoustics and ghosts, not on its viscous
    decay."""
    a = hit_temperatures[0.55]
    b = _hit_run(0.55, rates=(1.2, 1.0))
    t = np.linspace(0.2, 2.8, 27)
    ka, kb = np.interp(t, a["t"], a["ke"]), np.interp(t, b["t"], b["ke"])
    ra, rb = np.interp(t, a["t"], a["re_lambda"]), np.interp(t, b["t"], b["re_lambda"])
    dk, dr = float(np.abs(ka / kb - 1).max()), float(np.abs(ra / rb - 1).max())
    MEASURED.append(dict(test="hit_mrt", case="256^3 T 0.55 Ma_t 0.1 Re_lambda 72, t* 0.2-2.8", storage="f32",
                         component="KE / Re_lambda max rel diff vs LBGK", measured=[dk, dr], target=None,
                         bound=[0.01, 0.02]))
    assert dk < 0.01, dk
    assert dr < 0.02, dr


@pytest.mark.parametrize("walls", ["bounce-back", "grad"])
def test_channel_study_driver_runs(tmp_path, walls):
    """The Sec. 3.5 statistics driver end to end on its stretched lattice
    (384 x 192 x 192, lambda_x = 1.4, T = 0.55) for a few hundred steps, with
    halfway bounce-back or Grad walls: the run, the planar statistics and the
    wall-unit reduction produce finite profiles; the near-wall u+ of the
    seeded laminar-plus-noise start lies below the log law's centre-line
    value."""
    from paper_2101_04550_amd import channel_study as CS

    res = CS.run("stretched", tstar=0.02, stats_from=0.0, sample=100, storage="f32",
                 out=str(tmp_path / "channel.json"), walls=walls)
    assert res["samples_averaged"] >= 2
    up = np.array(res["u_plus"])
    assert np.isfinite(up).all() and up.size == 96
    assert 0 < up[0] < up[-1] < 30
    assert np.isfinite(res["re_tau_measured"])


# ---- the multi-relaxation-time collision on a shear layer LBGK cannot run ----
#
# The double shear layer at Re = 3e4 (u0 = 0.1) on 256^2 cubic nodes, T = 1/2
# (omega = 1.9932): the step linearised about the layer's stream has modes
# growing ~2% per step with LBGK and none with the MRT collision at
# omega_bulk = 1, omega_ghost = 1.5 (tests/test_oracle_mrt.py). Measured on
# one MI355X: LBGK diverges before t* = 0.4 (at 128^2-1024^2 before
# t* = 0.2-0.5); MRT runs to t* = 1 and ends within 0.2% (kinetic energy) and
# 1.7% (enstrophy) of LBGK at the paper's T = 1/3, where LBGK is stable.

DSL_N, DSL_RE = 256, 3.0e4


def _dsl_run(T, rates):
    E = lib()
    n = (DSL_N, DSL_N)
    omega = 1.0 / (U * DSL_N / DSL_RE / T + 0.5)
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    fld = I.double_shear_layer(n, U=U)
    lat = E.Lattice(E.make_params(n, T=T, omega=omega, **kw))
    lat.init(fld.rho, fld.u)
    steps = int(round(DSL_N / U))
    out = None
    for k in range(10):
        lat.step(steps // 10)
        d = lat.diag(check=False)
        if d["nan_count"] > 0 or not math.isfinite(d["ke"]):
            out = {"diverged_at": (k + 1) / 10}
            break
    else:
        out = {"ke": d["ke"], "enstrophy": d["enstrophy"]}
    lat.close()
    return out


def test_mrt_runs_the_shear_layer_that_lbgk_cannot():
    lbgk_hot = _dsl_run(0.5, None)
    mrt_hot = _dsl_run(0.5, (1.0, 1.5))
    lbgk_cold = _dsl_run(1.0 / 3.0, None)
    MEASURED.append(dict(test="dsl_mrt_256", lbgk_t05=lbgk_hot, mrt_t05=mrt_hot, lbgk_t033=lbgk_cold))
    assert "diverged_at" in lbgk_hot
    assert "ke" in mrt_hot and "ke" in lbgk_cold
    assert abs(mrt_hot["ke"] / lbgk_cold["ke"] - 1.0) < 5e-3
    assert abs(mrt_hot["enstrophy"] / lbgk_cold["enstrophy"] - 1.0) < 5e-2


def _bench_channel_run(rates, steps=6000, every=2000):
    """The benchmark channel (384 x 192 x 192, lambda = (2, 1, 1), T = 1/2,
    Re_tau = 180 force) from the seeded laminar-plus-noise start: the step at
    which the velocity first turns non-finite (sampled every `every` steps),
    or None, and the final bulk velocity."""
    from paper_2101_04550_amd import channel_study as CS

    E = lib()
    c = CS.setup("bench")
    fld = I.channel_field(c["n"], c["lam"], u0=c["u0"], seed_offset=3)
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    lat = E.Lattice(E.make_params(c["n"], lam=c["lam"], T=c["T"], omega=c["omega"], walls=(False, True, False),
                                  force=(c["g"], 0.0, 0.0), **kw))
    lat.init(fld.rho, fld.u)
    bad, bulk = None, None
    for done in range(every, steps + 1, every):
        lat.step(every)
        _, u = lat.fields()
        if not np.isfinite(u).all():
            bad = done
            break
        bulk = float(u[0].mean())
    lat.close()
    return bad, bulk


def test_benchmark_channel_runs_with_mrt_not_lbgk():
    """The benchmark channel's parameters (omega = 1.9768 on lambda = (2, 1,
    1) at T = 1/2) let LBGK diverge within a few thousand steps; the MRT
    collision with omega_bulk = omega_ghost = 1.5 runs them (6000 steps
    here; to t* = 30 with channel_study.py, turbulent, Re_tau 176.6 from the
    wall gradient) with the bulk velocity near the seed's. Measured: LBGK
    non-finite by step 3000."""
    bad_lbgk, _ = _bench_channel_run(None)
    bad_mrt, bulk = _bench_channel_run((1.5, 1.5))
    MEASURED.append(dict(test="bench_channel_mrt", lbgk_nonfinite_at=bad_lbgk, mrt_nonfinite_at=bad_mrt,
                         mrt_bulk=bulk))
    assert bad_lbgk is not None
    assert bad_mrt is None
    assert 0.06 < bulk < 0.09
