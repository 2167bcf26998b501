"""Host-side checks of the channel statistics driver (Sec. 3.5): its
constants follow the relations it states, and its wall-unit reduction returns
what a profile of known form must give."""
import math

import numpy as np
import pytest

from paper_2101_04550_amd import channel_study as CS


@pytest.mark.parametrize("lattice", ["stretched", "cubic", "bench"])
def test_constants(lattice):
    c = CS.setup(lattice)
    H = c["H"]
    # the log-law estimate of u_tau from the centre-line velocity u0 (Sec. 3.5)
    assert c["u0"] == pytest.approx(c["u_tau"] * (math.log(c["re_tau"]) / 0.41 + 5.5), rel=1e-14)
    assert c["re_tau"] == pytest.approx(c["u_tau"] * H / c["nu"], rel=1e-14)
    # BGK viscosity (Sec. 2.1) and the force that balances the wall friction
    assert c["nu"] == pytest.approx((1 / c["omega"] - 0.5) * c["T"], rel=1e-12)
    assert c["g"] * H == pytest.approx(c["u_tau"] ** 2, rel=1e-12)
    assert c["n"][1] == 2 * H
    if lattice != "bench":
        # 5.6 H x 2H x 2H (Sec. 3.5), to the nearest node on the cubic lattice
        assert abs(c["n"][0] * c["lam"][0] - 5.6 * H) <= 0.5
    # rest weights stay positive on every axis
    assert all(1 - c["T"] / lam ** 2 > 0 for lam in c["lam"])


def test_planar_stats():
    g = np.random.default_rng(7)
    nz, ny, nx = 6, 5, 8
    base = np.arange(ny, dtype=np.float64)
    u = np.zeros((3, nz, ny, nx))
    u[0] = base[None, :, None] + 0.3 * g.standard_normal((nz, ny, nx))
    mean, rms = CS.planar_stats(u)
    for y in range(ny):
        assert mean[0, y] == pytest.approx(u[0, :, y, :].mean(), abs=1e-14)
        assert rms[0, y] == pytest.approx(u[0, :, y, :].std(), abs=1e-14)
    assert np.all(rms[1:] == 0)


def test_wall_units_of_a_law_of_the_wall_profile():
    """A profile that is the viscous sublayer at the first row and the log law
    (kappa = 0.41, B = 5.5) from y+ = 30 on gives zero log-law deviation and
    the nominal friction velocity from the wall gradient."""
    c = CS.setup("cubic")
    H, nu, ut = c["H"], c["nu"], math.sqrt(c["g"] * c["H"])
    ny = 2 * H
    y = (np.arange(ny) + 0.5)
    yd = np.minimum(y, 2 * H - y)  # distance from the nearest wall
    yp = yd * ut / nu
    up = np.where(yp < 11.0, yp, np.log(yp) / 0.41 + 5.5)
    prof = np.stack([up * ut, 0.1 * ut * np.ones(ny), 0.5 * ut * np.ones(ny), 0.2 * ut * np.ones(ny)])
    r = CS.wall_units(prof, c, y)
    assert r["u_tau_wall"] == pytest.approx(ut, rel=1e-12)
    assert r["re_tau_measured"] == pytest.approx(c["re_tau"], rel=1e-12)
    assert r["log_law_deviation_rms"] < 1e-12
    lo, hi = r["log_law_range"]
    assert lo > 30 and hi < 0.3 * H * ut / nu
    assert r["turbulent"]  # v_rms+ = 0.5 > 0.2
    assert r["y_plus"][0] == pytest.approx(0.5 * ut / nu, rel=1e-12)
