"""Stored values under tests/golden/, each file citing the passage it comes from:
the oracle's equilibrium at rest against the textbook weights, and the channel
workload's constants against the values the paper prints (Sec. 3.5)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("D", [2, 3])
def test_rest_weights_at_lattice_temperature(D):
    """Equilibrium at u = 0, lambda = 1, T = 1/3 equals the stored weights exactly
    (to FP64 rounding), for every direction of the lattice."""
    Q = 3 ** D
    table = {int(r[1]): Fraction(int(r[2]), int(r[3])) for r in _rows("rest_weights_TL.txt") if int(r[0]) == Q}
    assert sorted(table) == list(range(D + 1))
    assert sum(table[k] * math.comb(D, k) * 2 ** k for k in table) == 1  # the stored weights sum to one
    p = O.Params(n=(1,) * D, T=1.0 / 3.0)
    w = O.equilibrium(np.array(1.0), np.zeros(D), p.T, p.lam, p.c)
    for i, ci in enumerate(p.c):
        assert abs(w[i] - float(table[int(np.abs(ci).sum())])) < 1e-15


def test_channel_constants():
    """u_tau from the log-law estimate, nu, omega (eq. nu) and g = Re_tau^2 nu^2 / H^3
    for H = 96, T = 0.5; the benchmark's channel workload uses the same values."""
    vals = {r[0]: (float(r[1]), float(r[2])) for r in _rows("channel_re180.txt")}
    re_tau, kappa, u0, H, T = (vals[k][0] for k in ("re_tau", "kappa", "u0", "H", "T"))
    u_tau = u0 / (math.log(re_tau) / kappa + 5.5)
    nu = u_tau * H / re_tau
    omega = 1.0 / (nu / T + 0.5)
    g = re_tau ** 2 * nu ** 2 / H ** 3
    for name, v in (("u_tau", u_tau), ("nu", nu), ("omega", omega), ("g", g)):
        want, rtol = vals[name]
        assert abs(v - want) <= rtol * abs(want), (name, v, want)
    # g is also u_tau^2 / H (the force balance of the wall shear stress)
    assert abs(g - u_tau ** 2 / H) <= 1e-12 * g

    import bench
    assert bench.CHANNEL_H == H and bench.CHANNEL_RE_TAU == re_tau and bench.CHANNEL_T == T
    assert bench.CHANNEL_N[1] == 2 * H
    assert abs(bench.CHANNEL_OMEGA - vals["omega"][0]) <= vals["omega"][1] * vals["omega"][0]
    assert abs(bench.channel_force() - vals["g"][0]) <= vals["g"][1] * vals["g"][0]
