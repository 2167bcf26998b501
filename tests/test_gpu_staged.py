"""The LDS-staged D3Q27 step kernel (16-bit storage, n_x a multiple of 64,
x and z periodic, y bounce-back with n_y a multiple of 16 or periodic with
n_y > 8: the last tile row may then overhang the axis).

It pulls the same stored values as the register-pull kernel and runs the same
per-node arithmetic, so the two agree to the last bit but for the rounding of
a final multiply-add (see the test); against the FP64 oracle one
step from an arbitrary state is held to the storage rounding: half an ulp of
the largest stored deviation, at most its unit roundoff times it (2^-11 for
FP16, 2^-8 for BF16), plus the FP32 arithmetic bound of the single-precision
tests.
"""
import os

import numpy as np
import pytest

import oracle as O
from gpu_helpers import dev_rel_l2, lib, params_for, random_state

pytestmark = pytest.mark.gpu

CASES = {
    "cube64": dict(n=(64, 64, 64), T=0.5, omega=1.89),
    "flat_force_stretched": dict(n=(128, 16, 12), lam=(2.0, 1.0, 1.0), T=0.4, omega=1.6,
                                 force=(1e-4, -5e-5, 2e-5)),
    "three_planes": dict(n=(64, 16, 3), T=1 / 3, omega=1.2),
    # bounce-back walls on y: two tile rows (one per wall), force (the channel
    # form); one tile row touching both walls
    "channel_walls_force": dict(n=(128, 32, 12), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9,
                                walls=(False, True, False), force=(1e-5, 0.0, 0.0)),
    "walls_one_row": dict(n=(64, 16, 8), T=1 / 3, omega=1.4, walls=(False, True, False)),
    # periodic y with n_y % 16 != 0: the last tile row overhangs the axis (8 of
    # 16 rows beyond it; stretched, force on two axes)
    "overhang_force": dict(n=(64, 24, 6), lam=(1.0, 1.4, 1.0), T=0.45, omega=1.7, force=(2e-5, 1e-5, 0.0)),
    # the shortest axis the kernel takes: n_y = 9, one tile row of 9 live
    # rows whose 18 staged rows span the axis twice
    "overhang_short": dict(n=(128, 9, 4), T=0.5, omega=1.5),
    # several tile rows and chunks, the last one overhanging by 8 rows
    "overhang_stretched": dict(n=(64, 40, 9), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9),
}
# not eligible (n_x % 64 != 0; periodic y with n_y <= 8; walls on y with
# n_y % 16 != 0; walls on x): take the register-pull kernel
RAGGED = dict(n=(96, 16, 5), T=0.5, omega=1.5)
SHORT_Y = dict(n=(64, 8, 5), T=0.5, omega=1.5)
WALLS_RAGGED = dict(n=(64, 24, 5), T=0.5, omega=1.5, walls=(False, True, False))
WALLS_X = dict(n=(64, 16, 6), T=0.5, omega=1.5, walls=(True, False, False))
EPS = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def lattice(p, storage, staged, f0):
    E = lib()
    old = os.environ.get("ELBM_STAGED")
    os.environ["ELBM_STAGED"] = "1" if staged else "0"
    try:
        lat = E.Lattice(params_for(p, storage))
    finally:
        if old is None:
            del os.environ["ELBM_STAGED"]
        else:
            os.environ["ELBM_STAGED"] = old
    lat.set_populations(f0)
    return lat


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_staged_equals_register_pull(case, storage):
    """Same stored values in, same arithmetic: after one step the stored bits
    agree except where the compiler rounds a population's final multiply-add
    to 16 bits once in one kernel and through FP32 in the other (one unit of
    the last place, rarely); after seven steps the states agree to that
    rounding level."""
    p = O.Params(**CASES[case])
    f0 = random_state(p, seed=7)
    a = lattice(p, storage, True, f0)
    b = lattice(p, storage, False, f0)
    assert a.kernel_info()["kernel"] == "staged"
    assert a.kernel_info()["block_threads"] == 1024
    assert b.kernel_info()["kernel"] == "register"
    a.step(1)
    b.step(1)
    d = np.abs(a.save().view(np.uint16).astype(np.int64) - b.save().view(np.uint16).astype(np.int64))
    assert d.max() <= 1, (case, storage)
    assert (d > 0).mean() <= 1e-4, (case, storage)
    a.step(6)
    b.step(6)
    ga, gb = a.populations(), b.populations()
    w = O.reference_weights(p).reshape((-1,) + (1,) * p.D)
    hmax = float(np.abs(gb - w).max())
    assert np.abs(ga - gb).max() <= 2 * EPS[storage] * hmax, (case, storage)
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_staged_one_step_against_oracle(case, storage):
    p = O.Params(**CASES[case])
    f0 = random_state(p, seed=11)
    lat = lattice(p, storage, True, f0)
    g0 = lat.populations()  # the stored (rounded) initial state
    lat.step(1)
    g1 = lat.populations()
    o1 = O.step(g0, p)
    w = O.reference_weights(p).reshape((-1,) + (1,) * p.D)
    hmax = float(np.abs(o1 - w).max())
    assert np.abs(g1 - o1).max() <= EPS[storage] * hmax * 1.05 + 2e-7, case
    assert dev_rel_l2(g1, o1, p) <= EPS[storage], case
    lat.close()


def test_kernel_choice():
    for case in (RAGGED, SHORT_Y, WALLS_RAGGED, WALLS_X):
        p = O.Params(**case)
        lat = lattice(p, "f16", True, random_state(p, seed=3))
        assert lat.kernel_info()["kernel"] == "register"
        lat.close()
    p = O.Params(**CASES["cube64"])
    lat = lattice(p, "f32", True, random_state(p, seed=3))
    info = lat.kernel_info()
    assert info["kernel"] == "register" and info["tile"][:2] == (64, 8) and info["tiles"] >= 1
    lat.close()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_walls_equal_mirrored_periodic_lattice(storage):
    """The wall path of the GPU kernels against their own periodic path: a
    purely wall-normal flow between y walls (16 rows) evolves like the
    periodic flow on 32 rows that continues it mirrored, u_y reversed (the
    equivalence the oracle pins for its wall treatment). FP32 runs the
    register-pull kernel, FP16 / BF16 the LDS-staged one on both lattices.
    The two lattices add the same values in different orders (the mirrored
    nodes hold permuted populations), so they agree to rounding: 2e-6 in
    FP32 after 20 steps, four units of the last stored place in 16 bits."""
    E = lib()
    H, T, omega = 16, 0.45, 1.3
    g = np.random.default_rng(7)
    rho_y = 1.0 + 0.05 * g.standard_normal(H)
    uy_y = 0.04 * g.standard_normal(H)

    def make(n, walls, rho1, uy1):
        p = O.Params(n=n, T=T, omega=omega, walls=walls)
        shape = (n[2], n[1], n[0])
        rho = np.broadcast_to(rho1.reshape(1, -1, 1), shape).copy()
        u = np.zeros((3,) + shape)
        u[1] = np.broadcast_to(uy1.reshape(1, -1, 1), shape)
        lat = E.Lattice(params_for(p, storage))
        lat.set_populations(O.init_state(rho, u, p))
        return lat

    lw = make((64, H, 8), (False, True, False), rho_y, uy_y)
    lp = make((64, 2 * H, 8), (False, False, False), np.concatenate([rho_y, rho_y[::-1]]),
              np.concatenate([uy_y, -uy_y[::-1]]))
    want = "register" if storage == "f32" else "staged"
    assert lw.kernel_info()["kernel"] == want and lp.kernel_info()["kernel"] == want
    lw.step(20)
    lp.step(20)
    fw = lw.populations()
    fp = lp.populations()[:, :, :H, :]
    w = O.reference_weights(O.Params(n=(64, H, 8), T=T, omega=omega)).reshape((-1, 1, 1, 1))
    err = np.abs(fw - fp).max()
    if storage == "f32":
        assert err <= 2e-6
    else:
        hmax = np.abs(fw - w).max()
        assert err <= 4 * EPS[storage] * hmax
    # the flow is still there
    _, u = lw.fields()
    assert np.abs(u[1]).max() > 1e-3


@pytest.mark.parametrize("chunk", [1, 2, 3])
def test_staged_short_chunks_equal_register_pull(chunk, monkeypatch):
    """The staged kernel with tiles of 1, 2 or 3 planes (forced): stage loads
    skipped on a tile's last plane, downward march of odd chunks, y walls;
    against the register-pull kernel on the same lattice after five steps, to
    the last-bit rounding bound of the equality test above."""
    monkeypatch.setenv("ELBM_CHUNK", str(chunk))
    p = O.Params(n=(64, 16, 9), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.7, walls=(False, True, False),
                 force=(1e-5, 0.0, 0.0))
    f0 = random_state(p, seed=33 + chunk)
    ls = lattice(p, "f16", True, f0)
    lr = lattice(p, "f16", False, f0)
    assert ls.kernel_info()["kernel"] == "staged" and ls.kernel_info()["tile"][2] == chunk
    assert lr.kernel_info()["kernel"] == "register"
    ls.step(5)
    lr.step(5)
    fs, fr = ls.populations(), lr.populations()
    w = O.reference_weights(p).reshape((-1, 1, 1, 1))
    hmax = np.abs(fr - w).max()
    assert np.abs(fs - fr).max() <= 2 * EPS["f16"] * hmax
