"""Diagnostics folded into the sample steps (diag_every > 0).

A sample step's record is formed by the step kernel from its pulled
(post-streaming) populations in FP64: at every node those are the moments of
the node's post-collision state, which the collision conserves (rho) or moves
by the force impulse (j). So the record written by step s must equal the
oracle's diagnostics of one oracle step taken from the GPU's own state after
s - 1 steps, to the FP64 summation order (mass, momentum, kinetic energy, mode)
and to the FP32 staging of u (enstrophy). Every kernel class is covered:
D2Q9, the D3Q27 register-pull kernel in all three storage formats with walls
and force, and the LDS-staged kernel, periodic and with walls.
"""
import math

import numpy as np
import pytest

import oracle as O
from gpu_helpers import MEASURED, lib, params_for, random_state

pytestmark = pytest.mark.gpu

CASES = {
    # D2Q9, stretched, advected reference, mode tracked
    "d2_shear_f32": dict(n=(32, 64), lam=(2.0, 1.0), T=1 / 3, omega=1.8, storage="f32", u_adv=(0.05, 0.0),
                         mode=((2 * math.pi / 64, 2 * math.pi / 64, 0.0), (-0.7071067811865476, 0.7071067811865476, 0.0))),
    "d2_shear_f16": dict(n=(48, 40), lam=(1.0, 1.0), T=0.5, omega=1.7, storage="f16",
                         mode=((2 * math.pi / 48, 0.0, 0.0), (0.0, 1.0, 0.0))),
    # D3Q27 register-pull kernel: walls on y, force along x, ragged tiles
    "d3_channel_f32": dict(n=(48, 24, 20), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, storage="f32",
                           walls=(False, True, False), force=(1e-5, 0.0, 0.0)),
    "d3_channel_bf16": dict(n=(40, 24, 12), lam=(1.4, 1.0, 1.0), T=0.55, omega=1.8, storage="bf16",
                            walls=(False, True, False), force=(2e-5, 0.0, 0.0)),
    "d3_box_f16_register": dict(n=(40, 20, 18), lam=(1.0, 1.0, 1.0), T=1 / 3, omega=1.9, storage="f16",
                                mode=((0.0, 0.0, 2 * math.pi / 18), (1.0, 0.0, 0.0))),
    # D3Q27 LDS-staged kernel: periodic with a mode, and walls with force
    "d3_box_f16_staged": dict(n=(64, 32, 24), lam=(1.0, 1.0, 1.0), T=0.5, omega=1.9, storage="f16",
                              mode=((2 * math.pi / 64, 0.0, 2 * math.pi / 24), (0.0, 1.0, 0.0))),
    "d3_channel_bf16_staged": dict(n=(128, 32, 12), lam=(2.0, 1.0, 1.0), T=0.5, omega=1.9, storage="bf16",
                                   walls=(False, True, False), force=(1e-5, 0.0, 0.0)),
    # LDS-staged kernel, periodic y with n_y % 16 != 0: rows of the last tile
    # row beyond the axis must add nothing to the record
    "d3_overhang_f16_staged": dict(n=(64, 20, 10), lam=(1.0, 1.2, 1.0), T=0.5, omega=1.8, storage="f16",
                                   mode=((0.0, 2 * math.pi / 20, 0.0), (1.0, 0.0, 0.0))),
}
STAGED = {"d3_box_f16_staged", "d3_channel_bf16_staged", "d3_overhang_f16_staged"}


def make(case, every, capacity=64, seed=0):
    E = lib()
    c = dict(CASES[case])
    storage = c.pop("storage")
    u_adv = c.pop("u_adv", None)
    mode = c.pop("mode", None)
    p = O.Params(**c)
    mk, md = mode if mode else (None, None)
    if mk is not None:
        mk, md = mk[:p.D], md[:p.D]
    lat = E.Lattice(params_for(p, storage, u_adv=u_adv, diag_every=every, diag_capacity=capacity, mode_k=mk,
                               mode_dir=md))
    f0 = random_state(p, seed, amp=0.03, noise=0.002)
    if u_adv is not None:
        # non-equilibrium state around the advected reference
        rho, u = O.moments(f0, p.c, p.lam)
        for a in range(p.D):
            u[a] = u[a] / rho + u_adv[a]
        f0 = O.equilibrium(rho, u, p.T, p.lam, p.c)
    lat.set_populations(f0)
    return p, lat, storage, mk, md


@pytest.mark.parametrize("case", sorted(CASES))
def test_sample_record_matches_oracle_step(case):
    every = 7
    p, lat, storage, mk, md = make(case, every)
    assert (lat.kernel_info()["kernel"] == "staged") == (case in STAGED)
    lat.step(2 * every - 1)
    f_prev = lat.populations()
    lat.step(1)
    hist = lat.diag_history()
    assert [h["step"] for h in hist] == [every, 2 * every]
    d = hist[-1]
    do = O.diagnostics(O.step(f_prev, p), p, mk, md)
    assert abs(d["mass"] / do.mass - 1) <= 1e-12
    for a in range(p.D):
        assert abs(d["mom"][a] - do.mom[a]) <= 1e-12 * do.mass, (a, d["mom"][a], do.mom[a])
    assert abs(d["ke"] / do.ke - 1) <= 1e-9
    assert abs(d["enstrophy"] / do.enstrophy - 1) <= 1e-5
    assert abs(d["min_rho"] - do.min_rho) <= 1e-12
    assert d["nan_count"] == 0
    if mk is not None:
        assert abs(d["mode"] - do.mode) <= 1e-9 * abs(do.mode) + 1e-15
        assert abs(d["max_uperp"] / do.max_uperp - 1) <= 1e-12
    MEASURED.append(dict(test="fused_diag", case=case, storage=storage, component="ke_rel",
                         measured=abs(d["ke"] / do.ke - 1), target=1e-9, bound=1e-9))


@pytest.mark.parametrize("case", sorted(CASES))
def test_sample_steps_leave_the_state_bitwise_unchanged(case):
    """The sample-step variant of each kernel runs the same collision: the
    state after 9 steps with a sample every 2 steps is bitwise the state
    without samples."""
    _, a, _, _, _ = make(case, 2, capacity=8, seed=3)
    _, b, _, _, _ = make(case, 0, capacity=0, seed=3)
    a.step(9)
    b.step(9)
    # (the checkpoints differ in their parameter header; the populations,
    # converted exactly from the stored values, must not)
    assert np.array_equal(a.populations(), b.populations())
    assert [h["step"] for h in a.diag_history()] == [2, 4, 6, 8]


def test_records_are_reproducible_and_ring_wraps():
    _, a, _, _, _ = make("d3_box_f16_staged", 3, capacity=4, seed=5)
    _, b, _, _, _ = make("d3_box_f16_staged", 3, capacity=4, seed=5)
    a.step(20)
    b.step(10)
    b.step(10)
    ha, hb = a.diag_history(), b.diag_history()
    assert [h["step"] for h in ha] == [9, 12, 15, 18]
    assert [h["step"] for h in ha] == [h["step"] for h in hb]
    for x, y in zip(ha, hb):
        for key in ("mass", "ke", "enstrophy", "min_rho"):
            assert x[key] == y[key]
        assert x["mom"] == y["mom"] and x["mode"] == y["mode"]


def test_explicit_diag_after_sample_step_agrees():
    """elbm_diag (a separate pass over the stored state) and the folded record
    of the same step differ only by the rounding of the stored post-collision
    values (FP32 storage) and by the enstrophy's FP32 staging."""
    every = 5
    p, lat, _, mk, md = make("d3_channel_f32", every)
    lat.step(every)
    d_fold = lat.diag_history()[-1]
    d_sep = lat.diag()
    assert d_sep["step"] == d_fold["step"] == every
    assert abs(d_sep["mass"] / d_fold["mass"] - 1) <= 1e-8
    assert abs(d_sep["ke"] / d_fold["ke"] - 1) <= 1e-6
    assert abs(d_sep["enstrophy"] / d_fold["enstrophy"] - 1) <= 1e-5
