"""The storage floors behind the FP16 / BF16 / FP32 parity bounds (no GPU).

tests/golden/storage_floors.txt holds, per parity case, storage format and
velocity component, the rel-L2 error that rounding the populations to the
storage format after every step causes in an otherwise exact FP64 run of the
oracle (tests/golden/make_storage_floors.py). The GPU parity tests take their
bound from it where the floor lies above the target tolerance. Here: the
rounding helper rounds as the formats do, the file is what its script writes
(one case recomputed), and the floors scale with the formats' precisions.
"""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_storage_floors as MSF  # noqa: E402
import storage_rounding as R  # noqa: E402


@pytest.mark.parametrize("storage,bits", [("f32", 24), ("f16", 11), ("bf16", 8)])
def test_rounding_is_round_to_nearest_of_the_format(storage, bits):
    g = np.random.default_rng(5)
    h = g.standard_normal(20000) * 10.0 ** g.uniform(-6, -1, 20000)
    r = R.round_values(h, storage)
    # (FP16 below 2^-14 in storage units is subnormal: absolute spacing 2^-24)
    sub = 2.0 ** -25 / R.SCALE[storage] if storage == "f16" else 0.0
    assert np.all(np.abs(r - h) <= np.abs(h) * 2.0 ** -bits + sub)
    assert np.array_equal(R.round_values(r, storage), r)  # representable values stay
    # a tie goes to the even neighbour: in storage units 1 + 2^-bits lies halfway
    # between 1 (even) and 1 + 2^(1-bits) (odd); 1 + 3 2^-bits between that odd
    # value and the even 1 + 2^(2-bits)
    s = R.SCALE[storage]
    assert R.round_values(np.array([(1.0 + 2.0 ** -bits) / s]), storage)[0] * s == 1.0
    assert R.round_values(np.array([(1.0 + 3 * 2.0 ** -bits) / s]), storage)[0] * s == 1.0 + 2.0 ** (2 - bits)


def test_golden_file_is_what_the_script_writes():
    table = MSF.load()
    name, got = MSF.floors("cfg1_T0.5_uadv")
    for st, vals in got.items():
        if st.endswith(":ux_dev"):
            assert got[st] == pytest.approx(table[(name, st.split(":")[0], "ux_dev")], rel=1e-6)
        else:
            for a, v in enumerate(vals):
                assert v == pytest.approx(table[(name, st, f"u{a}")], rel=1e-6)


def test_floors_scale_with_the_precision_of_the_format():
    table = MSF.load()
    cases = {k[0] for k in table if not k[0].startswith("visc_")}
    assert cases == set(MSF.CASES)
    for c in cases:
        comps = sorted({k[2] for k in table if k[0] == c and k[2] != "ux_dev"})
        worst = {s: max(table[(c, s, comp)] for comp in comps) for s in ("f32", "f16", "bf16")}
        # 2^13 between FP32 and FP16 significands, 2^3 between FP16 and BF16;
        # the worst component's error grows about in proportion (random
        # rounding, same dynamics); single components of a nearly uniform
        # flow can drift either way
        for comp in comps:
            assert 1e2 < table[(c, "f16", comp)] / table[(c, "f32", comp)] < 1e5, (c, comp)
        assert 2 < worst["bf16"] / worst["f16"] < 40, c


def test_viscosity_floor_entries():
    """The FP16 viscosity-fit floors the GPU viscosity test relies on: under 1%
    over 500 steps, and closer over 1000 (the fit sees a larger decay)."""
    table = MSF.load()
    for T in ("0.33", "0.5"):
        r500 = table[(f"visc_cfg1_T{T}_uadv", "f16", "nu500")]
        r1000 = table[(f"visc_cfg1_T{T}_uadv", "f16", "nu1000")]
        assert abs(r500 - 1) < 1e-2
        assert abs(r1000 - 1) < abs(r500 - 1)
