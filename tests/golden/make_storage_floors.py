"""Writes tests/golden/storage_floors.txt: the error that each storage format
alone causes in the workloads of the parity tests (calls only oracle/, inputs/
and the storage rounding of tests/storage_rounding.py).

For every case the FP64 oracle runs 100 steps twice from the same initial
state: once exactly, once with the state rounded to the storage format after
the initialisation and after every step (h = f - w rounded as the library
stores it). The relative L2 difference of each velocity component between the
two runs is the storage floor: no kernel that stores its populations in that
format, whatever precision it computes in, can be expected below it.

Usage (from the repository root): python tests/golden/make_storage_floors.py
"""
import math
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for d in (ROOT, os.path.dirname(HERE)):
    if d not in sys.path:
        sys.path.insert(0, d)

import numpy as np  # noqa: E402

import inputs as I  # noqa: E402
import oracle as O  # noqa: E402
from storage_rounding import round_state  # noqa: E402

OUT = os.path.join(HERE, "storage_floors.txt")
STEPS = 100
STORAGES = ("f32", "f16", "bf16")


def channel_params(n=(96, 48, 48), lam=(2.0, 1.0, 1.0), omega=1.976785, T=0.5, re_tau=180.0):
    """Sec. 3.5: nu = (1/omega - 1/2) T, g = Re_tau^2 nu^2 / H^3, H the half width."""
    H = 0.5 * n[1] * lam[1]
    nu = (1.0 / omega - 0.5) * T
    g = re_tau ** 2 * nu ** 2 / H ** 3
    return O.Params(n=n, lam=lam, T=T, omega=omega, walls=(False, True, False), force=(g, 0.0, 0.0))


def case(name):
    """(oracle params, field, u_adv) of a named parity case."""
    if name.startswith("cfg1"):
        T = 0.5 if "T0.5" in name else 1.0 / 3.0
        adv = name.endswith("uadv")
        fld = I.shear_wave_axis((64, 64), U0=0.0 if adv else 0.1, A=0.01)
        return O.Params(n=(64, 64), T=T, omega=1.8), fld, ((0.1, 0.0) if adv else None)
    if name == "dsl256":
        return O.Params(n=(256, 256), T=0.5, omega=1.973061), I.double_shear_layer((256, 256)), None
    if name == "hit64":
        return O.Params(n=(64, 64, 64), T=0.5, omega=1.892885), I.hit_field(64, k0=4.0, urms=0.05), None
    if name == "channel96":
        p = channel_params()
        return p, I.channel_field(p.n, p.lam), None
    if name == "channel128x48x32":
        p = channel_params(n=(128, 48, 32))
        return p, I.channel_field(p.n, p.lam), None
    raise KeyError(name)


CASES = ("cfg1_T0.5_uadv", "cfg1_T0.33_uadv", "cfg1_T0.5_rest", "cfg1_T0.33_rest", "dsl256", "hit64", "channel96",
         "channel128x48x32")


def floors(name, storages=STORAGES, steps=STEPS):
    """{storage: [rel-L2 of u_a]} for one case (and, for the axis-aligned wave,
    the maximum of |u_x - U0|, U0 = 0.1, under key storage + ':ux_dev')."""
    p, fld, uadv = case(name)
    f0 = O.init_state(fld.rho, fld.u, p, u_adv=uadv)
    w = O.reference_weights(p, uadv).reshape((-1,) + (1,) * p.D)
    fe = O.run(f0, p, steps)
    _, ue = O.velocity(fe, p)
    out = {}
    for st in storages:
        f = round_state(f0, w, st)
        for _ in range(steps):
            f = round_state(O.step(f, p), w, st)
        _, ur = O.velocity(f, p)
        out[st] = [float(np.linalg.norm(ur[a] - ue[a]) / np.linalg.norm(ue[a])) for a in range(p.D)]
        if name.startswith("cfg1"):
            out[st + ":ux_dev"] = float(np.abs(ur[0] - 0.1).max())
    return name, out


VISC_CASES = tuple((T, st, n) for T in (1.0 / 3.0, 0.5) for st in ("f16",) for n in (500, 1000))


def viscosity_floor(args):
    """Fitted nu / (1/omega - 1/2) T of the advected axis-aligned wave (64^2,
    a0 = 0.01, U0 = 0.1 as the deviation reference, omega = 1.8; Sec. 3.1)
    over n steps, with the state rounded to the storage format after every
    step: the part of the viscosity error the format alone causes."""
    T, st, nsteps = args
    fld = I.shear_wave_axis((64, 64), U0=0.0, A=0.01)
    p = O.Params(n=(64, 64), T=T, omega=1.8)
    uadv = (0.1, 0.0)
    w = O.reference_weights(p, uadv).reshape((-1, 1, 1))
    f = round_state(O.init_state(fld.rho, fld.u, p, u_adv=uadv), w, st)
    ts, amps = [], []
    for s in range(1, nsteps + 1):
        f = round_state(O.step(f, p), w, st)
        if s % 5 == 0:
            ts.append(s)
            amps.append(abs(O.diagnostics(f, p, fld.mode_k, fld.mode_dir).mode))
    return args, O.fit_decay_rate(ts, amps, 50) / fld.mode_k[0] ** 2 / p.nu


def main():
    with ProcessPoolExecutor(max_workers=min(len(CASES), os.cpu_count() or 1)) as ex:
        visc = list(ex.map(viscosity_floor, VISC_CASES))
        results = dict(ex.map(floors, CASES))
    lines = [
        "# Storage floors: rel-L2 per velocity component after 100 steps between the FP64 oracle",
        "# (Sec. 2.1-2.4 step) and the same oracle with its populations rounded to the storage",
        "# format after every step (deviations h = f - w from the reference equilibrium w: FP32 h,",
        "# FP16 h * 2^12, BF16 h, round to nearest even). Written by make_storage_floors.py.",
        "# columns: case storage component value   (component u0/u1/u2 = u_x/u_y/u_z, ux_dev = max|u_x - U0|)",
    ]
    for name in CASES:
        for key, val in results[name].items():
            if key.endswith(":ux_dev"):
                lines.append(f"{name} {key.split(':')[0]} ux_dev {val:.6e}")
            else:
                for a, v in enumerate(val):
                    lines.append(f"{name} {key} u{a} {v:.6e}")
    lines.append("# viscosity fits (Sec. 3.1): case storage nu<steps> fitted-nu / nu")
    for (T, st, nsteps), r in visc:
        lines.append(f"visc_cfg1_T{0.5 if T == 0.5 else 0.33}_uadv {st} nu{nsteps} {r:.6e}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(OUT)


def load(path=OUT):
    """{(case, storage, component): value} from the golden file."""
    table = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, st, comp, val = line.split()
        table[(name, st, comp)] = float(val)
    return table


if __name__ == "__main__":
    main()
