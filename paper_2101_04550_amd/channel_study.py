"""Turbulent channel at Re_tau = 180 (Sec. 3.5) run long enough for statistics,
through the library's C ABI.

Geometry: walls in y (halfway bounce-back, or with --walls grad Grad's
approximation as Sec. 3 uses; half width H = 96 rows,
lambda_y = 1), periodic x and z. Lattices:
  stretched -- Sec. 3.5's: 5.6H x 2H x 2H on 384 x 192 x 192 nodes with
               lambda_x = 1.4, T = 0.55;
  cubic     -- the same domain on 538 x 192 x 192 nodes, lambda = 1, at the
               lattice temperature T = 1/3 (T = 0.55 on the cubic lattice
               and T = 0.5 with lambda = (2, 1, 1) are linearly unstable for
               this flow at this viscosity: seeded perturbations of the
               laminar profile grow within a few thousand steps);
  bench      -- the benchmark's channel, 8H x 2H x 2H on 384 x 192 x 192,
               lambda_x = 2, T = 0.5 (kept to show that instability).
rho = 1. The friction velocity is estimated from the log law as in Sec. 3.5,
u_tau = u0 / ((1/kappa) ln Re_tau + B) with u0 = 0.1, kappa = 0.41, B = 5.5;
nu = u_tau H / Re_tau, omega from nu = (1/omega - 1/2) T (Sec. 2.1, eq. nu),
and the constant body force g = Re_tau^2 nu^2 / H^3 = u_tau^2 / H, which
balances the wall friction of a statistically steady channel. Time is
counted as t* = t u_tau / H (eddy turnovers; the paper prints t H / u_tau,
read as this). The flow starts from the laminar profile u_x = u0 (1 - eta^2)
plus a divergence-free perturbation of 10% rms that vanishes at the walls
(inputs.channel_field); there is no trigger forcing.

Every `sample` steps the velocity field is read back and averaged over x and z
(FP64): the mean profile U(y) and the rms fluctuations of each component. The
mean profile is averaged over the samples with t* >= stats_from and given in
wall units, u+ = U/u_tau, y+ = y u_tau / nu (y the distance from the wall
half a node below the first row), with u_tau from the force balance and from
the mean wall gradient. Output: one JSON document.

Usage: python -m paper_2101_04550_amd.channel_study --lattice stretched --tstar 30 --out result.json
       (--omega-bulk B --omega-ghost G: the multi-relaxation-time collision)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

KAPPA, B_LOG = 0.41, 5.5


def setup(lattice, H=96, re_tau=180.0, u0=0.1):
    if lattice == "stretched":
        n, lam, T = (384, 2 * H, 2 * H), (1.4, 1.0, 1.0), 0.55
    elif lattice == "cubic":
        n, lam, T = (538, 2 * H, 2 * H), (1.0, 1.0, 1.0), 1.0 / 3.0
    elif lattice == "bench":
        n, lam, T = (4 * H, 2 * H, 2 * H), (2.0, 1.0, 1.0), 0.5
    else:
        raise ValueError(lattice)
    u_tau = u0 / (math.log(re_tau) / KAPPA + B_LOG)
    nu = u_tau * H / re_tau
    omega = 1.0 / (nu / T + 0.5)
    g = re_tau ** 2 * nu ** 2 / H ** 3
    return dict(n=n, lam=lam, H=H, re_tau=re_tau, u0=u0, T=T, u_tau=u_tau, nu=nu, omega=omega, g=g)


def planar_stats(u):
    """Mean over x and z of each component, and rms fluctuations, per row y.
    u has shape (3, n_z, n_y, n_x)."""
    mean = u.mean(axis=(1, 3))                      # (3, n_y)
    fluct = u - mean[:, None, :, None]
    rms = np.sqrt((fluct * fluct).mean(axis=(1, 3)))
    return mean, rms


def wall_units(prof, c, y):
    """Mean profile and rms fluctuations in wall units.

    prof: (4, n_y) rows U, u_rms, v_rms, w_rms, folded onto the distance from
    the nearest wall; c: the constants of setup(); y: distance of each row
    from the lower wall. The friction velocity is taken from the force
    balance, u_tau^2 = g H (nominal), and also measured from the mean wall
    gradient, u_tau^2 = nu U(y_0) / y_0. The log law u+ = ln(y+)/kappa + B
    is compared over y+ > 30 and y < 0.3 H (its usual range)."""
    H, nu = c["H"], c["nu"]
    half = len(y) // 2
    U, urms, vrms, wrms = (p[:half] for p in prof)
    yy = y[:half]
    ut_force = math.sqrt(c["g"] * H)
    ut_wall = math.sqrt(nu * U[0] / yy[0])
    yplus = yy * ut_force / nu
    uplus = U / ut_force
    log_law = np.log(yplus) / KAPPA + B_LOG
    sel = (yplus > 30) & (yy < 0.3 * H)
    return dict(
        u_tau_force=ut_force, u_tau_wall=ut_wall, re_tau_measured=ut_wall * H / nu,
        bulk_velocity=float(U.mean()), y_plus=yplus.tolist(), u_plus=uplus.tolist(),
        urms_plus=(urms / ut_force).tolist(), vrms_plus=(vrms / ut_force).tolist(),
        wrms_plus=(wrms / ut_force).tolist(),
        log_law_deviation_rms=float(np.sqrt(np.mean((uplus[sel] - log_law[sel]) ** 2))) if sel.any() else None,
        log_law_range=[float(yplus[sel].min()), float(yplus[sel].max())] if sel.any() else None,
        turbulent=bool(np.mean(vrms / ut_force) > 0.2))


def run(lattice, tstar, stats_from, sample, storage, out, seed_offset=3, rates=None, walls="bounce-back"):
    """rates: (omega_bulk, omega_ghost) of the multi-relaxation-time collision,
    or None for LBGK; walls: "bounce-back" (halfway bounce-back of the step
    kernel) or "grad" (Grad's-approximation walls, elbm_faces_* on a lattice
    with one ghost row below and one above the fluid)."""
    import torch  # noqa: F401

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import inputs as I

    from . import elbm as E

    c = setup(lattice)
    n, lam, H = c["n"], c["lam"], c["H"]
    steps_total = int(round(tstar * H / c["u_tau"]))
    fld = I.channel_field(n, lam, u0=c["u0"], seed_offset=seed_offset)
    kw = dict(omega_bulk=rates[0], omega_ghost=rates[1]) if rates else {}
    grad = walls == "grad"
    if grad:
        ns = (n[0], n[1] + 2, n[2])
        rho0 = np.ones((ns[2], ns[1], ns[0]))
        u0 = np.zeros((3, ns[2], ns[1], ns[0]))
        rho0[:, 1:-1, :] = fld.rho
        u0[:, :, 1:-1, :] = fld.u
        lat = E.Lattice(E.make_params(ns, lam=lam, T=c["T"], omega=c["omega"], force=(c["g"], 0.0, 0.0),
                                      storage=storage, **kw))
        lat.init(rho0, u0)
        faces = E.Faces(lat, ["periodic", "periodic", "wall", "wall"])
        advance = faces.step
    else:
        lat = E.Lattice(E.make_params(n, lam=lam, T=c["T"], omega=c["omega"], walls=(False, True, False),
                                      force=(c["g"], 0.0, 0.0), storage=storage, **kw))
        lat.init(fld.rho, fld.u)
        advance = lat.step
    y = (np.arange(n[1]) + 0.5) * lam[1]              # distance from the lower wall
    series, acc, nacc = [], None, 0
    t0 = time.time()
    done = 0
    while done < steps_total:
        k = min(sample, steps_total - done)
        advance(k)
        done += k
        rho, u = lat.fields()
        if grad:
            rho, u = rho[:, 1:-1, :], u[:, :, 1:-1, :]
        if not np.isfinite(u).all():
            raise RuntimeError(f"non-finite velocity at step {done}")
        mean, rms = planar_stats(u)
        ts = done * c["u_tau"] / H
        # both halves folded onto distance from the nearest wall
        Uf = 0.5 * (mean[0] + mean[0][::-1])
        series.append(dict(step=done, tstar=ts, bulk=float(mean[0].mean()), centre=float(Uf[n[1] // 2 - 1]),
                           v_rms_centre=float(0.5 * (rms[1][n[1] // 2 - 1] + rms[1][n[1] // 2])),
                           v_rms_max=float(rms[1].max()), u_rms_max=float(rms[0].max()),
                           min_rho=float(rho.min())))
        if ts >= stats_from:
            prof = np.stack([Uf, 0.5 * (rms[0] + rms[0][::-1]), 0.5 * (rms[1] + rms[1][::-1]),
                             0.5 * (rms[2] + rms[2][::-1])])
            acc = prof if acc is None else acc + prof
            nacc += 1
        print(f"# {lattice} step {done}/{steps_total} t*={ts:.2f} bulk={series[-1]['bulk']:.5f} "
              f"v'rms(centre)={series[-1]['v_rms_centre']:.2e} ({time.time() - t0:.0f} s)", flush=True)
    if grad:
        faces.close()
    lat.close()
    res = dict(lattice=lattice, storage=storage, walls=walls, collision="mrt" if rates else "lbgk",
               rates=list(rates) if rates else None, n=n, lam=lam, constants=c, steps=steps_total, tstar=tstar,
               stats_from=stats_from, samples_averaged=nacc, series=series)
    if nacc:
        res.update(wall_units(acc / nacc, c, y))
    with open(out, "w") as fh:
        json.dump(res, fh)
    print(json.dumps({k: v for k, v in res.items() if k not in ("series", "y_plus", "u_plus", "urms_plus",
                                                                  "vrms_plus", "wrms_plus")}), flush=True)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--lattice", choices=("stretched", "cubic", "bench"), default="stretched")
    ap.add_argument("--tstar", type=float, default=30.0)
    ap.add_argument("--stats-from", type=float, default=20.0)
    ap.add_argument("--sample", type=int, default=5000)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--out", default="channel_study.json")
    ap.add_argument("--omega-bulk", type=float, default=None,
                    help="with --omega-ghost: the multi-relaxation-time collision (default LBGK)")
    ap.add_argument("--omega-ghost", type=float, default=None)
    ap.add_argument("--walls", choices=("bounce-back", "grad"), default="bounce-back",
                    help="halfway bounce-back (the step kernel's) or Grad's approximation (Sec. 3)")
    a = ap.parse_args(argv)
    rates = None
    if a.omega_bulk is not None or a.omega_ghost is not None:
        c = setup(a.lattice)
        rates = (a.omega_bulk if a.omega_bulk is not None else c["omega"],
                 a.omega_ghost if a.omega_ghost is not None else c["omega"])
    run(a.lattice, a.tstar, a.stats_from, a.sample, a.storage, a.out, rates=rates, walls=a.walls)


if __name__ == "__main__":
    main()
