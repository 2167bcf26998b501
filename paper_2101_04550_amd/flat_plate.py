"""Laminar boundary layer over a flat plate (Sec. 3.4) through the library's
C ABI, on the regular and the stretched D2Q9 lattice, against the Blasius
similarity solution.

Set-up (Sec. 3.4): Ma = u_inf / sqrt(T) = 0.1 at T = 1/3, Re = u_inf L / nu =
4000 with L the plate length, domain 200 x 200 (in units of the y spacing,
lambda_y = 1), the plate from x = L_x / 4 to the outlet (L = 150) with a
symmetry plane ahead of it. Faces (the library's open faces): velocity inlet
(u_inf, 0) at the halfway plane x = 0, outlet at density 1 on the last
column, bottom symmetry plane then Grad wall, top symmetry plane (free
stream; the paper does not name it). Nodes sit at x_i = (i + 1/2) lambda_x
and y_j = j + 1/2 from the inlet plane and the bottom face; a bottom node
belongs to the plate when x_i > L_x / 4 (so the leading edge is the cell
face at x = 50), and L = L_x - 50 = 150. The flow starts uniform at u_inf
and runs to a steady state; the fields analysed are the mean of the samples
taken after `avg_from` of the run (acoustic waves between inlet and outlet
decay slowly at omega near 2).

Outputs: the streamwise velocity profile near the end of the plate against
Blasius' f'(eta), eta = y sqrt(u_inf / (nu x)) (Sec. 3.4), and the skin
friction C_f = tau_w / (rho u_inf^2 / 2), tau_w = rho nu du/dy at the wall
(second-order one-sided difference through the wall, the first two rows),
against C_f = 0.664 / sqrt(Re_x) (Sec. 3.4).

Usage: python -m paper_2101_04550_amd.flat_plate --lambda-x 2 --steps 60000 --out plate.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def blasius(eta_max=10.0, h=5e-3):
    """Blasius' boundary layer: f''' + f f'' / 2 = 0, f(0) = f'(0) = 0,
    f'(inf) = 1, by RK4 integration and bisection on f''(0). Returns
    (f''(0), eta grid, f'(eta))."""
    def shoot(s):
        y = np.array([0.0, 0.0, s])
        n = int(round(eta_max / h))
        out = np.empty(n + 1)
        out[0] = 0.0

        def rhs(v):
            return np.array([v[1], v[2], -0.5 * v[0] * v[2]])
        for k in range(n):
            k1 = rhs(y)
            k2 = rhs(y + 0.5 * h * k1)
            k3 = rhs(y + 0.5 * h * k2)
            k4 = rhs(y + h * k3)
            y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
            out[k + 1] = y[1]
        return y[1], out
    lo, hi = 0.2, 0.5
    for _ in range(42):
        mid = 0.5 * (lo + hi)
        fp, _ = shoot(mid)
        if fp > 1.0:
            hi = mid
        else:
            lo = mid
    s = 0.5 * (lo + hi)
    _, prof = shoot(s)
    return s, np.linspace(0.0, eta_max, prof.size), prof


def setup(lam_x, scale=1, Ma=0.1, T=1.0 / 3.0, Re=4000.0):
    """Constants of the plate on a lattice stretched by lam_x; `scale` refines
    the paper's 200 x 200 domain (scale 2: 400 x 400 in units of the y
    spacing, the same Re, a twice larger nu in lattice units)."""
    Lx = Ly = 200.0 * scale
    nx = int(round(Lx / lam_x))
    ny = int(round(Ly))
    u_inf = Ma * math.sqrt(T)
    x = (np.arange(nx) + 0.5) * lam_x
    plate = x > Lx / 4.0
    x_le = float(x[plate][0] - 0.5 * lam_x)
    L = Lx - x_le
    nu = u_inf * L / Re
    omega = 1.0 / (nu / T + 0.5)
    return dict(nx=nx, ny=ny, lam=(float(lam_x), 1.0), T=T, u_inf=u_inf, nu=nu, omega=omega, x_le=x_le, L=L,
                plate=plate, x=x, Lx=Lx, scale=scale)


def analyse(u, c):
    """Profile near the plate's end and skin friction from the fluid velocity
    u (2, ny, nx), against Blasius both with the free-stream velocity u_inf
    and with the local edge velocity U_e(x) (the stream speeds up along the
    plate as the boundary layer displaces it within the closed top and the
    fixed inlet flux), U_e taken at eta = 8."""
    s, eta_b, fp_b = blasius()
    x, x_le, nu, U = c["x"], c["x_le"], c["nu"], c["u_inf"]
    ny = c["ny"]
    y = np.arange(ny) + 0.5  # distance from the halfway bottom face
    xs = x - x_le

    def edge(i):
        return float(np.interp(8.0 * math.sqrt(nu * xs[i] / U), y, u[0][:, i]))

    # profile at 90% of the plate (clear of the outlet)
    i_prof = int(np.argmin(np.abs(xs - 0.9 * c["L"])))
    xp = xs[i_prof]
    Ue = edge(i_prof)
    out = dict(fpp0=s, profile_x=float(xp), profile_edge_velocity=Ue / U)
    for tag, V in (("", U), ("_edge", Ue)):
        eta = y * math.sqrt(V / (nu * xp))
        sel = eta <= 8.0
        up = u[0][:, i_prof][sel] / V
        blas = np.interp(eta[sel], eta_b, fp_b)
        out.update({f"profile{tag}_eta": eta[sel].tolist(), f"profile{tag}_u": up.tolist(),
                    f"profile{tag}_blasius": blas.tolist(), f"profile{tag}_max_dev": float(np.abs(up - blas).max())})
    # skin friction along the plate
    dudy = (9.0 * u[0][0] - u[0][1]) / 3.0
    on = c["plate"] & (xs >= 0.2 * c["L"]) & (xs <= 0.9 * c["L"])
    idx = np.nonzero(on)[0]
    Ues = np.array([edge(i) for i in idx])
    out["cf_x"] = xs[on].tolist()
    for tag, V in (("", np.full(idx.size, U)), ("_edge", Ues)):
        cf = 2.0 * nu * dudy[on] / V ** 2
        cf_bl = 0.664 / np.sqrt(V * xs[on] / nu)
        dev = cf / cf_bl - 1.0
        out.update({f"cf{tag}": cf.tolist(), f"cf{tag}_blasius": cf_bl.tolist(),
                    f"cf{tag}_rms_rel_dev": float(np.sqrt(np.mean(dev ** 2))),
                    f"cf{tag}_max_rel_dev": float(np.abs(dev).max())})
    out["edge_velocity"] = (Ues / U).tolist()
    return out


def run(lam_x, steps, check_every=5000, out=None, scale=1, avg_from=0.5, storage="f32"):
    import torch  # noqa: F401

    from . import elbm as E

    c = setup(lam_x, scale)
    nx, ny = c["nx"], c["ny"]
    N = (nx + 2, ny + 2)
    lat = E.Lattice(E.make_params(N, lam=c["lam"], T=c["T"], omega=c["omega"], storage=storage))
    rho = np.ones((N[1], N[0]))
    u0 = np.zeros((2, N[1], N[0]))
    u0[0] = c["u_inf"]
    lat.init(rho, u0)
    bottom = [E.FACE_WALL if p else E.FACE_SYMMETRY for p in c["plate"]]
    faces = E.Faces(lat, ["inlet", "outlet", bottom, "symmetry"], inlet_velocity=((c["u_inf"], 0.0),) * 4)
    t0 = time.time()
    done, prev, hist = 0, None, []
    acc, nacc = None, 0
    while done < steps:
        k = min(check_every, steps - done)
        faces.step(k)
        done += k
        _, u = lat.fields()
        uf = u[:, 1:ny + 1, 1:nx + 1]
        if not np.isfinite(uf).all():
            raise RuntimeError(f"non-finite velocity at step {done}")
        change = None if prev is None else float(np.abs(uf - prev).max() / c["u_inf"])
        prev = uf.copy()
        if done > avg_from * steps:
            acc = uf.copy() if acc is None else acc + uf
            nacc += 1
        hist.append(dict(step=done, max_change=change))
        print(f"# lambda_x={lam_x} step {done}/{steps} max change {change} ({time.time() - t0:.1f} s)", flush=True)
    faces.close()
    lat.close()
    mean = acc / nacc
    res = dict(lambda_x=lam_x, scale=scale, storage=storage, nodes=[nx, ny], T=c["T"], u_inf=c["u_inf"], nu=c["nu"], omega=c["omega"],
               x_leading_edge=c["x_le"], plate_length=c["L"], steps=steps, samples_averaged=nacc,
               last_vs_mean=float(np.abs(prev - mean).max() / c["u_inf"]), history=hist)
    res.update(analyse(mean, c))
    if out:
        with open(out, "w") as fh:
            json.dump(res, fh)
    print(json.dumps({k: v for k, v in res.items() if not isinstance(v, list)}), flush=True)
    return res, mean


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--lambda-x", type=float, default=2.0)
    ap.add_argument("--steps", type=int, default=60000)
    ap.add_argument("--check-every", type=int, default=5000)
    ap.add_argument("--scale", type=int, default=1)
    ap.add_argument("--avg-from", type=float, default=0.5, help="average the fields over the checks after this fraction")
    ap.add_argument("--out", default="flat_plate.json")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    a = ap.parse_args(argv)
    run(a.lambda_x, a.steps, a.check_every, a.out, a.scale, a.avg_from, a.storage)


if __name__ == "__main__":
    main()
