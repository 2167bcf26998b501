"""Plain FP64 oracle of Grad's-approximation walls on D3Q27 channels: walls
on the two y faces, x and z periodic (the geometry of Sec. 3.5, whose walls
the paper takes as Grad's approximation, Sec. 3).

TEST INFRASTRUCTURE ONLY, like ``elbm_oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.

The paper does not define the wall, so parity against it is unpinned; the
reading is the three-dimensional form of the D2Q9 wall of ``elbm_faces``
(tests/test_oracle_walls3d.py pins its own properties). The walls sit
halfway below the first and above the last fluid row. A population i of a
boundary-row node x is missing when its pull source x - c_i lies beyond the
wall (c_iy = s, s = +1 at the low wall, -1 at the high wall); the others are
pulled as usual (x and z periodic). The missing ones are Grad's
approximation f^G_i(rho_t, u_t, Pi_t):

* u_t = (2 u_w + u_f) / 3, with u_w the wall velocity (along x) and u_f the
  reported velocity of the inward neighbour x + s e_y (post-collision state
  of the previous step);
* rho_t from the known populations by mass and normal-momentum balance,
  rho_t (1 - s u_t,y / lambda_y) = S_0 + 2 S_out (S_0: known populations
  with c_y = 0, S_out: those with c_y = -s);
* grad u_t: along y s (u_f - u_w) / (3 lambda_y / 2); along x and z the
  central difference of u_f along the wall, over 3;
* Pi_neq = -(rho_t T / omega) S, S = grad u_t + grad u_t^T (with the
  multi-relaxation-time collision of ``elbm_mrt``: S_dev / omega +
  S_iso / omega_bulk, S_iso = (tr S / 3) I);
* f^G_i = rho_t prod_a Psi_{c_ia}(u_t,a, P_aa) + sum_{a<b} c_ia c_ib
  Pi_neq,ab / (4 lambda_a lambda_b) Psi_{c_id}(u_t,d, P_dd), d the third
  axis, P_aa = T + u_t,a^2 + Pi_neq,aa / rho_t: the product form (Sec. 2.2,
  eq. prod) carries the density, momentum and diagonal second moments, each
  off-diagonal term one off-diagonal moment and nothing else.

The collision is ``elbm_oracle.collide`` (or ``elbm_mrt``) with the y axis
marked as a wall for the anomaly difference: odd ghost (reading R6 of the
bounce-back lattice; the anomaly is odd in the wall-normal momentum).
"""

from __future__ import annotations

import itertools

import numpy as np

from . import elbm_mrt as OM
from . import elbm_oracle as O


def grad_populations_3d(rho, u, Pi_neq, T, lam, c):
    """Grad's approximation on the D3Q27 product-form lattice (module
    docstring): density rho, velocity u[a], second moments
    rho (T I + u u) + Pi_neq[a][b]. Scalars or arrays of one shape (one value
    per wall node); returns the Q populations."""
    P = [T + u[a] ** 2 + Pi_neq[a][a] / rho for a in range(3)]
    out = []
    for i in range(c.shape[0]):
        ps = [O.psi(int(c[i, a]), u[a], P[a], lam[a]) for a in range(3)]
        g = rho * ps[0] * ps[1] * ps[2]
        for a, b in itertools.combinations(range(3), 2):
            d = 3 - a - b
            g = g + c[i, a] * c[i, b] * Pi_neq[a][b] / (4.0 * lam[a] * lam[b]) * ps[d]
        out.append(g)
    return np.array(out)


def _check(p: O.Params):
    if p.D != 3 or tuple(p.walls) != (False, True, False):
        raise ValueError("D3Q27 with walls=(False, True, False): the y axis carries the Grad walls")


def stream_walls(fpost, p: O.Params, wall_u=(0.0, 0.0), omega_bulk=None):
    """Pull streaming with Grad's walls on the y faces (module docstring);
    wall_u: x-velocity of the low and the high wall; omega_bulk: the trace
    rate of the multi-relaxation-time collision (None: LBGK). Every wall
    node of a face is handled at once (arrays over z and x)."""
    _check(p)
    c, lam, T = p.c, p.lam, p.T
    ny = p.n[1]
    f = O.stream(fpost, c, (False, False, False))  # periodic pull; the missing entries are replaced
    _, u_all = O.velocity(fpost, p)                 # reported velocity of the previous state
    for s, y in ((1, 0), (-1, ny - 1)):
        yf = y + s
        uw = [wall_u[0] if s == 1 else wall_u[1], 0.0, 0.0]
        uf = [u_all[a][:, yf, :] for a in range(3)]          # (n_z, n_x) each
        ut = [(2.0 * uw[a] + uf[a]) / 3.0 for a in range(3)]
        S0 = sum(f[i, :, y, :] for i in range(c.shape[0]) if c[i, 1] == 0)
        Sout = sum(f[i, :, y, :] for i in range(c.shape[0]) if c[i, 1] == -s)
        rho_t = (S0 + 2.0 * Sout) / (1.0 - s * ut[1] / lam[1])
        grad = [[None] * 3 for _ in range(3)]  # grad[a][b] = d u_b / d x_a
        for b in range(3):
            grad[1][b] = s * (uf[b] - uw[b]) / (1.5 * lam[1])
            grad[0][b] = (np.roll(uf[b], -1, axis=1) - np.roll(uf[b], 1, axis=1)) / (2.0 * lam[0]) / 3.0
            grad[2][b] = (np.roll(uf[b], -1, axis=0) - np.roll(uf[b], 1, axis=0)) / (2.0 * lam[2]) / 3.0
        S = [[grad[a][b] + grad[b][a] for b in range(3)] for a in range(3)]
        if omega_bulk is None:
            Pi = [[-(rho_t * T / p.omega) * S[a][b] for b in range(3)] for a in range(3)]
        else:
            iso = (S[0][0] + S[1][1] + S[2][2]) / 3.0
            Pi = [[-(rho_t * T) * ((S[a][b] - (iso if a == b else 0.0)) / p.omega
                                   + (iso / omega_bulk if a == b else 0.0)) for b in range(3)] for a in range(3)]
        fg = grad_populations_3d(rho_t, ut, Pi, T, lam, c)
        for i in range(c.shape[0]):
            if c[i, 1] == s:
                f[i, :, y, :] = fg[i]
    return f


def step(fpost, p: O.Params, wall_u=(0.0, 0.0), rates=None):
    """One time step: pull with the Grad walls, then the collision (LBGK, or
    the multi-relaxation-time one at rates = (omega_bulk, omega_ghost))."""
    if rates is None:
        return O.collide(stream_walls(fpost, p, wall_u), p)
    return OM.collide(stream_walls(fpost, p, wall_u, rates[0]), p, *rates)


def run(fpost, p: O.Params, nsteps: int, wall_u=(0.0, 0.0), rates=None):
    for _ in range(int(nsteps)):
        fpost = step(fpost, p, wall_u, rates)
    return fpost
