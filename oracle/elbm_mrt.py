"""Plain FP64 oracle of a multi-relaxation-time collision for the extended
product-form equilibrium.

TEST INFRASTRUCTURE ONLY, like ``elbm_oracle``.

The paper's conclusion (Sec. 4) names multi-relaxation-time collisions as a
direct extension of the model without giving one, so parity against the
paper is unpinned; the pins in tests/test_oracle_mrt.py are the limits and
properties any such collision must have. The reading taken here
relaxes three parts of the non-equilibrium f^neq = f - f* (f* the extended
product-form equilibrium of Sec. 2.3-2.4, as in ``elbm_oracle.collide``)
at three rates:

* the deviatoric non-equilibrium stress at omega (so the shear viscosity
  stays nu = (1/omega - 1/2) T, Sec. 2.1, eq. nu),
* its isotropic part (trace / D) at omega_bulk,
* everything above second order (the part of f^neq that Grad's
  approximation drops) at omega_ghost.

The stress parts are turned back into populations by the linear Grad map G
on the product-form lattice at the collision's own (rho, u, P*):
G_i(Pi) = sum_a dPsi_{c_ia}/dP (Pi_aa) prod_{b != a} Psi_{c_ib}
        + sum_{a<b} c_ia c_ib Pi_ab / (4 lam_a lam_b) prod_{d != a, b} Psi_{c_id},
which carries exactly the stress Pi and no mass or momentum. With
Pi = sum_i v_i v_i f^neq_i (v_ia = lam_a c_ia):
f'_i = f*_i + (1 - omega_ghost) f^neq_i + (omega_ghost - omega) G_i(Pi_dev)
     + (omega_ghost - omega_bulk) G_i(Pi_iso)   (+ the body force of elbm_oracle).
With omega_bulk = omega_ghost = omega this is the LBGK step exactly.

The pressure correction of Sec. 2.4 (eq. Paastar) compensates the anomaly in
a stress that relaxes at omega, with the factor (2 - omega)/(2 omega). Here
the diagonal stress relaxes at two rates, so the correction is split the same
way: its isotropic part (the mean over the axes of d_a Q~_a) takes
(2 - omega_bulk)/(2 omega_bulk), its deviatoric part (2 - omega)/(2 omega).
(With the BGK factor on both parts, the sound waves of a stretched lattice
decay at a rate that depends on the stretching; with the split they decay by
(nu + nu_bulk) k^2 / 2 on every D2Q9 lattice and by (2 nu + nu_bulk) k^2 / 3
on D3Q27, nu_bulk = (1/omega_bulk - 1/2) T, tests/test_oracle_mrt.py.)
"""

from __future__ import annotations

import itertools

import numpy as np

from . import elbm_oracle as O


def _dpsi_dP(c, lam):
    return -1.0 / lam ** 2 if c == 0 else 0.5 / lam ** 2


def grad_map(Pi, u, P, lam, c):
    """The linear Grad map G(Pi) on the product-form lattice: populations that
    carry the second moments Pi (shape (D, D) + grid) at the triplets
    Psi(u, P, lam), and no mass or momentum."""
    Q, D = c.shape
    out = np.zeros((Q,) + np.shape(Pi[0][0]))
    for i in range(Q):
        psis = [O.psi(int(c[i, a]), u[a], P[a], lam[a]) for a in range(D)]
        g = 0.0
        for a in range(D):
            term = _dpsi_dP(int(c[i, a]), lam[a]) * Pi[a][a]
            for b in range(D):
                if b != a:
                    term = term * psis[b]
            g = g + term
        for a, b in itertools.combinations(range(D), 2):
            term = c[i, a] * c[i, b] * Pi[a][b] / (4.0 * lam[a] * lam[b])
            for d in range(D):
                if d != a and d != b:
                    term = term * psis[d]
            g = g + term
        out[i] = g
    return out


def pressure(rho, j, p: O.Params, omega_bulk: float, diff=None):
    """Diagonal pressure of the collision target with the correction split
    into its isotropic and deviatoric parts (module docstring). ``diff(q, a)``
    is the central difference of the anomaly along axis a (default: the
    lattice's own, periodic or next to bounce-back walls)."""
    u = j / rho
    P = O.equilibrium_pressure(u, p.T)
    if p.extended:
        Qt = O.anomaly(rho, j, p.T, p.lam)
        if diff is None:
            G = [O.central_difference(Qt[a], a, p.lam[a], p.walls[a], p.D) for a in range(p.D)]
        else:
            G = [diff(Qt[a], a) for a in range(p.D)]
        iso = sum(G) / p.D
        cd = (2.0 - p.omega) / (2.0 * rho * p.omega)
        cb = (2.0 - omega_bulk) / (2.0 * rho * omega_bulk)
        for a in range(p.D):
            P[a] = P[a] + cd * (G[a] - iso) + cb * iso
    return P


def relax(f, p: O.Params, rho, u, P, omega_bulk: float, omega_ghost: float):
    """The relaxation of the module docstring towards the product form at
    (rho, u, P), plus the body force."""
    c = p.c
    D = p.D
    fstar = O.product_form(rho, u, P, p.lam, c)
    fneq = f - fstar
    v = [p.lam[a] * c[:, a].astype(np.float64) for a in range(D)]
    Pi = [[np.tensordot(v[a] * v[b], fneq, axes=(0, 0)) for b in range(D)] for a in range(D)]
    tr = sum(Pi[a][a] for a in range(D)) / D
    zero = np.zeros_like(tr)
    iso = [[tr if a == b else zero for b in range(D)] for a in range(D)]
    dev = [[Pi[a][b] - iso[a][b] for b in range(D)] for a in range(D)]
    fnew = (fstar + (1.0 - omega_ghost) * fneq + (omega_ghost - p.omega) * grad_map(dev, u, P, p.lam, c)
            + (omega_ghost - omega_bulk) * grad_map(iso, u, P, p.lam, c))
    if p.has_force:
        g = np.array(p.force).reshape((D,) + (1,) * D)
        fnew = fnew + O.equilibrium(rho, u + g, p.T, p.lam, c) - O.equilibrium(rho, u, p.T, p.lam, c)
    return fnew


def collide(f, p: O.Params, omega_bulk: float, omega_ghost: float):
    """Multi-relaxation-time collision (module docstring), plus the body force."""
    rho, j = O.moments(f, p.c, p.lam)
    return relax(f, p, rho, j / rho, pressure(rho, j, p, omega_bulk), omega_bulk, omega_ghost)


def step(fpost, p: O.Params, omega_bulk: float, omega_ghost: float):
    """One time step with the multi-relaxation-time collision."""
    return collide(O.stream(fpost, p.c, p.walls), p, omega_bulk, omega_ghost)


def run(fpost, p: O.Params, nsteps: int, omega_bulk: float, omega_ghost: float):
    for _ in range(int(nsteps)):
        fpost = step(fpost, p, omega_bulk, omega_ghost)
    return fpost
