"""Plain FP64 oracle of open boundaries for D2Q9 lattices: Grad's-approximation
walls, symmetry planes, velocity inlets and outlets.

TEST INFRASTRUCTURE ONLY, like ``elbm_oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.

The paper (Sec. 3, opening paragraph) states that its wall-bounded cases use
Grad's approximation for the walls, after a cited reference, without defining
it, and its flat plate (Sec. 3.4) also has an inlet, an outlet and a symmetry
plane that it does not specify. What follows is the reading taken here
(parity of the time step itself is as in ``elbm_oracle``):

Geometry. The fluid nodes are the n_x x n_y lattice; each face (x-, x+, y-,
y+) has a kind per face node: PERIODIC (the whole face, paired with the
opposite one), SYMMETRY, WALL, INLET or OUTLET. Walls and symmetry planes sit
halfway between the boundary row and the (absent) row outside. A population
i of boundary node x is *missing* when its pull source x - c_i lies outside
along a non-periodic axis. Streaming pulls every other population as usual;
the missing ones are set, per the kind of the face the node is on:

* SYMMETRY (free slip, specular reflection at the halfway plane): the
  population that left the boundary-row node x - c_i,t e_t (shifted along the
  face only) in the mirrored direction i* (normal component reversed).
* WALL (Grad's approximation): f_i = f^G_i(rho_t, u_t, Pi_t) with
  - u_t = (2 u_w + u_f) / 3, the velocity at the boundary node on the line
    through the wall velocity u_w (tangential; zero normal) at distance
    lambda_n / 2 and the velocity u_f of the inward neighbour x_f at distance
    3 lambda_n / 2;
  - rho_t from the known populations and the normal component of u_t, by
    mass and normal-momentum balance: rho_t (1 - s u_t,n / lambda_n) =
    S_0 + 2 S_out (S_0: known populations with c_n = 0, S_out: those moving
    out through the face, s = +1 on a low face, -1 on a high face);
  - Pi_t = rho_t (T I + u_t u_t) + Pi_neq, Pi_neq = -(rho_t T / omega)
    (grad u_t + grad u_t^T) (with the multi-relaxation-time collision of
    ``elbm_mrt``: the deviatoric part of grad u_t + grad u_t^T over omega,
    its trace part over omega_bulk, the rates the bulk relaxes those parts
    at): the normal derivative s (u_f - u_w) /
    (3 lambda_n / 2), the tangential one a central difference of u_f along
    the face over 3 (as u_t = (2 u_w + u_f)/3 with u_w constant);
  - f^G_i = rho_t Psi_{c_ix}(u_t,x, P_xx) Psi_{c_iy}(u_t,y, P_yy)
    + c_ix c_iy Pi_neq,xy / (4 lambda_x lambda_y), P_aa = Pi_t,aa / rho_t:
    the product form (Sec. 2.2, eq. prod) carries every diagonal second
    moment; the last term adds the off-diagonal one without changing rho,
    j or the diagonal moments.
* INLET (prescribed velocity u_in at the halfway plane): bounce-back from a
  surface moving at u_in, f_i = f'_{-i}(x) + f^eq_i(rho_x, u_in) -
  f^eq_{-i}(rho_x, u_in), with the equilibrium of Sec. 2.3 (eq. 27eq) and
  rho_x the node's own post-collision density. (Setting the missing
  populations to an equilibrium at the boundary node instead -- with or
  without a non-equilibrium part -- lets disturbances grow at the inlet on
  the lambda_x = 2 lattice at omega = 1.97; this form stays stable.)
* OUTLET (prescribed density rho_out): the equilibrium at rho_out and the
  inward neighbour's velocity plus the neighbour's non-equilibrium part,
  f_i = f^eq_i(rho_out, u_f) + f_i(x_f) - f^eq_i(rho_f, u_f), with f_i(x_f)
  the neighbour's pulled population. (A plain zero-gradient copy lets the
  mass drift when a wall displaces the stream.)
u_f and rho_f are the moments of the inward neighbour's post-collision
state of the previous step (reported velocity, as ``elbm_oracle.velocity``).
A corner node (on two non-periodic faces) takes the rule of its x face,
which must be INLET or OUTLET; it is set after the other boundary nodes, so
an OUTLET corner uses its neighbour's completed pulled populations.

Collision as ``elbm_oracle.collide`` with one change: the central difference
of the anomaly Q~_a (Sec. 2.3, eq. Paastar1) across a face uses an odd ghost
Q~(outside) = -Q~(boundary node) for SYMMETRY and WALL nodes (the anomaly is
odd in the normal momentum, which vanishes there) and an even ghost
(zero gradient) for INLET and OUTLET nodes.

Parity of these rules against the paper is unpinned (the paper does not
define them); ``tests/test_oracle_faces.py`` pins their own properties:
Grad's populations carry exactly the moments they are built from, a uniform
stream through inlet and outlet stays uniform, a symmetry plane reproduces
the mirrored walled channel, and the force-driven channel between Grad walls
converges to the Navier-Stokes parabola at second order.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import elbm_oracle as O
from . import elbm_mrt as OM

PERIODIC, SYMMETRY, WALL, INLET, OUTLET = 0, 1, 2, 3, 4
FACES = ("x-", "x+", "y-", "y+")


@dataclass
class Faces:
    """Kinds of the four faces of an n_x x n_y D2Q9 fluid lattice.

    kind[F] is either one int for the whole face F (0: x-, 1: x+, 2: y-,
    3: y+) or a sequence with one kind per face node (n_y for x faces, n_x for
    y faces); wall_velocity[F] is the tangential velocity of WALL nodes of F;
    inlet_velocity[F] the (u_x, u_y) of its INLET nodes; outlet_density[F]
    the density of its OUTLET nodes.
    """
    n: tuple
    kind: list
    wall_velocity: tuple = (0.0, 0.0, 0.0, 0.0)
    inlet_velocity: tuple = ((0.0, 0.0),) * 4
    outlet_density: tuple = (1.0, 1.0, 1.0, 1.0)
    node_kind: list = field(init=False)

    def __post_init__(self):
        nx, ny = self.n
        self.node_kind = []
        for F in range(4):
            m = ny if F < 2 else nx
            k = self.kind[F]
            arr = np.full(m, int(k), dtype=np.int64) if np.isscalar(k) else np.asarray(k, dtype=np.int64)
            if arr.shape != (m,):
                raise ValueError(f"face {FACES[F]}: {m} node kinds expected")
            self.node_kind.append(arr)
        for a in range(2):
            lo, hi = self.node_kind[2 * a], self.node_kind[2 * a + 1]
            if (lo == PERIODIC).any() or (hi == PERIODIC).any():
                if not ((lo == PERIODIC).all() and (hi == PERIODIC).all()):
                    raise ValueError("a periodic axis is periodic on both faces, for every node")

    def periodic(self, a):
        return bool((self.node_kind[2 * a] == PERIODIC).all())


def _face_of(F, x, y):
    """Tangential index of node (x, y) on face F."""
    return y if F < 2 else x


def _on_face(F, x, y, nx, ny):
    return (F == 0 and x == 0) or (F == 1 and x == nx - 1) or (F == 2 and y == 0) or (F == 3 and y == ny - 1)


def _node_state(fpost, p, x, y):
    """rho and reported velocity of the post-collision state at one node."""
    rho, u = O.velocity(fpost[:, y:y + 1, x:x + 1], p)
    return float(rho[0, 0]), np.array([u[0][0, 0], u[1][0, 0]])


def grad_populations(rho, u, Pi_neq, T, lam, c):
    """Grad's approximation on the D2Q9 product-form lattice: populations
    with density rho, velocity u and second moments rho (T I + u u) + Pi_neq.

    The product form of Sec. 2.2 (eq. prod) with P_aa = T + u_a^2 +
    Pi_neq,aa / rho has the density, momentum and diagonal second moments;
    c_ix c_iy Pi_neq,xy / (4 lam_x lam_y) adds the off-diagonal one."""
    P = [T + u[a] ** 2 + Pi_neq[a][a] / rho for a in range(2)]
    f = np.empty(c.shape[0])
    for i in range(c.shape[0]):
        f[i] = rho * O.psi(int(c[i, 0]), u[0], P[0], lam[0]) * O.psi(int(c[i, 1]), u[1], P[1], lam[1])
        f[i] += c[i, 0] * c[i, 1] * Pi_neq[0][1] / (4.0 * lam[0] * lam[1])
    return f


def _inlet(f, fpost, p, fc, F, x, y, M):
    """Bounce-back from a surface moving at the inlet velocity."""
    c = p.c
    Q = c.shape[0]
    rho_x, _ = _node_state(fpost, p, x, y)
    feq = O.equilibrium(np.array(rho_x), np.array(fc.inlet_velocity[F], dtype=np.float64), p.T, p.lam, c)
    for i in M:
        j = Q - 1 - i
        f[i, y, x] = fpost[j, y, x] + feq[i] - feq[j]


def _outlet(f, fpost, p, fc, F, x, y, xf, M):
    """Prescribed density, the neighbour's velocity and non-equilibrium part."""
    c = p.c
    rho_f, u_f = _node_state(fpost, p, *xf)
    f_out = O.equilibrium(np.array(float(fc.outlet_density[F])), u_f, p.T, p.lam, c)
    f_nb = O.equilibrium(np.array(rho_f), u_f, p.T, p.lam, c)
    for i in M:
        f[i, y, x] = f_out[i] + f[i, xf[1], xf[0]] - f_nb[i]


def stream_open(fpost, p: O.Params, fc: Faces, omega_bulk=None):
    """Pull streaming with the open-boundary rules (module docstring);
    omega_bulk: the trace rate of the multi-relaxation-time collision (None:
    LBGK)."""
    c = p.c
    nx, ny = p.n
    lam = p.lam
    Q = c.shape[0]
    per = (fc.periodic(0), fc.periodic(1))
    f = O.stream(fpost, c, (False, False))  # periodic pull; missing entries are replaced below

    def inside(x, y):
        return (per[0] or 0 <= x < nx) and (per[1] or 0 <= y < ny)

    def wrap(x, y):
        return x % nx, y % ny

    def missing(x, y):
        return [i for i in range(Q) if not inside(x - c[i, 0], y - c[i, 1])]

    def faces_of(x, y):
        return [F for F in range(4) if not per[F // 2] and _on_face(F, x, y, nx, ny)]

    def inward(F):
        return (1 if F % 2 == 0 else -1)

    corners, single = [], []
    for y in range(ny):
        for x in range(nx):
            fs = faces_of(x, y)
            if len(fs) == 1:
                single.append((x, y, fs[0]))
            elif len(fs) == 2:
                corners.append((x, y, fs))

    mirror = {}
    for a in range(2):
        for i in range(Q):
            cm = c[i].copy()
            cm[a] = -cm[a]
            mirror[(a, i)] = int(np.where((c == cm).all(axis=1))[0][0])

    for (x, y, F) in single:
        kind = int(fc.node_kind[F][_face_of(F, x, y)])
        n_ax, t_ax = F // 2, 1 - F // 2
        s = inward(F)
        M = missing(x, y)
        xf = (x + s, y) if n_ax == 0 else (x, y + s)
        if kind == SYMMETRY:
            for i in M:
                src = [x, y]
                src[t_ax] -= int(c[i, t_ax])
                sx, sy = wrap(*src)
                f[i, y, x] = fpost[mirror[(n_ax, i)], sy, sx]
        elif kind == WALL:
            rho_f, u_f = _node_state(fpost, p, *xf)
            uw = np.zeros(2)
            uw[t_ax] = fc.wall_velocity[F]
            ut = (2.0 * uw + u_f) / 3.0
            S0 = sum(f[i, y, x] for i in range(Q) if c[i, n_ax] == 0)
            Sout = sum(f[i, y, x] for i in range(Q) if c[i, n_ax] == -s)
            rho_t = (S0 + 2.0 * Sout) / (1.0 - s * ut[n_ax] / lam[n_ax])
            grad = np.zeros((2, 2))  # grad[a][b] = d u_b / d x_a
            grad[n_ax] = s * (u_f - uw) / (1.5 * lam[n_ax])
            tp, tm = [list(xf), list(xf)]
            tp[t_ax] += 1
            tm[t_ax] -= 1
            _, u_p = _node_state(fpost, p, *wrap(*tp))
            _, u_m = _node_state(fpost, p, *wrap(*tm))
            grad[t_ax] = (u_p - u_m) / (2.0 * lam[t_ax]) / 3.0
            S = grad + grad.T
            if omega_bulk is None:
                Pi_neq = -(rho_t * p.T / p.omega) * S
            else:
                iso = 0.5 * np.trace(S) * np.eye(2)
                Pi_neq = -(rho_t * p.T) * ((S - iso) / p.omega + iso / omega_bulk)
            fg = grad_populations(rho_t, ut, Pi_neq, p.T, lam, c)
            for i in M:
                f[i, y, x] = fg[i]
        elif kind == INLET:
            _inlet(f, fpost, p, fc, F, x, y, M)
        elif kind == OUTLET:
            _outlet(f, fpost, p, fc, F, x, y, xf, M)
        else:
            raise ValueError(f"face kind {kind} at a boundary node")

    for (x, y, fs) in corners:
        F = [g for g in fs if g < 2][0]
        kind = int(fc.node_kind[F][_face_of(F, x, y)])
        s = inward(F)
        xf = (x + s, y)
        M = missing(x, y)
        if kind == INLET:
            _inlet(f, fpost, p, fc, F, x, y, M)
        elif kind == OUTLET:
            _outlet(f, fpost, p, fc, F, x, y, xf, M)
        else:
            raise ValueError("a corner node needs an INLET or OUTLET x face")
    return f


def _ghost_parity(fc: Faces, F, t):
    k = int(fc.node_kind[F][t])
    return -1.0 if k in (SYMMETRY, WALL) else 1.0


def central_difference_open(q, a, p: O.Params, fc: Faces):
    """Central difference of q along axis a (spacing lam_a) with the face
    ghosts of the module docstring (odd at SYMMETRY / WALL, even at INLET /
    OUTLET, wrap on a periodic axis)."""
    if fc.periodic(a):
        return O.central_difference(q, a, p.lam[a], False, 2)
    ny, nx = q.shape
    if a == 0:
        glo = np.array([_ghost_parity(fc, 0, y) for y in range(ny)]) * q[:, 0]
        ghi = np.array([_ghost_parity(fc, 1, y) for y in range(ny)]) * q[:, -1]
        ext = np.concatenate([glo[:, None], q, ghi[:, None]], axis=1)
        return (ext[:, 2:] - ext[:, :-2]) / (2.0 * p.lam[0])
    glo = np.array([_ghost_parity(fc, 2, x) for x in range(nx)]) * q[0, :]
    ghi = np.array([_ghost_parity(fc, 3, x) for x in range(nx)]) * q[-1, :]
    ext = np.concatenate([glo[None, :], q, ghi[None, :]], axis=0)
    return (ext[2:, :] - ext[:-2, :]) / (2.0 * p.lam[1])


def collide_open(f, p: O.Params, fc: Faces):
    """``elbm_oracle.collide`` with the face ghosts in the anomaly difference."""
    c = p.c
    rho, j = O.moments(f, c, p.lam)
    u = j / rho
    P = O.equilibrium_pressure(u, p.T)
    if p.extended:
        Qt = O.anomaly(rho, j, p.T, p.lam)
        pref = (2.0 - p.omega) / (2.0 * rho * p.omega)
        for a in range(2):
            P[a] = P[a] + pref * central_difference_open(Qt[a], a, p, fc)
    fstar = O.product_form(rho, u, P, p.lam, c)
    fnew = f + p.omega * (fstar - f)
    if p.has_force:
        g = np.array(p.force).reshape((2, 1, 1))
        fnew = fnew + O.equilibrium(rho, u + g, p.T, p.lam, c) - O.equilibrium(rho, u, p.T, p.lam, c)
    return fnew


def collide_open_mrt(f, p: O.Params, fc: Faces, omega_bulk: float, omega_ghost: float):
    """``elbm_mrt.collide`` with the face ghosts in the anomaly difference."""
    rho, j = O.moments(f, p.c, p.lam)
    P = OM.pressure(rho, j, p, omega_bulk, diff=lambda q, a: central_difference_open(q, a, p, fc))
    return OM.relax(f, p, rho, j / rho, P, omega_bulk, omega_ghost)


def step_open(fpost, p: O.Params, fc: Faces, rates=None):
    """One time step with open boundaries: pull with the face rules, then
    collide (LBGK, or the multi-relaxation-time collision at rates =
    (omega_bulk, omega_ghost))."""
    if any(p.walls):
        raise ValueError("open faces replace the bounce-back walls: Params.walls must be all False")
    if rates is None:
        return collide_open(stream_open(fpost, p, fc), p, fc)
    return collide_open_mrt(stream_open(fpost, p, fc, rates[0]), p, fc, *rates)


def run_open(fpost, p: O.Params, fc: Faces, nsteps: int, rates=None):
    for _ in range(int(nsteps)):
        fpost = step_open(fpost, p, fc, rates)
    return fpost
