"""Plain FP64 NumPy oracle of the extended lattice Boltzmann (LBGK) time step.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module. The product path
(HIP kernels behind the C ABI) never calls it, shares no code with it, and
fails loudly when its own extension is missing.

It follows Saadat, Dorschner and Karlin, "Extended Lattice Boltzmann Model"
(arXiv:2101.04550), Section 2, step by step and in FP64 throughout:

1. Pull streaming, the shift in the LBGK equation (Sec. 2.1, eq. LBGK):
   f_i(x) = f'_i(x - c_i) on a periodic axis; on a bounce-back axis a source
   outside the fluid is replaced by the post-collision population of the
   opposite direction at the same node (halfway bounce-back; the paper's own
   walls use Grad's approximation, Sec. 3, so this is a reading).
2. Moments rho = sum_i f_i and rho u = sum_i v_i f_i (Sec. 2.1, eqs. density,
   momentum) with stretched velocities v_ia = lam_a c_ia (Sec. 2.2).
3. Diagonal anomaly Q~_aaa = rho u_a (lam_a^2 - 3RT) - rho u_a^3 (Sec. 2.3,
   eq. Deviation), R = 1.
4. Its second-order central difference along axis a, node spacing lam_a
   (Sec. 2.3, eq. Paastar1).
5. Extended diagonal pressure P*_aa = T + u_a^2 + (2-w)/(2 rho w) d_a Q~_aaa
   (Sec. 2.4, eq. Paastar), or P^eq_aa = T + u_a^2 for the uncorrected
   product-form control (Sec. 2.3, eq. Peqa).
6. Product-form populations f*_i = rho prod_a Psi_{c_ia}(u_a, P*_aa, lam_a)
   (Sec. 2.2, eqs. phi0S/phiPlusS/phiMinusS and prod; Sec. 2.3, eq. 27eqext).
7. Relaxation f'_i = f_i + w (f*_i - f_i) (Sec. 2.1, eq. LBGK), plus an
   optional constant body force by the exact-difference method
   F_i = f^eq_i(rho, u + g) - f^eq_i(rho, u) (the paper fixes only the force
   magnitude, Sec. 3.5; the scheme is a reading).

Array layout: populations ``f[Q] + grid`` with grid ``(n_y, n_x)`` or
``(n_z, n_y, n_x)``; velocity component ``a`` lives on array axis ``D-1-a``.
The velocity index is lexicographic, i = sum_a (c_ia + 1) 3^a, so the
opposite direction of i is Q-1-i.

Parity pins (closed forms, invariants and special cases fixed by the paper)
live in ``tests/test_oracle_*.py``. Functions without such a pin say so in
their docstring ("parity unpinned").
"""

from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# Velocity set (Sec. 2.2)
# ----------------------------------------------------------------------------

def velocity_set(D: int) -> np.ndarray:
    """Tensor-product velocity set c_ia in {-1, 0, 1}, Q = 3^D (Sec. 2.2, eq. d3q27vel).

    D = 3 gives D3Q27; D = 2 gives its two-dimensional analogue D2Q9 (the paper
    uses 2-D cases in Sec. 3.1, 3.3, 3.4 without naming the lattice).
    Row i holds (c_ix, c_iy[, c_iz]) with i = sum_a (c_ia + 1) 3^a.
    """
    Q = 3 ** D
    c = np.zeros((Q, D), dtype=np.int64)
    for i in range(Q):
        r = i
        for a in range(D):
            c[i, a] = r % 3 - 1
            r //= 3
    return c


def opposite(c: np.ndarray) -> np.ndarray:
    """Index of -c_i for every i, found by search (not by formula)."""
    Q = c.shape[0]
    opp = np.empty(Q, dtype=np.int64)
    for i in range(Q):
        for k in range(Q):
            if np.all(c[k] == -c[i]):
                opp[i] = k
    return opp


def _axis(a: int, D: int) -> int:
    return D - 1 - a


# ----------------------------------------------------------------------------
# Product form (Sec. 2.2) and equilibria (Sec. 2.3)
# ----------------------------------------------------------------------------

def psi(ci: int, u, P, lam: float):
    """The triplet Psi_{-1,0,+1}(u, P, lam) (Sec. 2.2, eqs. phi0S, phiPlusS, phiMinusS)."""
    if ci == 0:
        return 1.0 - P / lam ** 2
    if ci == 1:
        return 0.5 * (u / lam + P / lam ** 2)
    if ci == -1:
        return 0.5 * (-u / lam + P / lam ** 2)
    raise ValueError(ci)


def product_form(rho, u, P, lam, c):
    """f_i = rho * prod_a Psi_{c_ia}(u_a, P_a, lam_a) (Sec. 2.2, eq. prod).

    ``u`` and ``P`` have shape (D,) + grid (or (D,) for one node).
    """
    Q, D = c.shape
    rho = np.asarray(rho, dtype=np.float64)
    out = np.empty((Q,) + rho.shape)
    for i in range(Q):
        v = rho.copy()
        for a in range(D):
            v = v * psi(int(c[i, a]), u[a], P[a], lam[a])
        out[i] = v
    return out


def equilibrium_pressure(u, T):
    """P^eq_aa = R T + u_a^2 with R = 1 (Sec. 2.3, eq. Peqa)."""
    return T + np.asarray(u) ** 2


def equilibrium(rho, u, T, lam, c):
    """f^eq_i = rho Psi_i(u, P^eq, lam) (Sec. 2.3, eq. 27eq)."""
    return product_form(rho, u, equilibrium_pressure(u, T), lam, c)


# ----------------------------------------------------------------------------
# Moments (Sec. 2.1, 2.2)
# ----------------------------------------------------------------------------

def moments(f, c, lam):
    """rho = sum_i f_i and j_a = rho u_a = sum_i lam_a c_ia f_i (Sec. 2.1, eqs. density, momentum)."""
    Q, D = c.shape
    rho = f.sum(axis=0)
    j = np.stack([lam[a] * np.tensordot(c[:, a].astype(np.float64), f, axes=(0, 0))
                  for a in range(D)])
    return rho, j


def anomaly(rho, j, T, lam):
    """Diagonal third-moment anomaly Q~_aaa = rho u_a (lam_a^2 - 3 R T) - rho u_a^3, R = 1
    (Sec. 2.3, eq. Deviation), written with j = rho u: j_a (lam_a^2 - 3T) - j_a^3 / rho^2."""
    D = j.shape[0]
    return np.stack([j[a] * (lam[a] ** 2 - 3.0 * T) - j[a] ** 3 / rho ** 2 for a in range(D)])


def central_difference(q, a, lam_a, wall, D):
    """Second-order central difference of the node field q along axis a, spacing lam_a
    (Sec. 2.3, eq. Paastar1: 'second-order central difference').

    Periodic axis: neighbours wrap. Bounce-back axis (reading; the paper is
    silent on the gradient next to a wall): odd ghost about the halfway wall,
    q(-1) = -q(0) and q(n) = -q(n-1), since the anomaly is odd in the
    wall-normal momentum, which vanishes at the wall. (Pinned: for a purely
    wall-normal flow this is exactly the mirrored periodic continuation.)
    """
    ax = _axis(a, D)
    if not wall:
        qp = np.roll(q, -1, axis=ax)
        qm = np.roll(q, 1, axis=ax)
    else:
        first = np.take(q, [0], axis=ax)
        last = np.take(q, [q.shape[ax] - 1], axis=ax)
        ext = np.concatenate([-first, q, -last], axis=ax)
        n = q.shape[ax]
        qp = np.take(ext, np.arange(2, n + 2), axis=ax)
        qm = np.take(ext, np.arange(0, n), axis=ax)
    return (qp - qm) / (2.0 * lam_a)


# ----------------------------------------------------------------------------
# Parameters and the time step
# ----------------------------------------------------------------------------

@dataclass
class Params:
    """Problem statement of one lattice (Sec. 2, Sec. 3).

    n      -- extents (n_x, n_y[, n_z]); D = len(n)
    lam    -- stretching factors lam_a (Sec. 2.2)
    T      -- temperature, R = 1 (Sec. 3)
    omega  -- relaxation; nu = (1/omega - 1/2) T (Sec. 2.1, eq. nu)
    walls  -- per axis: False periodic, True halfway bounce-back on both faces
    force  -- constant body force g (acceleration) per axis (Sec. 3.5)
    extended -- True: extended equilibrium (eq. 27eqext); False: the
               uncorrected product-form equilibrium (eq. 27eq) as collision target
    """
    n: tuple
    lam: tuple = None
    T: float = 1.0 / 3.0
    omega: float = 1.0
    walls: tuple = None
    force: tuple = None
    extended: bool = True

    def __post_init__(self):
        D = len(self.n)
        self.n = tuple(int(v) for v in self.n)
        self.lam = tuple(float(v) for v in (self.lam if self.lam is not None else (1.0,) * D))
        self.walls = tuple(bool(v) for v in (self.walls if self.walls is not None else (False,) * D))
        self.force = tuple(float(v) for v in (self.force if self.force is not None else (0.0,) * D))

    @property
    def D(self):
        return len(self.n)

    @property
    def c(self):
        return velocity_set(self.D)

    @property
    def has_force(self):
        return any(g != 0.0 for g in self.force)

    @property
    def nu(self):
        """Kinematic viscosity nu = (1/omega - 1/2) R T delta t (Sec. 2.1, eq. nu)."""
        return (1.0 / self.omega - 0.5) * self.T


def stream(fpost, c, walls):
    """Pull streaming f_i(x) = f'_i(x - c_i); halfway bounce-back on wall axes."""
    Q, D = c.shape
    f = np.empty_like(fpost)
    for i in range(Q):
        g = fpost[i]
        for a in range(D):
            if c[i, a] != 0:
                g = np.roll(g, int(c[i, a]), axis=_axis(a, D))
        f[i] = g
    if any(walls):
        opp = opposite(c)
        grid = fpost.shape[1:]
        for i in range(Q):
            mask = np.zeros(grid, dtype=bool)
            for a in range(D):
                if not walls[a] or c[i, a] == 0:
                    continue
                ax = _axis(a, D)
                sl = [slice(None)] * D
                sl[ax] = 0 if c[i, a] == 1 else grid[ax] - 1
                mask[tuple(sl)] = True
            f[i][mask] = fpost[opp[i]][mask]
    return f


def pressure(rho, j, p: Params):
    """Diagonal pressure used in the collision target.

    extended: P*_aa = T + u_a^2 + (2-w)/(2 rho w) d_a Q~_aaa (Sec. 2.4, eq. Paastar),
    the difference of the node values of Q~ at the same time level (reading).
    control:  P^eq_aa = T + u_a^2 (Sec. 2.3, eq. Peqa).
    """
    u = j / rho
    P = equilibrium_pressure(u, p.T)
    if p.extended:
        Qt = anomaly(rho, j, p.T, p.lam)
        pref = (2.0 - p.omega) / (2.0 * rho * p.omega)
        for a in range(p.D):
            P[a] = P[a] + pref * central_difference(Qt[a], a, p.lam[a], p.walls[a], p.D)
    return P


def collide(f, p: Params):
    """Relaxation toward the (extended) product-form equilibrium, plus the body force."""
    c = p.c
    rho, j = moments(f, c, p.lam)
    u = j / rho
    P = pressure(rho, j, p)
    fstar = product_form(rho, u, P, p.lam, c)
    fnew = f + p.omega * (fstar - f)
    if p.has_force:
        g = np.array(p.force).reshape((p.D,) + (1,) * p.D)
        fnew = fnew + equilibrium(rho, u + g, p.T, p.lam, c) - equilibrium(rho, u, p.T, p.lam, c)
    return fnew


def step(fpost, p: Params):
    """One LBGK time step t -> t+1 on the post-collision state (Sec. 2.1, eq. LBGK)."""
    return collide(stream(fpost, p.c, p.walls), p)


def run(fpost, p: Params, nsteps: int):
    for _ in range(int(nsteps)):
        fpost = step(fpost, p)
    return fpost


def init_state(rho, u, p: Params, u_adv=None):
    """Initial post-collision state f'(x, 0) = f^eq(rho, u + u_adv) (reading: the paper
    does not state its initialisation; equilibrium with P^eq, no correction)."""
    u = np.array(u, dtype=np.float64, copy=True)
    if u_adv is not None:
        for a in range(p.D):
            u[a] += u_adv[a]
    return equilibrium(np.asarray(rho, dtype=np.float64), u, p.T, p.lam, p.c)


def reference_weights(p: Params, u_ref=None):
    """f^eq(1, u_ref) per direction; at u_ref = 0 these are the lattice weights
    w_i = prod_a Psi_{c_ia}(0, T, lam_a) (Sec. 2.3 at rest)."""
    D = p.D
    u = np.zeros(D) if u_ref is None else np.asarray(u_ref[:D], dtype=np.float64)
    return equilibrium(np.array(1.0), u.reshape(D), p.T, p.lam, p.c)


# ----------------------------------------------------------------------------
# Single-node update (used to check full-size runs at sampled nodes)
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def _opposite_of_set(D):
    return opposite(velocity_set(D))


def _pull_node(fpost, c, walls, idx):
    """Post-streaming populations at one node (array index tuple)."""
    Q, D = c.shape
    grid = fpost.shape[1:]
    opp = _opposite_of_set(D)
    out = np.empty(Q)
    for i in range(Q):
        src = list(idx)
        outside = False
        for a in range(D):
            ax = _axis(a, D)
            s = idx[ax] - int(c[i, a])
            if s < 0 or s >= grid[ax]:
                if walls[a]:
                    outside = True
                s %= grid[ax]
            src[ax] = s
        out[i] = fpost[(opp[i],) + tuple(idx)] if outside else fpost[(i,) + tuple(src)]
    return out


def step_node(fpost, p: Params, idx):
    """Post-collision populations at node ``idx`` after one step, computed from the
    input state by the same steps as ``step`` but for a single node.

    Parity pinned against ``step`` on small lattices (tests), so that a full-size
    GPU step can be checked node by node without a full-size FP64 step.
    """
    c = p.c
    Q, D = c.shape
    grid = fpost.shape[1:]
    f = _pull_node(fpost, c, p.walls, idx)
    rho = f.sum()
    j = np.array([p.lam[a] * (c[:, a] * f).sum() for a in range(D)])
    u = j / rho
    P = T_plus = p.T + u ** 2
    if p.extended:
        pref = (2.0 - p.omega) / (2.0 * rho * p.omega)
        P = T_plus.copy()
        for a in range(D):
            ax = _axis(a, D)
            vals = []
            for s in (+1, -1):
                nb = list(idx)
                k = idx[ax] + s
                if 0 <= k < grid[ax] or not p.walls[a]:
                    nb[ax] = k % grid[ax]
                    fn = _pull_node(fpost, c, p.walls, tuple(nb))
                    rn = fn.sum()
                    jn = p.lam[a] * (c[:, a] * fn).sum()
                    vals.append(jn * (p.lam[a] ** 2 - 3.0 * p.T) - jn ** 3 / rn ** 2)
                else:
                    qa = j[a] * (p.lam[a] ** 2 - 3.0 * p.T) - j[a] ** 3 / rho ** 2
                    vals.append(-qa)
            P[a] = P[a] + pref * (vals[0] - vals[1]) / (2.0 * p.lam[a])
    fstar = product_form(np.array(rho), u, P, p.lam, c)
    fnew = f + p.omega * (fstar - f)
    if p.has_force:
        g = np.array(p.force)
        fnew = fnew + equilibrium(np.array(rho), u + g, p.T, p.lam, c) \
            - equilibrium(np.array(rho), u, p.T, p.lam, c)
    return fnew


# ----------------------------------------------------------------------------
# Diagnostics (Sec. 3) -- taken from the stored post-collision state
# ----------------------------------------------------------------------------

def velocity(fpost, p: Params):
    """rho and the reported velocity u = j'/rho - g/2 of a post-collision state
    (= (j + rho g/2)/rho with j the pre-force momentum; exact-difference force)."""
    rho, j = moments(fpost, p.c, p.lam)
    u = j / rho
    if p.has_force:
        for a in range(p.D):
            u[a] = u[a] - 0.5 * p.force[a]
    return rho, u


def _grad(q, a, p: Params):
    """Central difference of a velocity component along axis a, spacing lam_a;
    on a wall axis the no-slip ghost q(-1) = -q(0), q(n) = -q(n-1)."""
    return central_difference(q, a, p.lam[a], p.walls[a], p.D)


def vorticity_sq(u, p: Params):
    """|curl u|^2 from central differences (Sec. 3.3 enstrophy integrand)."""
    D = p.D
    if D == 2:
        wz = _grad(u[1], 0, p) - _grad(u[0], 1, p)
        return wz * wz
    wx = _grad(u[2], 1, p) - _grad(u[1], 2, p)
    wy = _grad(u[0], 2, p) - _grad(u[2], 0, p)
    wz = _grad(u[1], 0, p) - _grad(u[0], 1, p)
    return wx * wx + wy * wy + wz * wz


@dataclass
class Diag:
    mass: float
    mom: tuple
    ke: float          # (1/2) <u.u>            (Sec. 3.2)
    enstrophy: float   # <|curl u|^2>           (Sec. 3.3)
    mode: complex      # <u_perp exp(-i k.x)>   (Sec. 3.1 decay measurement)
    max_uperp: float   # max |u_perp|           (Sec. 3.1 'maximum flow velocity')
    min_rho: float
    nan_count: int


def diagnostics(fpost, p: Params, mode_k=None, mode_dir=None) -> Diag:
    """Global FP64 diagnostics of a post-collision state."""
    D = p.D
    rho, u = velocity(fpost, p)
    N = rho.size
    mass = float(rho.sum())
    mom = tuple(float((rho * u[a]).sum()) for a in range(D))
    ke = 0.5 * float((u * u).sum(axis=0).mean())
    ens = float(vorticity_sq(u, p).mean())
    mode = 0j
    maxu = 0.0
    if mode_k is not None and mode_dir is not None:
        lam = p.lam
        phase = np.zeros(rho.shape)
        uperp = np.zeros(rho.shape)
        for a in range(D):
            idx = np.arange(p.n[a], dtype=np.float64) * lam[a]
            bshape = [1] * D
            bshape[_axis(a, D)] = p.n[a]
            phase = phase + mode_k[a] * idx.reshape(bshape)
            uperp = uperp + mode_dir[a] * u[a]
        mode = complex((uperp * np.exp(-1j * phase)).sum() / N)
        maxu = float(np.abs(uperp).max())
    bad = int(np.count_nonzero(~np.isfinite(fpost).all(axis=0)))
    return Diag(mass, mom, ke, ens, mode, maxu, float(rho.min()), bad)


def fit_decay_rate(t, amp, t_start=50):
    """Least-squares slope of ln|amp| against t over t >= t_start, as a positive rate."""
    t = np.asarray(t, dtype=np.float64)
    a = np.log(np.abs(np.asarray(amp)))
    sel = t >= t_start
    A = np.stack([t[sel], np.ones(sel.sum())], axis=1)
    slope, _ = np.linalg.lstsq(A, a[sel], rcond=None)[0]
    return -float(slope)


def measure_viscosity(f0, p: Params, mode_k, mode_dir, nsteps, t_start=50, every=1):
    """Run ``nsteps`` steps recording the mode amplitude |<u_perp e^{-ik.x}>| and fit
    nu = rate / |k|^2 (Sec. 3.1: viscosity from the decay of a shear wave)."""
    k2 = float(sum(k * k for k in mode_k[:p.D]))
    ts, amps = [], []
    f = f0
    for s in range(1, nsteps + 1):
        f = step(f, p)
        if s % every == 0:
            d = diagnostics(f, p, mode_k, mode_dir)
            ts.append(s)
            amps.append(abs(d.mode))
    rate = fit_decay_rate(ts, amps, t_start)
    return rate / k2, f
