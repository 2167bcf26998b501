"""The D3Q27 step linearised about a uniform state, for one Fourier mode: a
27 x 27 matrix built here from the paper's equations (moments, Sec. 2.1;
product form, Sec. 2.2; anomaly and its central difference, Sec. 2.3, eqs.
Deviation and Paastar1; extended pressure, Sec. 2.4, eq. Paastar;
relaxation and pull streaming, eq. LBGK), the three-dimensional counterpart
of tests/test_oracle_linear.py. It

* pins the oracle's nonlinear FP64 D3Q27 step: a small perturbation of all
  27 populations at one wave vector on a stretched box evolves by the matrix
  (1e-6);
* pins the paper's isotropy claim in three dimensions at 1e-4: both shear
  modes of a wave along the body diagonal of a physically cubic box decay
  at nu |k|^2, nu = (1/omega - 1/2) T, on cubic and stretched lattices, at
  rest and advected;
* checks the uncorrected product form against a closed form: its anomaly
  (lambda_a^2 - 3T) j_a adds (nu / T)(lambda_a^2 - 3T) d_a u_a to the normal
  stress of axis a, so a shear mode with wave direction n and velocity
  direction t decays at nu |k|^2 (1 + sum_a (lambda_a^2 - 3T) n_a^2 t_a^2 / T)
  (in two dimensions this is the 1 + (lambda_x^2 + lambda_y^2 - 6T)/(4T) of
  the diagonal wave).
"""
import math

import numpy as np
import pytest

import oracle as O


def _psi(c, u, P, lam):
    return 1.0 - P / lam ** 2 if c == 0 else 0.5 * (c * u / lam + P / lam ** 2)


def _dpsi_du(c, lam):
    return 0.0 if c == 0 else 0.5 * c / lam


def _dpsi_dP(c, lam):
    return -1.0 / lam ** 2 if c == 0 else 0.5 / lam ** 2


def step_matrix_3d(k, U, T, omega, lam, extended=True):
    """One-step operator on the Fourier amplitudes of the post-collision
    populations about rho = 1, u = U (node coordinates x_a = n_a lam_a):
    pull streaming, then the collision."""
    c = O.velocity_set(3)
    Q = c.shape[0]
    Pb = [T + U[a] ** 2 for a in range(3)]
    Mm = np.zeros((4, Q))  # rows: drho, dj_x, dj_y, dj_z
    Mm[0] = 1.0
    for a in range(3):
        Mm[1 + a] = lam[a] * c[:, a]
    du = np.zeros((3, 4), dtype=complex)
    dP = np.zeros((3, 4), dtype=complex)
    for a in range(3):
        du[a, 0] = -U[a]
        du[a, 1 + a] = 1.0
        dP[a] = 2.0 * U[a] * du[a]
        if extended:
            # dQ~_a = (lam_a^2 - 3T) dj_a - d(j_a^3 / rho^2) at rho = 1, j = U
            dQ = np.zeros(4, dtype=complex)
            dQ[1 + a] = lam[a] ** 2 - 3.0 * T - 3.0 * U[a] ** 2
            dQ[0] = 2.0 * U[a] ** 3
            grad = 1j * math.sin(k[a] * lam[a]) / lam[a]
            dP[a] = dP[a] + (2.0 - omega) / (2.0 * omega) * grad * dQ
    J = np.zeros((Q, Q), dtype=complex)
    for i in range(Q):
        ci = [int(c[i, a]) for a in range(3)]
        ps = [_psi(ci[a], U[a], Pb[a], lam[a]) for a in range(3)]
        row = np.zeros(4, dtype=complex)
        row[0] = ps[0] * ps[1] * ps[2]
        for a in range(3):
            others = np.prod([ps[b] for b in range(3) if b != a])
            row += (_dpsi_du(ci[a], lam[a]) * du[a] + _dpsi_dP(ci[a], lam[a]) * dP[a]) * others
        J[i] = row @ Mm
    coll = np.eye(Q) + omega * (J - np.eye(Q))
    shift = np.diag([np.exp(-1j * sum(k[a] * c[i, a] * lam[a] for a in range(3))) for i in range(Q)])
    return coll @ shift


def shear_eigenvalue_3d(k, U, T, omega, lam, t, extended=True):
    """The eigenvalue whose eigenvector carries the most momentum along the
    unit vector t (normal to k), among the six with |mu| closest to 1."""
    M = step_matrix_3d(k, U, T, omega, lam, extended)
    w, V = np.linalg.eig(M)
    c = O.velocity_set(3)
    best, score = None, -1.0
    for m in np.argsort(-np.abs(w))[:6]:
        v = V[:, m]
        j = np.array([lam[a] * (c[:, a] * v).sum() for a in range(3)])
        s = abs(np.dot(t, j)) / (np.abs(v).sum() + 1e-300)
        if s > score:
            best, score = w[m], s
    return best


N_HAT = np.ones(3) / math.sqrt(3.0)
T1 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2.0)
T2 = np.array([1.0, 1.0, -2.0]) / math.sqrt(6.0)


def test_oracle_step_is_the_linear_map():
    """The D3Q27 oracle on a physically cubic stretched box (8 x 12 x 6 nodes,
    lambda = (1.5, 1, 2)) with a 1e-8 perturbation of all 27 populations at
    k = 2 pi / 12 (1, 1, 1): the Fourier amplitudes follow the matrix to 1e-6
    over five steps."""
    lam, T, omega = (1.5, 1.0, 2.0), 0.55, 1.6
    n = (8, 12, 6)
    p = O.Params(n=n, lam=lam, T=T, omega=omega)
    L = n[0] * lam[0]
    k = (2.0 * math.pi / L,) * 3
    X = (np.arange(n[0]) * lam[0])[None, None, :]
    Y = (np.arange(n[1]) * lam[1])[None, :, None]
    Z = (np.arange(n[2]) * lam[2])[:, None, None]
    ph = k[0] * X + k[1] * Y + k[2] * Z
    g = np.random.default_rng(7)
    F = O.equilibrium(np.ones(ph.shape), np.zeros((3,) + ph.shape), T, lam, p.c)
    amp = 1e-8 * (g.standard_normal(27) + 1j * g.standard_normal(27))
    f = F + np.real(amp[:, None, None, None] * np.exp(1j * ph)[None])
    M = step_matrix_3d(k, (0.0, 0.0, 0.0), T, omega, lam)

    def delta(f):
        return ((f - F) * np.exp(-1j * ph)[None]).sum(axis=(1, 2, 3)) / ph.size * 2.0

    for _ in range(5):
        d0 = delta(f)
        f = O.step(f, p)
        assert np.abs(delta(f) - M @ d0).max() < 1e-6 * np.abs(d0).max()


@pytest.mark.parametrize("lam,T,U", [
    ((1.0, 1.0, 1.0), 1 / 3, (0.0, 0.0, 0.0)),
    ((2.0, 1.0, 1.0), 0.5, (0.0, 0.0, 0.0)),
    ((1.4, 1.0, 2.0), 0.55, (0.0, 0.0, 0.0)),
    ((1.4, 1.0, 2.0), 0.55, (0.05, -0.03, 0.02)),
])
@pytest.mark.parametrize("omega", [1.2, 1.8])
def test_shear_decay_along_the_body_diagonal(lam, T, U, omega):
    """Sec. 3.1 in three dimensions: a wave of 1024 x lambda_x along (1, 1, 1)
    of a physically cubic box; both shear modes decay per step by nu |k|^2 to
    1e-4, on the cubic and two stretched lattices, at rest and advected (where
    they also turn by k.U, Galilean invariance, to 1e-4)."""
    Lx = 1024 * lam[0]
    k = tuple(2.0 * math.pi / Lx for _ in range(3))
    kk = 3.0 * k[0] ** 2
    nu = (1.0 / omega - 0.5) * T
    for t in (T1, T2):
        mu = shear_eigenvalue_3d(k, U, T, omega, lam, t)
        assert -math.log(abs(mu)) / (nu * kk) == pytest.approx(1.0, abs=1e-4)
        kU = sum(k[a] * U[a] for a in range(3))
        assert -np.angle(mu) == pytest.approx(kU, abs=1e-4 * k[0])


@pytest.mark.parametrize("lam,T", [((1.0, 1.0, 2.0), 0.5), ((1.5, 1.5, 1.0), 0.4), ((1.0, 1.0, 1.0), 0.5)])
def test_uncorrected_product_form_against_its_closed_form(lam, T):
    """The uncorrected product form (extended = 0) with lambda_x = lambda_y,
    which leaves the shear modes along t1 = (1, -1, 0)/sqrt 2 and
    t2 = (1, 1, -2)/sqrt 6 uncoupled: each decays at
    nu |k|^2 (1 + sum_a (lambda_a^2 - 3T) n_a^2 t_a^2 / T) to 1e-4 (e.g. 0.667
    and 2.0 for lambda = (1, 1, 2), T = 1/2); the extended equilibrium brings
    both to 1."""
    omega = 1.8
    nu = (1.0 / omega - 0.5) * T
    Lx = 1024 * lam[0]
    k = tuple(2.0 * math.pi / Lx for _ in range(3))
    kk = 3.0 * k[0] ** 2
    for t in (T1, T2):
        want = 1.0 + sum((lam[a] ** 2 - 3.0 * T) * N_HAT[a] ** 2 * t[a] ** 2 for a in range(3)) / T
        mu = shear_eigenvalue_3d(k, (0.0, 0.0, 0.0), T, omega, lam, t, extended=False)
        assert -math.log(abs(mu)) / (nu * kk) == pytest.approx(want, abs=1e-4)
        mu = shear_eigenvalue_3d(k, (0.0, 0.0, 0.0), T, omega, lam, t, extended=True)
        assert -math.log(abs(mu)) / (nu * kk) == pytest.approx(1.0, abs=1e-4)
