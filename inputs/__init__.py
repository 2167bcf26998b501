"""Seeded synthetic initial fields for the extended lattice Boltzmann workloads.

This module is shared by the FP64 oracle, the tests and the benchmark. It holds
no lattice Boltzmann arithmetic: every generator returns only macroscopic
fields (density and velocity) on the node grid, in FP64, built from closed-form
flow profiles or from a seeded PCG64 generator.

Array conventions (used by every caller):

* A D-dimensional field has array shape ``(n_y, n_x)`` (D=2) or
  ``(n_z, n_y, n_x)`` (D=3): the x index is fastest in memory.
* A velocity field has shape ``(D,) + grid``; component ``a`` (0=x, 1=y, 2=z)
  lives on array axis ``D - 1 - a``.
* Physical coordinates: node ``i_a`` sits at ``x_a = i_a * lam_a``. A particle
  with lattice speed ``c = 1`` travels ``lam_a`` per time step (paper, Sec. 2.2,
  stretched velocities), so ``lam_a`` is the node spacing along axis ``a``.

Workload recipes (paper Sec. 3):

* ``shear_wave_axis``   -- advected decaying shear wave, axis aligned (Sec. 3.1).
* ``shear_wave_rotated``-- the same wave rotated by pi/4, on a cubic or
  stretched lattice whose physical extent is square (Sec. 3.1).
* ``double_shear_layer``-- periodic double shear layer (Sec. 3.3).
* ``hit_field``         -- solenoidal random field with the spectrum
  E(k) ~ k^4 exp(-2 (k/k0)^2) (Sec. 3.2).
* ``channel_field``     -- laminar channel profile plus a divergence-free,
  wall-vanishing perturbation (Sec. 3.5 geometry).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 210104550


def rng(seed_offset: int = 0) -> np.random.Generator:
    """Seeded PCG64 generator: ``SEED_BASE + seed_offset``."""
    return np.random.Generator(np.random.PCG64(SEED_BASE + int(seed_offset)))


def grid_shape(n):
    """Array shape of a field on extents ``n = (n_x, n_y[, n_z])``."""
    return tuple(int(v) for v in reversed(tuple(n)))


def coords(n, lam):
    """Physical node coordinates, one array per axis, broadcast to the grid."""
    D = len(n)
    shape = grid_shape(n)
    out = []
    for a in range(D):
        idx = np.arange(n[a], dtype=np.float64) * float(lam[a])
        bshape = [1] * D
        bshape[D - 1 - a] = n[a]
        out.append(np.broadcast_to(idx.reshape(bshape), shape))
    return out


@dataclass
class Field:
    """Initial macroscopic state: ``rho`` (grid) and ``u`` ((D,) + grid)."""
    rho: np.ndarray
    u: np.ndarray
    n: tuple
    lam: tuple
    # optional measurement direction for a plane wave (diagnostic mode)
    mode_k: tuple = (0.0, 0.0, 0.0)
    mode_dir: tuple = (0.0, 0.0, 0.0)

    @property
    def D(self):
        return len(self.n)


def uniform(n, lam=None, u0=None, rho0=1.0) -> Field:
    """Uniform state: rho = rho0, u = u0 everywhere."""
    D = len(n)
    lam = tuple(lam) if lam is not None else (1.0,) * D
    u0 = tuple(u0) if u0 is not None else (0.0,) * D
    shape = grid_shape(n)
    rho = np.full(shape, float(rho0))
    u = np.stack([np.full(shape, float(u0[a])) for a in range(D)])
    return Field(rho, u, tuple(n), lam)


def shear_wave_axis(n=(64, 64), U0=0.1, A=0.01, lam=(1.0, 1.0)) -> Field:
    """Axis-aligned advected shear wave (Sec. 3.1).

    u_x = U0 (advection along the wave vector), u_y = A sin(2 pi x / L_x),
    rho = 1. The decaying component is u_y, the wave vector is along x.
    """
    nx, ny = n
    x, _ = coords(n, lam)
    Lx = nx * lam[0]
    k = 2.0 * math.pi / Lx
    shape = grid_shape(n)
    rho = np.ones(shape)
    u = np.stack([np.full(shape, float(U0)), A * np.sin(k * x)])
    return Field(rho, u, tuple(n), tuple(lam), mode_k=(k, 0.0, 0.0), mode_dir=(0.0, 1.0, 0.0))


def shear_wave_rotated(n=(64, 64), lam=(1.0, 1.0), U0=0.0, a0=1e-3) -> Field:
    """Shear wave rotated by pi/4 (Sec. 3.1), on a physically square domain.

    With nhat = (1, 1)/sqrt(2) and that = (-1, 1)/sqrt(2):
    u = U0 nhat + a0 sin(k nhat.x) that,  k = 2 pi sqrt(2) / L,
    where L = n_x lam_x = n_y lam_y is the physical side.
    """
    nx, ny = n
    Lx, Ly = nx * lam[0], ny * lam[1]
    if abs(Lx - Ly) > 1e-12:
        raise ValueError("rotated wave needs a physically square domain")
    L = Lx
    x, y = coords(n, lam)
    s2 = math.sqrt(2.0)
    nhat = (1.0 / s2, 1.0 / s2)
    that = (-1.0 / s2, 1.0 / s2)
    k = 2.0 * math.pi * s2 / L
    phase = k * (nhat[0] * x + nhat[1] * y)
    amp = a0 * np.sin(phase)
    shape = grid_shape(n)
    rho = np.ones(shape)
    u = np.stack([U0 * nhat[0] + amp * that[0], U0 * nhat[1] + amp * that[1]])
    return Field(rho, u, tuple(n), tuple(lam),
                 mode_k=(k * nhat[0], k * nhat[1], 0.0), mode_dir=(that[0], that[1], 0.0))


def double_shear_layer(n=(1024, 1024), lam=(1.0, 1.0), U=0.1, kappa=80.0, delta=0.05) -> Field:
    """Periodic double shear layer (Sec. 3.3) on the physical square L x L.

    u_x = U tanh(kappa (y/L - 1/4)) for y <= L/2, U tanh(kappa (3/4 - y/L)) above;
    u_y = delta U sin(2 pi (x/L + 1/4)); rho = 1.
    """
    nx, ny = n
    L = ny * lam[1]
    if abs(nx * lam[0] - L) > 1e-12:
        raise ValueError("double shear layer needs a physically square domain")
    x, y = coords(n, lam)
    ux = np.where(y <= L / 2, U * np.tanh(kappa * (y / L - 0.25)), U * np.tanh(kappa * (0.75 - y / L)))
    uy = delta * U * np.sin(2.0 * math.pi * (x / L + 0.25))
    shape = grid_shape(n)
    return Field(np.ones(shape), np.stack([ux, uy]), tuple(n), tuple(lam))


def hit_field(N=256, k0=4.0, urms=0.05, seed_offset=2) -> Field:
    """Solenoidal random velocity with spectrum E(k) ~ k^4 exp(-2 (k/k0)^2) (Sec. 3.2).

    Gaussian random Fourier coefficients are projected perpendicular to the
    (integer) wave vector, scaled shell by shell to the target spectrum, and
    transformed back; the result is rescaled so that
    u_rms = sqrt(<u.u>/3) equals ``urms``. rho = 1. Cubic lattice.
    """
    g = rng(seed_offset)
    kk = np.fft.fftfreq(N, d=1.0 / N)
    kz, ky, kx = np.meshgrid(kk, kk, kk, indexing="ij")
    kvec = np.stack([kx, ky, kz])
    k2 = kx * kx + ky * ky + kz * kz
    kmag = np.sqrt(k2)
    coef = g.standard_normal((3, N, N, N)) + 1j * g.standard_normal((3, N, N, N))
    k2s = np.where(k2 == 0, 1.0, k2)
    kdot = (kvec * coef).sum(axis=0) / k2s
    coef = coef - kvec * kdot
    shell = np.rint(kmag).astype(np.int64)
    spec = np.where(kmag > 0, kmag ** 4 * np.exp(-2.0 * (kmag / k0) ** 2), 0.0)
    # normalise each integer shell to carry energy proportional to E(k)
    energy = (np.abs(coef) ** 2).sum(axis=0)
    shell_e = np.bincount(shell.ravel(), weights=energy.ravel())
    kint = np.arange(shell_e.size, dtype=np.float64)
    target = np.where(kint > 0, kint ** 4 * np.exp(-2.0 * (kint / k0) ** 2), 0.0)
    scale = np.where(shell_e > 0, np.sqrt(target / np.where(shell_e > 0, shell_e, 1.0)), 0.0)
    coef = coef * scale[shell]
    coef[:, 0, 0, 0] = 0.0
    del spec
    u = np.real(np.fft.ifftn(coef, axes=(1, 2, 3)))
    rms = math.sqrt((u * u).sum(axis=0).mean() / 3.0)
    u *= urms / rms
    return Field(np.ones((N, N, N)), u, (N, N, N), (1.0, 1.0, 1.0))


def channel_field(n=(384, 192, 192), lam=(2.0, 1.0, 1.0), u0=0.1, amp=0.1, nmodes=24,
                  seed_offset=3) -> Field:
    """Channel flow start (Sec. 3.5 geometry): walls at y = -1/2 and n_y - 1/2 (node units).

    u_x = u0 (1 - eta^2) with eta = (y - H)/H, y the physical distance from the
    lower wall, H the half width; plus u' = curl(W(eta) A), where A is a smooth
    seeded random vector potential (periodic in x and z) and W = (1 - eta^2)^2
    makes u' and its normal derivative of W vanish at the walls. u' is scaled
    to ``amp * u0`` rms. rho = 1.
    """
    nx, ny, nz = n
    g = rng(seed_offset)
    Lx, Lz = nx * lam[0], nz * lam[2]
    H = 0.5 * ny * lam[1]
    shape = grid_shape(n)
    xi = np.arange(nx) * lam[0]
    yi = (np.arange(ny) + 0.5) * lam[1]
    zi = np.arange(nz) * lam[2]
    Z, Y, X = np.meshgrid(zi, yi, xi, indexing="ij")
    eta = (Y - H) / H
    W = (1.0 - eta ** 2) ** 2
    dW = -4.0 * eta * (1.0 - eta ** 2) / H  # dW/dy
    # A_c = sum_m a_mc cos(kx x + ky y + kz z + phi_mc); derivatives analytic.
    A = np.zeros((3,) + shape)
    dA = np.zeros((3, 3) + shape)  # dA[c, d] = d A_c / d x_d
    for _ in range(nmodes):
        mx = int(g.integers(1, 5))
        mz = int(g.integers(1, 5))
        kx = 2.0 * math.pi * mx / Lx * (1 if g.random() < 0.5 else -1)
        kz = 2.0 * math.pi * mz / Lz * (1 if g.random() < 0.5 else -1)
        ky = math.pi * float(g.uniform(0.5, 3.0)) / H
        kv = (kx, ky, kz)
        ph = g.uniform(0.0, 2.0 * math.pi, size=3)
        a = g.standard_normal(3)
        for c in range(3):
            arg = kx * X + ky * Y + kz * Z + ph[c]
            A[c] += a[c] * np.cos(arg)
            s = -a[c] * np.sin(arg)
            for d in range(3):
                dA[c, d] += kv[d] * s
    # B = W A ; dB_c/dx_d = W dA_c/dx_d + delta_{d,y} dW A_c
    dB = W * dA
    dB[:, 1] += dW * A
    ux = dB[2, 1] - dB[1, 2]
    uy = dB[0, 2] - dB[2, 0]
    uz = dB[1, 0] - dB[0, 1]
    up = np.stack([ux, uy, uz])
    rms = math.sqrt((up * up).sum(axis=0).mean())
    up *= amp * u0 / rms
    base = u0 * (1.0 - eta ** 2)
    u = up.copy()
    u[0] += base
    return Field(np.ones(shape), u, tuple(n), tuple(lam))
