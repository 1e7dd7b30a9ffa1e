"""Seeded synthetic fields shaped like particle-in-cell simulation output.

Every generator returns float32 values at the cell centres (i + 1/2) of the
local volume plus `guard` layers on each side, indexed [z][y][x] or
[z][y][x][c].  Analytic fields extend naturally into the guard layers; i.i.d.
noise is drawn for guard cells too.  Large fields are produced slab by slab
along z to bound host memory.
"""

from __future__ import annotations

import math

import numpy as np


def _centres(n: int, guard: int) -> np.ndarray:
    return np.arange(-guard, n + guard, dtype=np.float64) + 0.5


def gaussian_blobs(rng: np.random.Generator, dims, guard: int = 0, n_blobs: int = 8,
                   sigma=(4.0, 12.0), amplitude=(0.2, 1.0), noise: float = 0.01,
                   scale: float = 1.0) -> np.ndarray:
    """Sum of Gaussian blobs plus uniform noise in [0, noise).

    Centres are uniform in the volume, widths uniform in `sigma` (multiplied by
    `scale`, for volumes larger or smaller than 64 cells), amplitudes uniform in
    `amplitude`.
    """
    nx, ny, nz = dims
    c = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([nx, ny, nz], dtype=np.float64)
    s = rng.uniform(sigma[0], sigma[1], size=n_blobs) * scale
    a = rng.uniform(amplitude[0], amplitude[1], size=n_blobs)
    xs, ys, zs = _centres(nx, guard), _centres(ny, guard), _centres(nz, guard)
    out = np.zeros((zs.size, ys.size, xs.size), dtype=np.float64)
    for b in range(n_blobs):
        k = -0.5 / (s[b] * s[b])
        gx = np.exp(k * (xs - c[b, 0]) ** 2)
        gy = np.exp(k * (ys - c[b, 1]) ** 2)
        gz = np.exp(k * (zs - c[b, 2]) ** 2)
        out += a[b] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    if noise:
        out += rng.uniform(0.0, noise, size=out.shape)
    return out.astype(np.float32)


def lognormal_wake(rng: np.random.Generator, dims, guard: int = 1) -> np.ndarray:
    """Density: lognormal(0,1) i.i.d. background times a cylindrical wake modulation.

    m = 1 - 0.8 exp(-r^2 / 2R^2) (1 + cos(2 pi (y - y0) / lambda)) / 2, with r
    the distance from the y-axis line through the volume centre.
    """
    nx, ny, nz = dims
    R = rng.uniform(16.0, 48.0)
    lam = rng.uniform(32.0, 96.0)
    y0 = rng.uniform(0.0, ny)
    xs, ys, zs = _centres(nx, guard), _centres(ny, guard), _centres(nz, guard)
    cx, cz = nx / 2.0, nz / 2.0
    out = np.empty((zs.size, ys.size, xs.size), dtype=np.float32)
    wave = 0.5 * (1.0 + np.cos(2.0 * math.pi * (ys - y0) / lam))
    for iz, z in enumerate(zs):
        r2 = (xs - cx) ** 2 + (z - cz) ** 2
        m = 1.0 - 0.8 * np.exp(-r2 / (2.0 * R * R))[None, :] * wave[:, None]
        bg = np.exp(rng.standard_normal(size=(ys.size, xs.size)))
        out[iz] = (bg * m).astype(np.float32)
    return out


def divergence_free_sinusoids(rng: np.random.Generator, dims, guard: int = 1, n_modes: int = 4,
                              wavelength=(16.0, 128.0), amplitude=(0.05, 0.25)) -> np.ndarray:
    """Vector field sum_m A_m e_m sin(k_m . x + phi_m) with e_m orthogonal to k_m.

    Each mode is exactly divergence-free; |k_m| = 2 pi / lambda_m.
    """
    nx, ny, nz = dims
    khat = rng.standard_normal(size=(n_modes, 3))
    khat /= np.linalg.norm(khat, axis=1, keepdims=True)
    lam = rng.uniform(wavelength[0], wavelength[1], size=n_modes)
    k = khat * (2.0 * math.pi / lam)[:, None]
    r = rng.standard_normal(size=(n_modes, 3))
    e = r - (r * khat).sum(axis=1, keepdims=True) * khat
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    A = rng.uniform(amplitude[0], amplitude[1], size=n_modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    xs, ys, zs = _centres(nx, guard), _centres(ny, guard), _centres(nz, guard)
    out = np.zeros((zs.size, ys.size, xs.size, 3), dtype=np.float32)
    for iz, z in enumerate(zs):
        acc = np.zeros((ys.size, xs.size, 3), dtype=np.float64)
        for m in range(n_modes):
            ph = k[m, 0] * xs[None, :] + k[m, 1] * ys[:, None] + (k[m, 2] * z + phi[m])
            acc += (A[m] * np.sin(ph))[..., None] * e[m][None, None, :]
        out[iz] = acc.astype(np.float32)
    return out


def ramp(dims, guard: int, alpha: float, beta: float, axis: int = 0) -> np.ndarray:
    """Affine field alpha * (i + 1/2) + beta along one axis, constant in the others."""
    nx, ny, nz = dims
    cs = [_centres(nx, guard), _centres(ny, guard), _centres(nz, guard)]
    shape = (cs[2].size, cs[1].size, cs[0].size)
    line = alpha * cs[axis] + beta
    if axis == 0:
        v = np.broadcast_to(line[None, None, :], shape)
    elif axis == 1:
        v = np.broadcast_to(line[None, :, None], shape)
    else:
        v = np.broadcast_to(line[:, None, None], shape)
    return np.ascontiguousarray(v, dtype=np.float32)


def constant(dims, guard: int, value, f_dim: int = 1) -> np.ndarray:
    """Homogeneous field (the analytic example source that is 42 everywhere is one)."""
    nx, ny, nz = dims
    shape = (nz + 2 * guard, ny + 2 * guard, nx + 2 * guard)
    if f_dim == 1:
        return np.full(shape, value, dtype=np.float32)
    v = np.asarray(value, dtype=np.float32).reshape(1, 1, 1, f_dim)
    return np.ascontiguousarray(np.broadcast_to(v, shape + (f_dim,)))


def uniform_random(rng: np.random.Generator, dims, guard: int, f_dim: int = 1,
                   low: float = 0.0, high: float = 1.0) -> np.ndarray:
    nx, ny, nz = dims
    shape = (nz + 2 * guard, ny + 2 * guard, nx + 2 * guard) + ((f_dim,) if f_dim > 1 else ())
    return rng.uniform(low, high, size=shape).astype(np.float32)
