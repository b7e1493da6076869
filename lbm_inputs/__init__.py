"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  Holds no arithmetic of the method itself: only velocity fields, force
fields and wall masks of the shapes the paper's workloads and the benchmark
configurations use, as NumPy float64 arrays in the (3, nz, ny, nx) / (nz, ny, nx)
layout (x fastest).
"""
import math

import numpy as np


def taylor_green(n, u0=0.02, nz=None, ny=None):
    """Taylor-Green vortex on node coordinates (i, j, k), k0 = 2 pi / n:
    u = u0 sin(k0 x) cos(k0 y) cos(k0 z), v = -u0 cos(k0 x) sin(k0 y) cos(k0 z), w = 0."""
    nz = n if nz is None else nz
    ny = n if ny is None else ny
    k0 = 2 * math.pi / n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(n), indexing="ij")
    u = np.zeros((3, nz, ny, n))
    u[0] = u0 * np.sin(k0 * x) * np.cos(k0 * y) * np.cos(k0 * z)
    u[1] = -u0 * np.cos(k0 * x) * np.sin(k0 * y) * np.cos(k0 * z)
    return u


def random_spectrum_velocity(n, seed, shells=(1, 8), slope=-5.0 / 3.0, rms=0.03):
    """Solenoidal random-phase field on an n^3 periodic box: integer wavevectors
    with shell s = round(|k|) in [shells], complex Gaussian coefficients scaled
    to sqrt(E(s)/n_s) with E ~ s^slope, projected on k-perpendicular, real part
    of the inverse FFT, rescaled to per-component rms `rms`."""
    rng = np.random.default_rng(seed)
    k = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    kk = np.sqrt(kx**2 + ky**2 + kz**2)
    shell = np.rint(kk).astype(int)
    lo, hi = shells
    active = (shell >= lo) & (shell <= hi)
    counts = np.bincount(shell[active].ravel(), minlength=hi + 1)
    amp = np.zeros_like(kk)
    s_act = shell[active]
    amp[active] = np.sqrt(s_act.astype(float) ** slope / counts[s_act])
    coef = (rng.standard_normal((3,) + kk.shape) + 1j * rng.standard_normal((3,) + kk.shape)) * amp
    K = np.stack([kx, ky, kz])
    kk_safe = np.where(kk > 0, kk, 1.0)
    dot = (coef * K).sum(axis=0) / kk_safe**2
    coef = coef - K * dot
    u = np.real(np.fft.ifftn(coef, axes=(1, 2, 3)))
    cur = math.sqrt((u**2).sum(axis=0).mean() / 3.0)
    return u * (rms / cur)


def kolmogorov_force(n, amplitude=1e-6, waves=4, nz=None, ny=None, nx=None):
    """F_x = amplitude sin(2 pi waves y / n), F_y = F_z = 0."""
    nz = n if nz is None else nz
    ny = n if ny is None else ny
    nx = n if nx is None else nx
    y = np.arange(ny)
    F = np.zeros((3, nz, ny, nx))
    F[0] = amplitude * np.sin(2 * math.pi * waves * y / n)[None, :, None]
    return F


def gaussian_force(shape, sigma, seed):
    """i.i.d. N(0, sigma^2) per node and component, shape (3, nz, ny, nx)."""
    return np.random.default_rng(seed).normal(0.0, sigma, (3,) + tuple(shape))


def duct_mask(nx, ny, nz):
    """Square duct along x: solid planes y in {0, ny-1} and z in {0, nz-1}."""
    solid = np.zeros((nz, ny, nx), dtype=bool)
    solid[0] = solid[-1] = True
    solid[:, 0] = solid[:, -1] = True
    return solid


def channel_mask(nx, ny, nz):
    """Plates normal to z: solid planes z in {0, nz-1}."""
    solid = np.zeros((nz, ny, nx), dtype=bool)
    solid[0] = solid[-1] = True
    return solid


def random_state_perturbation(shape, q, scale, seed):
    """Small seeded perturbation for populations, shape (q, nz, ny, nx)."""
    return np.random.default_rng(seed).normal(0.0, scale, (q,) + tuple(shape))
