"""Seeded synthetic initial conditions (host, numpy).

This module only lays out initial density fields of the shapes the paper's
validation cases use (Sec. 3): a liquid droplet in its vapour, optionally
with a mode-2 shape perturbation (Sec. 3.1, 3.2), and a radial density wave
in a single phase (Sec. 3.3).  It holds none of the method's arithmetic:
coexistence densities, temperatures and relaxation times are passed in by
the caller.  Both the HIP path and the CPU oracle are fed from here.

Arrays are float64 of shape (nr, nz): row j is r = j + 1/2, column k is z = k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _noise(shape, amplitude: float, seed: int) -> np.ndarray:
    """Relative density noise xi ~ U[-amplitude, amplitude] from default_rng(seed)."""
    if amplitude == 0.0:
        return np.zeros(shape)
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, size=shape)


def droplet(nz: int, nr: int, rho_v: float, rho_l: float, radius: float,
            zc: float | None = None, width: float = 5.0, eps: float = 0.0,
            noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Axisymmetric droplet centred on the axis at z = zc.

    rho(d) = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (d - R(theta)) / width),
    d the distance from (zc, 0) in the (z, r) plane, R(theta) = R (1 + eps P2(cos theta)),
    cos theta = (z - zc)/d, P2(x) = (3x^2 - 1)/2; then rho <- rho (1 + xi).
    """
    if zc is None:
        zc = nz / 2.0
    z = np.arange(nz, dtype=np.float64) - zc
    r = np.arange(nr, dtype=np.float64) + 0.5
    Z, Rr = np.meshgrid(z, r)
    d = np.sqrt(Z * Z + Rr * Rr)
    cos = Z / d
    p2 = 0.5 * (3.0 * cos * cos - 1.0)
    rad = radius * (1.0 + eps * p2)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (d - rad) / width)
    return np.ascontiguousarray(rho * (1.0 + _noise(rho.shape, noise, seed)))


def ellipsoid(nz: int, nr: int, rho_v: float, rho_l: float, r_a: float, r_z: float,
              zc: float | None = None, width: float = 5.0, noise: float = 0.0,
              seed: int = 0) -> np.ndarray:
    """Axisymmetric ellipsoidal drop (r/r_a)^2 + ((z - zc)/r_z)^2 = 1 on the axis (Sec. 3.2):
    the droplet profile with R(theta) the ellipse's distance from its centre along the ray,
    1 / R(theta)^2 = (sin theta / r_a)^2 + (cos theta / r_z)^2; then rho <- rho (1 + xi)."""
    if zc is None:
        zc = nz / 2.0
    z = np.arange(nz, dtype=np.float64) - zc
    r = np.arange(nr, dtype=np.float64) + 0.5
    Z, Rr = np.meshgrid(z, r)
    d = np.sqrt(Z * Z + Rr * Rr)
    rad = 1.0 / np.sqrt((Rr / (d * r_a)) ** 2 + (Z / (d * r_z)) ** 2)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (d - rad) / width)
    return np.ascontiguousarray(rho * (1.0 + _noise(rho.shape, noise, seed)))


def radial_wave(nz: int, nr: int, rho_g: float, amplitude: float = 1e-2,
                wavelength: float = 256.0, noise: float = 0.0, seed: int = 0) -> np.ndarray:
    """Single-phase field rho_g (1 + amplitude cos(2 pi r / wavelength)) (1 + xi)."""
    r = np.arange(nr, dtype=np.float64) + 0.5
    prof = rho_g * (1.0 + amplitude * np.cos(2.0 * np.pi * r / wavelength))
    rho = np.repeat(prof[:, None], nz, axis=1)
    return np.ascontiguousarray(rho * (1.0 + _noise(rho.shape, noise, seed)))


def gaussian_pulse(nz: int, nr: int, rho0: float, amplitude: float, r0: float,
                   width: float) -> np.ndarray:
    """rho0 + amplitude exp(-((r - r0)/width)^2), uniform in z (a ring-shaped disturbance)."""
    r = np.arange(nr, dtype=np.float64) + 0.5
    prof = rho0 + amplitude * np.exp(-((r - r0) / width) ** 2)
    return np.ascontiguousarray(np.repeat(prof[:, None], nz, axis=1))


def slab(nz: int, nr: int, rho_v: float, rho_l: float, z0: float, z1: float,
         width: float = 5.0) -> np.ndarray:
    """Planar liquid layer between z0 and z1 (uniform in r), tanh interfaces of the given
    width: rho = rho_v + (rho_l - rho_v)/2 [tanh(2 (z - z0)/width) - tanh(2 (z - z1)/width)]."""
    z = np.arange(nz, dtype=np.float64)
    prof = rho_v + 0.5 * (rho_l - rho_v) * (np.tanh(2.0 * (z - z0) / width) - np.tanh(2.0 * (z - z1) / width))
    return np.ascontiguousarray(np.repeat(prof[None, :], nr, axis=0))


@dataclass
class Instance:
    """One member of a batched droplet ensemble."""
    index: int
    nz: int
    nr: int
    t_reduced: float   # T / T_c
    tau: float
    radius: float
    eps: float         # P2 shape amplitude (0 for a static droplet)
    noise_seed: int


def ensemble(n: int = 256, seed: int = 151201977, nr_lo: int = 32, nr_hi: int = 256,
             t_lo: float = 0.55, t_hi: float = 0.9, tau_lo: float = 0.6, tau_hi: float = 1.2,
             eps: float = 0.05) -> list[Instance]:
    """Uneven droplet ensemble: nr ~ U{nr_lo..nr_hi}, nz = 2 nr, T/T_c ~ U[t_lo, t_hi],
    tau ~ U[tau_lo, tau_hi], R = 0.3 nr; even members are static, odd members carry a
    P2 perturbation of amplitude eps; member k draws its noise from seed + 1 + k."""
    rng = np.random.default_rng(seed)
    nr = rng.integers(nr_lo, nr_hi + 1, size=n)
    tr = rng.uniform(t_lo, t_hi, size=n)
    tau = rng.uniform(tau_lo, tau_hi, size=n)
    out = []
    for k in range(n):
        out.append(Instance(index=k, nz=int(2 * nr[k]), nr=int(nr[k]), t_reduced=float(tr[k]),
                            tau=float(tau[k]), radius=0.3 * float(nr[k]),
                            eps=0.0 if k % 2 == 0 else eps, noise_seed=seed + 1 + k))
    return out
