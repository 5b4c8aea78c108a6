"""Seeded band tables and angular quadratures (inputs of the method).

The quadratures are the discrete-ordinates sets (s_i, w_i) the solver takes as
input; the band tables are synthetic stand-ins for ab-initio (C, v, tau) data.
"""
from __future__ import annotations

import numpy as np

H_PLANCK = 6.62607015e-34
K_BOLTZ = 1.380649e-23


def inplane_quadrature(D):
    """D in-plane directions phi_j = (j + 1/2) 2 pi / D, s_z = 0, equal weights 2 pi / D.
    The half offset keeps every direction off the axes."""
    phi = (np.arange(D) + 0.5) * 2.0 * np.pi / D
    s = np.stack([np.cos(phi), np.sin(phi), np.zeros(D)], axis=1)
    w = np.full(D, 2.0 * np.pi / D)
    return s, w


def gl_azimuth_quadrature(n_polar, n_azim):
    """Gauss-Legendre in mu = cos(polar angle about z) times n_azim uniform
    half-offset azimuths; weights sum to 4 pi."""
    mu, wm = np.polynomial.legendre.leggauss(n_polar)
    phi = (np.arange(n_azim) + 0.5) * 2.0 * np.pi / n_azim
    M, P = np.meshgrid(mu, phi, indexing="ij")
    WM = np.repeat(wm[:, None], n_azim, axis=1)
    st = np.sqrt(1.0 - M ** 2)
    s = np.stack([st * np.cos(P), st * np.sin(P), M], axis=-1).reshape(-1, 3)
    w = (WM * 2.0 * np.pi / n_azim).ravel()
    return s, w


def bose_einstein_bands(rng, B, tau_lo=1e-12, tau_hi=5e-9, v_max=8000.0, n_at=5e28, T=300.0):
    """Synthetic non-gray band table:
      frequencies linear in 0.5-15 THz, heat capacity from the Bose-Einstein
      mode heat capacity at T with a Debye-shell mode density,
      v_b = v_max cos(pi k_b / 2) with k_b = (b + 1/2)/B,
      tau log-uniform in [tau_lo, tau_hi] from rng."""
    f = np.linspace(0.5e12, 15e12, B)
    x = H_PLANCK * f / (K_BOLTZ * T)
    b = np.arange(B)
    g = 3.0 * n_at * ((b + 1.0) ** 3 - b ** 3) / B ** 3
    C = g * K_BOLTZ * x ** 2 * np.exp(x) / np.expm1(x) ** 2
    k = (b + 0.5) / B
    v = v_max * np.cos(np.pi * k / 2.0)
    tau = np.exp(rng.uniform(np.log(tau_lo), np.log(tau_hi), B))
    return C, v, tau


def mean_free_path(C, v, tau):
    """Heat-capacity-and-velocity weighted mean free path sum(C v^2 tau)/sum(C v)."""
    return float(np.sum(C * v * v * tau) / np.sum(C * v))
