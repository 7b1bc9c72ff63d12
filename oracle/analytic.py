"""Closed-form whole-space fields of an electric dipole (oracle pin).

The diffusive Maxwell equations of Section 2.1 with M = 0 and the exp(-i w t)
convention, curl E = i w mu H and curl H = sigma E + J, give for a homogeneous
conductivity sigma and a point dipole J = p d delta(x - x_s)

    E = (1/sigma) (k^2 + grad div) (p d g),   H = curl (p d g),
    g = exp(i k r)/(4 pi r),  k = sqrt(i w mu sigma), Im k > 0.

Written out with X = x - x_s, r = |X|:
    E_i = p exp(ikr)/(4 pi sigma r^3) [ d_i (k^2 r^2 + i k r - 1)
                                        + X_i (X.d)/r^2 (3 - 3 i k r - k^2 r^2) ]
    H   = p (i k r - 1) exp(ikr)/(4 pi r^3) (X x d)
The static limit of the inline x-component is p/(2 pi sigma r^3).
"""
from __future__ import annotations

import numpy as np

MU0 = 4.0e-7 * np.pi


def wavenumber(freq: float, sigma: float) -> complex:
    k = np.sqrt(1j * 2.0 * np.pi * freq * MU0 * sigma)
    return k if k.imag > 0 else -k


def dipole_fields(src, direction, rec, freq: float, sigma: float, moment: float = 1.0):
    """Returns (E[nrec][3], H[nrec][3]) complex, per `moment` A.m."""
    k = wavenumber(freq, sigma)
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    X = np.atleast_2d(np.asarray(rec, dtype=np.float64)) - np.asarray(src, dtype=np.float64)
    r = np.linalg.norm(X, axis=1)
    ikr = 1j * k * r
    ph = np.exp(ikr)
    Xd = X @ d
    a = (k * k * r * r + ikr - 1.0)
    b = (3.0 - 3.0 * ikr - k * k * r * r) * Xd / r ** 2
    pref = moment * ph / (4.0 * np.pi * sigma * r ** 3)
    E = pref[:, None] * (a[:, None] * d[None, :] + b[:, None] * X)
    H = (moment * (ikr - 1.0) * ph / (4.0 * np.pi * r ** 3))[:, None] * np.cross(X, d[None, :])
    return E, H
