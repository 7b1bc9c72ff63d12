"""Air above the sea surface (Section 3.3): ghost planes filled each half
step.  Test infrastructure, like the rest of `oracle/`.

Reading used here (the paper gives the wavenumber relations, not their
discrete placement):
* The sea surface is the first interior z node k_s (z = x3[0]); no cell
  above it is updated, and there is no absorbing layer on the top face.
* In the air the conductivity is zero and there is no source, so H is curl
  and divergence free: H = grad(psi) with Laplace(psi) = 0.  A horizontal
  Fourier mode exp(i (kx x + ky y)) of psi that vanishes far above the
  surface (z is positive down) goes as exp(|kappa| z), so every component
  decays by exp(-|kappa| h) at height h, and the horizontal components
  follow from the vertical one: Hx^ = (i kx/|kappa|) Hz^,
  Hy^ = (i ky/|kappa|) Hz^ (the paper's relation with its sign correction).
* E is extrapolated with Laplace(E) = 0 in the air: each mode of E1, E2
  decays by exp(-|kappa| h).
* Ghost planes: E1, E2 at the r - 1 integer nodes above k_s (the D+ taps
  of the H update at the half node just below the surface reach that far);
  H1, H2 at the r half nodes above k_s (the D- taps of the E update at k_s),
  from H3 at k_s.  H1 sits half a cell before H3 in x, H2 half a cell
  before it in y: their spectra carry exp(-i kx dx/2), exp(-i ky dy/2).
* The transform is a plain 2-D DFT over the whole padded x-y plane, which
  needs uniform x and y spacing; the kappa = 0 mode of the H relation is 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class AirOps:
    ks: int              # surface node (first updated z plane)
    kx: np.ndarray       # [n2][n1] horizontal wavenumbers of the DFT bins
    ky: np.ndarray
    kappa: np.ndarray    # |(kx, ky)|
    dx: float
    dy: float
    hE: list             # heights of the E ghost nodes ks - m, m = 1 .. r - 1
    hH: list             # heights of the H ghost half nodes ks - m, m = 1 .. r


def uniform_spacing(x: np.ndarray) -> float:
    d = np.diff(x)
    if not np.allclose(d, d[0], rtol=1e-9, atol=0.0):
        raise ValueError("the air boundary needs uniform x and y spacing")
    return float(d[0])


def make_ops(axes, ks: int, r: int) -> AirOps:
    x, y, z = axes
    dx, dy = uniform_spacing(x), uniform_spacing(y)
    if ks - r < 0:
        raise ValueError("not enough planes above the surface for the ghost nodes")
    kx1 = 2.0 * np.pi * np.fft.fftfreq(len(x), dx)
    ky1 = 2.0 * np.pi * np.fft.fftfreq(len(y), dy)
    ky, kx = np.meshgrid(ky1, kx1, indexing="ij")
    kappa = np.sqrt(kx * kx + ky * ky)
    hE = [z[ks] - z[ks - m] for m in range(1, r)]
    hH = [z[ks] - 0.5 * (z[ks - m] + z[ks - m + 1]) for m in range(1, r + 1)]
    return AirOps(ks, kx, ky, kappa, dx, dy, hE, hH)


def fill_E(E1: np.ndarray, E2: np.ndarray, ops: AirOps) -> None:
    """E1, E2 [n3][n2][n1]: overwrite the ghost planes above ops.ks."""
    for F in (E1, E2):
        S = np.fft.fft2(F[ops.ks])
        for m, h in enumerate(ops.hE, start=1):
            F[ops.ks - m] = np.real(np.fft.ifft2(S * np.exp(-ops.kappa * h)))


def fill_H(H1: np.ndarray, H2: np.ndarray, H3: np.ndarray, ops: AirOps) -> None:
    """H1, H2 ghost half planes above ops.ks from H3 at ops.ks."""
    S = np.fft.fft2(H3[ops.ks])
    live = ops.kappa > 0.0
    kap = np.where(live, ops.kappa, 1.0)
    rx = np.where(live, 1j * ops.kx / kap, 0.0) * np.exp(-0.5j * ops.kx * ops.dx)
    ry = np.where(live, 1j * ops.ky / kap, 0.0) * np.exp(-0.5j * ops.ky * ops.dy)
    for m, h in enumerate(ops.hH, start=1):
        d = S * np.exp(-ops.kappa * h)
        H1[ops.ks - m] = np.real(np.fft.ifft2(d * rx))
        H2[ops.ks - m] = np.real(np.fft.ifft2(d * ry))
