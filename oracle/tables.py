"""Oracle set-up: padded grid, FD tables, time step, CPML, wavelet, DFT
phases and interpolation stencils.  Plain FP64 NumPy, one quantity per
function, each citing the passage it follows.

Index conventions (shared reading of the paper's staggered grid, Section 3.1):
  arrays are [n3pad][n2pad][n1pad], x fastest (Section 3.8);
  E1 at (i+1/2, j, k), E2 at (i, j+1/2, k), E3 at (i, j, k+1/2),
  H1 at (i, j+1/2, k+1/2), H2 at (i+1/2, j, k+1/2), H3 at (i+1/2, j+1/2, k);
  array index m on a half-staggered axis means position m+1/2.
  D- at integer node i uses half nodes i-r .. i+r-1 (eq. HFD2);
  D+ at half node i+1/2 uses integer nodes i-r+1 .. i+r (eq. HFD1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .weights import derivative_weights, lagrange_weights

MU0 = 4.0e-7 * np.pi

# staggering flags (half along x, y, z) of the six channels Ex..Hz
STAGGER = ((1, 0, 0), (0, 1, 0), (0, 0, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0))


# ------------------------------------------------------------------ padding
def pad_axis(x: np.ndarray, nbe: int) -> np.ndarray:
    """Extend the node coordinates by nbe nodes on each side with the end
    interval (Section 3.4 gives only the layer counts; constant spacing equal
    to the adjacent end interval is the reading used)."""
    x = np.asarray(x, dtype=np.float64)
    lo = x[0] - (x[1] - x[0]) * np.arange(nbe, 0, -1)
    hi = x[-1] + (x[-1] - x[-2]) * np.arange(1, nbe + 1)
    return np.concatenate([lo, x, hi])


def half_nodes(xp: np.ndarray) -> np.ndarray:
    """Half-node positions x_{i+1/2} = (x_i + x_{i+1})/2, i = 0..n-2
    (midpoints: the paper does not state them on a non-uniform grid)."""
    return 0.5 * (xp[:-1] + xp[1:])


def pad_model(rho: np.ndarray, nbe: int) -> np.ndarray:
    """Replicate the nearest interior value into the padding layers
    (the model extension of Section 3.4 / Algorithm 1)."""
    return np.pad(np.asarray(rho, dtype=np.float64), nbe, mode="edge")


# ------------------------------------------------------------- FD tables
def fd_tables(xp: np.ndarray, r: int):
    """c_minus[i][0..2r-1] (D- at integer node i over half nodes i-r..i+r-1)
    and c_plus[i][0..2r-1] (D+ at half node i+1/2 over integer nodes
    i-r+1..i+r), eqs. HFD1/HFD2 with coefficients from the derivative row of
    the inverse Vandermonde matrix.  Rows outside [r, n-1-r] stay zero."""
    n = len(xp)
    xh = half_nodes(xp)
    cm = np.zeros((n, 2 * r))
    cp = np.zeros((n, 2 * r))
    for i in range(r, n - r):
        cm[i] = derivative_weights(xp[i], xh[i - r:i + r])
        cp[i] = derivative_weights(xh[i], xp[i - r + 1:i + r + 1])
    return cm, cp


# --------------------------------------------------------------- time step
def velocity_max(rhos, omega0: float) -> float:
    """v = 1/sqrt(mu eps) with eps = 1/(2 omega0 rho) (Section 2.2)."""
    rmax = max(float(np.max(a)) for a in rhos)
    return float(np.sqrt(2.0 * omega0 * rmax / MU0))


def time_step(tables, rhos, omega0: float, cfl: float = 0.99) -> float:
    """dt = cfl/eta, eta = 1/2 v_max sqrt(Dx^2 + Dy^2 + Dz^2), D_d = max over
    the axis and both staggerings of sum |c| (Section 3.2)."""
    dmax = []
    for cm, cp in tables:
        dmax.append(max(np.abs(cm).sum(axis=1).max(), np.abs(cp).sum(axis=1).max()))
    eta = 0.5 * velocity_max(rhos, omega0) * np.sqrt(np.sum(np.square(dmax)))
    return cfl / eta


# ------------------------------------------------------------------- CPML
@dataclass
class CpmlParams:
    npow: float = 2.0
    R: float = 1e-5
    alpha_max: float = 0.0     # filled with pi * f_peak when 0


def cpml_axis(xp: np.ndarray, nb: int, dt: float, v_lo: float, v_hi: float,
              alpha_max: float, npow: float = 2.0, R: float = 1e-5):
    """CPML coefficients (Section 3.4): psi^{n+1} = b psi^n + a d^{n+1/2},
    b = exp(-(d/kappa + alpha) dt), a = d (b - 1)/(kappa (d + kappa alpha)),
    kappa = 1.  Profile d = d0 (l/L)^N, alpha = alpha_max (1 - l/L),
    d0 = -(N+1) v ln R/(2L), l the depth into the layer from its inner face.
    Returns (a_int, b_int, a_half, b_half), each of length n; entries outside
    the slabs (index >= nb and <= n-1-nb) are zero."""
    n = len(xp)
    xh = np.concatenate([half_nodes(xp), [np.inf]])
    out = []
    for pos in (xp, xh):
        a = np.zeros(n)
        b = np.zeros(n)
        if nb > 0:
            L_lo = xp[nb] - xp[0]
            L_hi = xp[n - 1] - xp[n - 1 - nb]
            for i in range(n):
                if i < nb:
                    ell, L, v = (xp[nb] - pos[i]) / L_lo, L_lo, v_lo
                elif i > n - 1 - nb:
                    ell, L, v = (pos[i] - xp[n - 1 - nb]) / L_hi, L_hi, v_hi
                else:
                    continue
                if not np.isfinite(ell) or ell <= 0.0:
                    continue
                d0 = -(npow + 1.0) * v * np.log(R) / (2.0 * L)
                d = d0 * ell ** npow
                alpha = alpha_max * (1.0 - ell)
                b[i] = np.exp(-(d + alpha) * dt)
                a[i] = d * (b[i] - 1.0) / (d + alpha)
        out += [a, b]
    return tuple(out)


def slab_velocities(rhos_pad, axis: int, nb: int, omega0: float):
    """Max velocity in the low and high CPML slab of one axis (all three
    resistivity components).  Arrays are [z][y][x]: axis 0 = x -> array axis 2."""
    ax = 2 - axis
    n = rhos_pad[0].shape[ax]
    if nb == 0:
        return 0.0, 0.0
    lo = max(float(np.take(a, np.arange(nb), axis=ax).max()) for a in rhos_pad)
    hi = max(float(np.take(a, np.arange(n - nb, n), axis=ax).max()) for a in rhos_pad)
    v = lambda rho: float(np.sqrt(2.0 * omega0 * rho / MU0))
    return v(lo), v(hi)


# ---------------------------------------------------------- source wavelet
def peak_frequency(freqs, f0: float, fpeak: float = 0.0) -> float:
    """Wavelet peak frequency: the paper normalises the source out of the
    Green's function (Section 2.2) and leaves the wavelet free; the reading
    is f_p = 2 sqrt(f_max f0) unless given."""
    return fpeak if fpeak > 0.0 else 2.0 * np.sqrt(np.max(freqs) * f0)


def wavelet(nt: int, dt: float, fp: float) -> np.ndarray:
    """s_n = s((n+1/2) dt), s(t) = -((t-t0)/tau) exp(-((t-t0)/tau)^2),
    tau = 1/(pi f_p), t0 = 4 tau; J^{n+1/2} is sampled at half steps."""
    tau = 1.0 / (np.pi * fp)
    t = (np.arange(nt) + 0.5) * dt
    u = (t - 4.0 * tau) / tau
    return -u * np.exp(-u * u)


def omega_prime(freqs, omega0: float) -> np.ndarray:
    """omega' = (1 + i) sqrt(omega omega0)  (eq. correspondence)."""
    w = 2.0 * np.pi * np.asarray(freqs, dtype=np.float64)
    return (1.0 + 1.0j) * np.sqrt(w * omega0)


def auto_nt(freqs, f0: float, dt: float, fp: float) -> int:
    """Fixed step count replacing the paper's convergence monitor
    (Section 3.5): wavelet duration 7 tau plus the time for the slowest
    DFT kernel exp(i omega' t) to decay by 1e-6, rounded up to 100 steps."""
    tau = 1.0 / (np.pi * fp)
    decay = np.min(np.imag(omega_prime(freqs, 2.0 * np.pi * f0)))
    T = 7.0 * tau + np.log(1e6) / decay
    return int(np.ceil(T / dt / 100.0) * 100)


def dft_phases(freqs, omega0: float, dt: float, nt: int):
    """exp(i omega' t) at the stamps of the fields recorded in step n:
    E^{n+1} at (n+1) dt and H^{n+1/2} at (n+1/2) dt (Section 3.5 DTFT with
    the exact staggered time of each field).  Returns [nt][nfreq] each."""
    wp = omega_prime(freqs, omega0)
    n = np.arange(nt, dtype=np.float64)[:, None]
    return np.exp(1j * wp[None, :] * (n + 1.0) * dt), np.exp(1j * wp[None, :] * (n + 0.5) * dt)


def source_spectrum(s: np.ndarray, freqs, omega0: float, dt: float) -> np.ndarray:
    """S_f = sum_n s_n exp(i omega' (n+1/2) dt): the DTFT of J^{n+1/2}."""
    wp = omega_prime(freqs, omega0)
    t = (np.arange(len(s)) + 0.5) * dt
    return np.exp(1j * np.outer(wp, t)) @ s


# ------------------------------------------------- interpolation stencils
def bracket(coords: np.ndarray, p: float, r: int) -> int:
    """Base index of the 2r support nodes around p: coords[m] <= p <
    coords[m+1], support m-r+1 .. m+r (symmetric bracketing)."""
    m = int(np.searchsorted(coords, p, side="right")) - 1
    return m - r + 1


def point_stencil(axes_pad, p, stagger, r: int):
    """Tensor-product Lagrange stencil (Section 3.1: 3D operators as the
    tensor product of three 1D interpolators) on the staggered grid given by
    `stagger`.  Returns (base[3], w[3][2r])."""
    base, w = [], []
    for a in range(3):
        xp = axes_pad[a]
        coords = half_nodes(xp) if stagger[a] else xp
        b = bracket(coords, p[a], r)
        if b < 0 or b + 2 * r > len(coords):
            raise ValueError("point outside the grid")
        base.append(b)
        w.append(lagrange_weights(p[a], coords[b:b + 2 * r]))
    return np.array(base), np.array(w)


def dual_volume(axes_pad, comp: int, base, r: int) -> np.ndarray:
    """Control volume of each E_comp node in the (2r)^3 support: the primal
    interval along the component's own axis times the dual intervals across
    it.  Returns [2r][2r][2r] indexed [kz][jy][ix]."""
    ext = []
    for a in range(3):
        xp = axes_pad[a]
        idx = base[a] + np.arange(2 * r)
        if a == comp:
            ext.append(xp[idx + 1] - xp[idx])
        else:
            xh = half_nodes(xp)
            ext.append(xh[idx] - xh[idx - 1])
    return ext[2][:, None, None] * ext[1][None, :, None] * ext[0][None, None, :]


def inside(base, n_pad, nbe: int, r: int) -> bool:
    """Every support index must lie in the unpadded interior [nbe, n-1-nbe]."""
    return all(nbe <= base[a] and base[a] + 2 * r - 1 <= n_pad[a] - 1 - nbe
               for a in range(3))
