"""Rectilinear axis builders for the synthetic workloads.

These produce node coordinates only; they are inputs shared by the HIP path and
the oracle and hold none of the time-stepping arithmetic.

`create_nugrid` follows the optimal geometric-progression grid of the paper
(Section 3.7, the relation L = dx (q^n - 1)/(q - 1) and its fixed-point
iteration q <- (L (q - 1)/dx + 1)^(1/n)).  The paper's version works in single
precision with a stopping threshold that single precision can never meet and
claims |g'(q)| < 1 for every q > 1 (in fact g'(1+) = L/(n dx) > 1).  Here the
iteration runs in double precision, stops at |dq| <= 1e-14 q, is capped at
10^4 iterations and takes the uniform shortcut when |n dx - L| <= 1e-12 L.
Convergence from q0 > 1 still holds: g is concave with fixed points 1 and q*.
"""
from __future__ import annotations

import numpy as np


def uniform_axis(n: int, d: float, x0: float) -> np.ndarray:
    """n equally spaced nodes x0, x0 + d, ..., x0 + (n-1) d."""
    return x0 + d * np.arange(n, dtype=np.float64)


def centred_uniform_axis(n: int, d: float) -> np.ndarray:
    """n nodes spaced d, symmetric about 0 (e.g. n=48, d=100 -> -2350..2350)."""
    return uniform_axis(n, d, -0.5 * d * (n - 1))


def create_nugrid(n: int, length: float, dx: float) -> tuple[float, np.ndarray]:
    """Geometric grid of n intervals (n+1 nodes) over [0, length], first
    interval dx, common ratio q >= 1 (Section 3.7).  Returns (q, x)."""
    if n < 1 or length <= 0.0 or dx <= 0.0:
        raise ValueError("create_nugrid needs n >= 1, length > 0, dx > 0")
    if n * dx > length * (1.0 + 1e-12):
        raise ValueError("n*dx exceeds length: a ratio q >= 1 does not exist")
    if abs(n * dx - length) <= 1e-12 * length:
        return 1.0, dx * np.arange(n + 1, dtype=np.float64)
    q = 1.1
    for _ in range(10000):
        q_next = (length * (q - 1.0) / dx + 1.0) ** (1.0 / n)
        if abs(q_next - q) <= 1e-14 * q:
            q = q_next
            break
        q = q_next
    i = np.arange(n + 1, dtype=np.float64)
    x = (q ** i - 1.0) * dx / (q - 1.0)
    return q, x


def geometric_intervals(d0: float, ratio: float, count: int) -> np.ndarray:
    """count interval lengths d0, d0*ratio, d0*ratio^2, ..."""
    return d0 * ratio ** np.arange(count, dtype=np.float64)


def axis_from_intervals(x_start: float, intervals: np.ndarray) -> np.ndarray:
    """Nodes x_start, x_start + h0, x_start + h0 + h1, ..."""
    return np.concatenate([[x_start], x_start + np.cumsum(intervals)])


def marine_z_axis(z_seafloor: float, dz: float, n_up: int, n_down: int,
                  down_ratio: float, down_cap: float | None = None,
                  n_grow: int | None = None) -> np.ndarray:
    """z axis positive down with its finest interval dz at the seafloor.

    Above the seafloor, `create_nugrid(n_up, z_seafloor, dz)` is mirrored so
    that the smallest interval touches the seafloor and the top node sits at
    the sea surface z = 0.  Below, intervals grow as dz * down_ratio^k; with
    `down_cap` they grow for `n_grow` intervals and are then held at the cap.
    """
    _, up = create_nugrid(n_up, z_seafloor, dz)
    above = z_seafloor - up[::-1]          # 0 ... z_seafloor, finest at the bottom
    above[0] = 0.0
    if down_cap is None:
        h = geometric_intervals(dz, down_ratio, n_down)
    else:
        g = n_grow if n_grow is not None else n_down
        h = np.minimum(geometric_intervals(dz, down_ratio, n_down), down_cap)
        h[g:] = down_cap
    below = axis_from_intervals(z_seafloor, h)
    return np.concatenate([above, below[1:]])
