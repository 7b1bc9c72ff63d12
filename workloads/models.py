"""Resistivity models on a rectilinear mesh: layers and axis-aligned boxes,
homogenized onto the three staggered resistivity arrays.

The method takes three resistivity arrays rho11, rho22, rho33 of shape
[n3][n2][n1] (x fastest) that sit at the Ex, Ey and Ez positions, i.e. half a
cell shifted along x, y and z respectively (Section 5, resistivity files).
They are built outside the modelling kernel with the medium averaging of
Section 3.6: the component along an axis sees the cells along that axis in
series and the cells across its dual face in parallel.  The printed formula is
garbled (it averages sigma_xx arithmetically along x and has a z/x typo); the
reading used here is: each component's conductivity is the harmonic mean along
its own axis of the arithmetic mean of sigma over the dual-cell face in the
other two axes.  For piecewise-constant models made of layers and boxes this
is evaluated exactly from the overlap lengths of each dual cell with the
model's own breakpoints.

This module is input synthesis shared by both implementations; it holds none
of the time-stepping arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Box:
    """Axis-aligned box [x0,x1] x [y0,y1] x [z0,z1] of resistivity rho (ohm-m).
    Use +-inf extents for layers."""
    x0: float
    x1: float
    y0: float
    y1: float
    z0: float
    z1: float
    rho: float


@dataclass
class BlockModel:
    """Background resistivity with boxes painted in order (later boxes win)."""
    background: float
    boxes: list[Box] = field(default_factory=list)

    def add_layer(self, z0: float, z1: float, rho: float) -> "BlockModel":
        inf = np.inf
        self.boxes.append(Box(-inf, inf, -inf, inf, z0, z1, rho))
        return self

    def add_box(self, x0, x1, y0, y1, z0, z1, rho) -> "BlockModel":
        self.boxes.append(Box(x0, x1, y0, y1, z0, z1, rho))
        return self

    def breakpoints(self, axis: int) -> np.ndarray:
        pts = []
        for b in self.boxes:
            lo, hi = [(b.x0, b.x1), (b.y0, b.y1), (b.z0, b.z1)][axis]
            pts += [p for p in (lo, hi) if np.isfinite(p)]
        return np.unique(np.asarray(pts, dtype=np.float64))

    def sigma_on_partition(self, bx, by, bz) -> np.ndarray:
        """Conductivity on the tensor partition defined by breakpoints
        (-inf, b0, b1, ..., +inf) per axis; returns [nz][ny][nx] intervals."""
        def mids(b):
            e = np.concatenate([[-np.inf], b, [np.inf]])
            m = np.empty(len(e) - 1)
            for i in range(len(m)):
                lo, hi = e[i], e[i + 1]
                if np.isinf(lo) and np.isinf(hi):
                    m[i] = 0.0
                elif np.isinf(lo):
                    m[i] = hi - 1.0
                elif np.isinf(hi):
                    m[i] = lo + 1.0
                else:
                    m[i] = 0.5 * (lo + hi)
            return m
        mx, my, mz = mids(bx), mids(by), mids(bz)
        rho = np.full((len(mz), len(my), len(mx)), self.background, dtype=np.float64)
        for b in self.boxes:
            sx = (mx > b.x0) & (mx < b.x1)
            sy = (my > b.y0) & (my < b.y1)
            sz = (mz > b.z0) & (mz < b.z1)
            rho[np.ix_(sz, sy, sx)] = b.rho
        return 1.0 / rho


def _extend(x: np.ndarray) -> np.ndarray:
    """Append one node at each end, one end-interval away (only used to close
    the dual cells of the outermost nodes)."""
    return np.concatenate([[x[0] - (x[1] - x[0])], x, [x[-1] + (x[-1] - x[-2])]])


def _cells(x: np.ndarray, staggered: bool) -> tuple[np.ndarray, np.ndarray]:
    """Extents of the averaging cells along one axis for the n nodes of x.
    staggered: primal interval [x_i, x_{i+1}] (the half node i+1/2);
    otherwise the dual interval [x_{i-1/2}, x_{i+1/2}] around node i."""
    xe = _extend(x)
    if staggered:
        return xe[1:-1], xe[2:]
    h = 0.5 * (xe[:-1] + xe[1:])
    return h[:-1], h[1:]


def _overlap(lo: np.ndarray, hi: np.ndarray, bp: np.ndarray) -> np.ndarray:
    """Overlap lengths [ncell][ninterval] of cells [lo,hi] with the intervals
    (-inf,b0), (b0,b1), ..., (bk,+inf)."""
    e = np.concatenate([[-np.inf], bp, [np.inf]])
    a = np.maximum(lo[:, None], e[None, :-1])
    b = np.minimum(hi[:, None], e[None, 1:])
    return np.clip(b - a, 0.0, None)


def homogenize(model: BlockModel, x1: np.ndarray, x2: np.ndarray, x3: np.ndarray):
    """Return float64 (rho11, rho22, rho33), each [n3][n2][n1]."""
    bps = [model.breakpoints(a) for a in range(3)]
    sig = model.sigma_on_partition(*bps)          # [Iz][Iy][Ix]
    axes = (x1, x2, x3)
    out = []
    for comp in range(3):
        ov = []
        for a in range(3):
            lo, hi = _cells(axes[a], staggered=(a == comp))
            o = _overlap(lo, hi, bps[a])
            ov.append(o / (hi - lo)[:, None])       # fractions
        fx, fy, fz = ov                             # [n][I]
        if comp == 0:
            # parallel over (y, z): face mean for each x interval, then series along x
            face = np.einsum("kc,jb,cba->akj", fz, fy, sig)   # [Ix][n3][n2]
            res = np.einsum("ia,akj->kji", fx, 1.0 / face)
        elif comp == 1:
            face = np.einsum("kc,ia,cba->bki", fz, fx, sig)   # [Iy][n3][n1]
            res = np.einsum("jb,bki->kji", fy, 1.0 / face)
        else:
            face = np.einsum("jb,ia,cba->cji", fy, fx, sig)   # [Iz][n2][n1]
            res = np.einsum("kc,cji->kji", fz, 1.0 / face)
        out.append(np.ascontiguousarray(res))
    return tuple(out)
