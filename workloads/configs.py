"""Concrete synthetic workloads (grids, homogenized models, acquisition).

Every workload is deterministic (seeded where random).  The paper's own
examples (a 101^3 layered marine model, a bathymetry model, Section 6) need
models and reference outputs that are not available, so these stand in for
them with shapes and values in the paper's range: 100 m horizontal spacing,
0.25/0.75/1.25 Hz, 0.3125 ohm-m sea water, a 100 ohm-m resistor, the
transmitter 50 m above the seabed, towed x-directed electric dipoles.

This module is input synthesis shared by the HIP path and the oracle.  It
holds none of the time-stepping arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import grids
from .models import BlockModel, homogenize

CHANNELS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
ALL_CHANNELS = 0x3F


@dataclass
class Workload:
    name: str
    x1: np.ndarray
    x2: np.ndarray
    x3: np.ndarray
    rho11: np.ndarray          # float32 [n3][n2][n1]
    rho22: np.ndarray
    rho33: np.ndarray
    sources: np.ndarray        # float64 [nsrc][3]  (x, y, z), metres
    receivers: np.ndarray      # float64 [nrec][3]
    freqs: np.ndarray          # float64 [nfreq], Hz
    src_comp: np.ndarray = None  # int32 [nsrc]: 0 = Jx, 1 = Jy, 2 = Jz
    chan_mask: int = ALL_CHANNELS
    rd: int = 2
    nb: int = 10
    ne: int = 7
    f0: float = 1.0
    nt: int = 0                # 0: automatic
    dft_mode: int = 0
    cfl: float = 0.99
    airwave: bool = False      # air above the first z node (sea surface) instead of an absorbing top
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.src_comp is None:
            self.src_comp = np.zeros(len(self.sources), dtype=np.int32)

    @property
    def shape(self):
        return (len(self.x1), len(self.x2), len(self.x3))

    @property
    def padded_cells(self) -> int:
        p = 2 * (self.nb + self.ne)
        n1, n2, n3 = self.shape
        return (n1 + p) * (n2 + p) * (n3 + p)

    @property
    def channels(self) -> list[int]:
        return [c for c in range(6) if self.chan_mask >> c & 1]

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _model_arrays(model: BlockModel, x1, x2, x3):
    r11, r22, r33 = homogenize(model, x1, x2, x3)
    return _f32(r11), _f32(r22), _f32(r33)


def _uniform_rho(n1, n2, n3, rho):
    a = np.full((n3, n2, n1), rho, dtype=np.float32)
    return a, a.copy(), a.copy()


# --------------------------------------------------------------------------
# Plain forward: 48^3 uniform 100 m, homogeneous 1 ohm-m whole space,
# unit x-dipole at the centre (between nodes), 21 inline receivers, 1 Hz.
# --------------------------------------------------------------------------
def plain_forward(nt: int = 0) -> Workload:
    n = 48
    x = grids.centred_uniform_axis(n, 100.0)          # -2350 ... 2350
    r11, r22, r33 = _uniform_rho(n, n, n, 1.0)
    rx = np.arange(-2000.0, 2000.0 + 1, 200.0)
    rec = np.stack([rx, np.zeros_like(rx), np.zeros_like(rx)], axis=1)
    return Workload("plain_forward_48cube", x, x.copy(), x.copy(), r11, r22, r33,
                    sources=np.array([[0.0, 0.0, 0.0]]), receivers=rec,
                    freqs=np.array([1.0]), rd=2, nb=10, ne=7, f0=1.0, nt=nt)


def plain_forward_offaxis(nt: int = 0) -> Workload:
    """The plain-forward model with 6 receivers off the source's axis
    (y = 450 m, z = -350 m) after the 21 inline ones: on the axis the
    magnetic field and the transverse E components vanish, so the off-axis
    receivers carry the channels that a comparison can hold to a tolerance."""
    w = plain_forward(nt)
    xs = np.array([-1800.0, -1200.0, -600.0, 600.0, 1200.0, 1800.0])
    off = np.stack([xs, np.full_like(xs, 450.0), np.full_like(xs, -350.0)], axis=1)
    return w.with_(receivers=np.concatenate([w.receivers, off]))


# --------------------------------------------------------------------------
# Marine layered: 128 x 128 x 96 nodes, 100 m horizontal; z positive down,
# sea surface at 0, seafloor node at 1000 m with 25 m spacing, geometric
# stretching up (create_nugrid over the 1000 m water column) and down
# (ratio 1.05); 0.3125 ohm-m water over 1 ohm-m sediment with a 100 ohm-m
# 4000 x 4000 x 100 m box buried 1000 m below the seafloor.
# --------------------------------------------------------------------------
def marine_z_128x128x96() -> np.ndarray:
    return grids.marine_z_axis(1000.0, 25.0, n_up=23, n_down=72, down_ratio=1.05)


def marine_model(box_rho: float = 100.0) -> BlockModel:
    m = BlockModel(background=1.0)
    m.add_layer(-np.inf, 1000.0, 0.3125)
    m.add_box(-2000.0, 2000.0, -2000.0, 2000.0, 2000.0, 2100.0, box_rho)
    return m


def marine_layered(nt: int = 0, box_rho: float = 100.0) -> Workload:
    x = grids.centred_uniform_axis(128, 100.0)        # -6350 ... 6350
    z = marine_z_128x128x96()
    r11, r22, r33 = _model_arrays(marine_model(box_rho), x, x, z)
    rx = np.arange(-5000.0, 5000.0 + 1, 100.0)
    rec = np.stack([rx, np.zeros_like(rx), np.full_like(rx, 1000.0)], axis=1)
    return Workload("marine_layered_128x128x96", x, x.copy(), z, r11, r22, r33,
                    sources=np.array([[0.0, 0.0, 950.0]]), receivers=rec,
                    freqs=np.array([0.25, 0.75, 1.25]), rd=2, nb=10, ne=7,
                    f0=1.0, nt=nt)


def shallow_marine(nt: int = 0, water_depth: float = 100.0) -> Workload:
    """Shallow-water marine survey with the air above the sea surface (the
    paper's air-water top boundary): 128 x 128 x 80 nodes, x and y uniform
    100 m (the FFTs of the air boundary need it), z from the surface z = 0:
    16 intervals of 25 m, then 63 intervals growing by 1.05 (~10.9 km).
    Water 0.3125 ohm-m down to `water_depth`, sediment 1 ohm-m, a 100 ohm-m
    box 4000 x 4000 x 100 m with its top 1000 m below the seafloor.  One
    x-dipole 50 m above the seafloor, 101 seafloor receivers, 0.25 / 0.75 /
    1.25 Hz, r = 2."""
    x = grids.centred_uniform_axis(128, 100.0)
    z = grids.axis_from_intervals(0.0, np.concatenate([np.full(16, 25.0),
                                                       grids.geometric_intervals(25.0, 1.05, 63)]))
    m = BlockModel(background=1.0)
    m.add_layer(-np.inf, water_depth, 0.3125)
    top = water_depth + 1000.0
    m.add_box(-2000.0, 2000.0, -2000.0, 2000.0, top, top + 100.0, 100.0)
    r11, r22, r33 = _model_arrays(m, x, x, z)
    rx = np.arange(-5000.0, 5000.0 + 1, 100.0)
    rec = np.stack([rx, np.zeros_like(rx), np.full_like(rx, water_depth)], axis=1)
    return Workload("shallow_marine_air_128x128x80", x, x.copy(), z, r11, r22, r33,
                    sources=np.array([[0.0, 0.0, water_depth - 50.0]]), receivers=rec,
                    freqs=np.array([0.25, 0.75, 1.25]), rd=2, nb=10, ne=7, f0=1.0, nt=nt,
                    airwave=True)


def towline_sources(count: int = 16, spacing: float = 500.0, z: float = 950.0):
    xs = spacing * (np.arange(count) - 0.5 * (count - 1))
    return np.stack([xs, np.zeros_like(xs), np.full_like(xs, z)], axis=1)


def towline_small(count: int = 16, spacing: float = 250.0) -> Workload:
    """`count` x-dipoles every `spacing` m along the x axis (y = z = 0) of
    the 48^3 plain-forward model: the towline of a multi-transmitter survey
    on a grid small enough (82^3 padded cells) that one source alone leaves
    most of the chip idle.  16 at 250 m span x = -1875..1875."""
    w = plain_forward()
    xs = spacing * (np.arange(count) - 0.5 * (count - 1))
    src = np.stack([xs, np.zeros_like(xs), np.zeros_like(xs)], axis=1)
    return w.with_(name=f"towline_{count}x{spacing:g}m_48cube", sources=src,
                   src_comp=np.zeros(count, dtype=np.int32))


def differentiation_48cube(nt: int = 0) -> tuple:
    """The misfit-gradient workload: the 48^3 plain-forward model (1 ohm-m,
    100 m cells) as the prediction, and the same grid with a 200 ohm-m box
    (|x|, |y| <= 500 m, 300 <= z <= 500 m) as the model that makes the
    observed data; the x-dipole at the origin, the 21 inline receivers, Ex
    only, 0.25 / 0.75 / 1.25 Hz.  Returns (prediction, observed-data model)."""
    w = plain_forward(nt=nt)
    w = w.with_(name="differentiation_48cube", chan_mask=1, freqs=np.array([0.25, 0.75, 1.25]))
    m = BlockModel(background=1.0)
    m.add_box(-500.0, 500.0, -500.0, 500.0, 300.0, 500.0, 200.0)
    r11, r22, r33 = _model_arrays(m, w.x1, w.x2, w.x3)
    return w, w.with_(name="differentiation_48cube_box", rho11=r11, rho22=r22, rho33=r33)


def interior_cells(w, count: int, seed: int, margin: int = 2, weight=None) -> np.ndarray:
    """`count` distinct (component, k, j, i) cells of the input grid, at
    least `margin` nodes inside every face, drawn with numpy's default_rng
    (seed); with `weight` ([3][n3][n2][n1], >= 0) the draw is weighted by it."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = w.shape
    mask = np.zeros((3, n3, n2, n1), dtype=bool)
    mask[:, margin:n3 - margin, margin:n2 - margin, margin:n1 - margin] = True
    p = mask.astype(np.float64) if weight is None else mask * np.asarray(weight, dtype=np.float64)
    flat = rng.choice(p.size, size=count, replace=False, p=p.ravel() / p.sum())
    return np.stack(np.unravel_index(flat, p.shape), axis=1)


# --------------------------------------------------------------------------
# Random layered + box models (seeded), uniform 100 m grid.
# --------------------------------------------------------------------------
def random_layered_box(seed: int, n1: int, n2: int, n3: int, nt: int = 0,
                       rd: int = 2) -> Workload:
    rng = np.random.default_rng(seed)
    x = grids.centred_uniform_axis(n1, 100.0)
    y = grids.centred_uniform_axis(n2, 100.0)
    z = grids.uniform_axis(n3, 100.0, 0.0)

    def logu(lo, hi, size=None):
        return np.exp(rng.uniform(np.log(lo), np.log(hi), size))

    m = BlockModel(background=float(logu(0.3, 100.0)))
    nl = int(rng.integers(2, 6))
    depths = np.sort(rng.uniform(z[0], z[-1], nl - 1))
    edges = np.concatenate([[-np.inf], depths, [np.inf]])
    for i in range(nl):
        m.add_layer(edges[i], edges[i + 1], float(logu(0.3, 100.0)))
    hx, hy = rng.uniform(500.0, 4000.0, 2)
    hz = rng.uniform(50.0, 300.0)
    cz = rng.uniform(z[0] + 0.3 * (z[-1] - z[0]), z[-1] - 0.3 * (z[-1] - z[0]))
    m.add_box(-hx / 2, hx / 2, -hy / 2, hy / 2, cz - hz / 2, cz + hz / 2,
              float(logu(0.3, 100.0)))
    r11, r22, r33 = _model_arrays(m, x, y, z)
    zs = 0.5 * (z[0] + z[-1]) - 49.0
    span = min(2000.0, 0.5 * (x[-1] - x[0]) - 300.0)
    rx = np.linspace(-span, span, 21)
    rec = np.stack([rx, np.full_like(rx, 30.0), np.full_like(rx, zs + 50.0)], axis=1)
    return Workload(f"random_layered_box_s{seed}_{n1}x{n2}x{n3}", x, y, z,
                    r11, r22, r33, sources=np.array([[10.0, -20.0, zs]]),
                    receivers=rec, freqs=np.array([0.25, 0.75, 1.25]), rd=rd,
                    nb=10, ne=rd + 5, f0=1.0, nt=nt)


def batched_models(count: int = 8, nt: int = 0) -> list[Workload]:
    """Eight seeded models from 64^3 to 160 x 160 x 120 nodes."""
    out = []
    for m in range(count):
        n12 = int(round(64 + m * 96 / 7))
        n3 = int(round(64 + m * 56 / 7))
        out.append(random_layered_box(m, n12, n12, n3, nt=nt))
    return out


# --------------------------------------------------------------------------
# Small parity cases: ragged shapes, non-uniform axes, CPML, off-grid sources
# and receivers, all six channels.  Sized so the oracle finishes in seconds.
# --------------------------------------------------------------------------
def small_case(seed: int = 0, shape=(37, 29, 23), rd: int = 2, nb: int = 6,
               ne: int | None = None, nt: int = 600, nu_axes=(False, False, True),
               nsrc: int = 1, nrec: int = 7, freqs=(0.5, 1.5),
               src_comp=None) -> Workload:
    rng = np.random.default_rng(1000 + seed)
    ne = rd + 2 if ne is None else ne
    axes = []
    for a, n in enumerate(shape):
        if nu_axes[a]:
            h = 100.0 * np.exp(rng.uniform(np.log(0.5), np.log(1.6), n - 1))
            h = np.convolve(h, np.ones(3) / 3, mode="same")  # gentle stretching
            ax = grids.axis_from_intervals(0.0, h)
            ax -= 0.5 * (ax[0] + ax[-1])
        else:
            ax = grids.centred_uniform_axis(n, 100.0)
        axes.append(ax)
    x1, x2, x3 = axes
    m = BlockModel(background=float(np.exp(rng.uniform(np.log(0.5), np.log(5)))))
    zc = 0.5 * (x3[0] + x3[-1])
    m.add_layer(-np.inf, zc - 300.0, float(np.exp(rng.uniform(np.log(0.3), np.log(1.0)))))
    m.add_box(-600.0, 500.0, -400.0, 700.0, zc + 100.0, zc + 350.0,
              float(np.exp(rng.uniform(np.log(10.0), np.log(60.0)))))
    r11, r22, r33 = _model_arrays(m, x1, x2, x3)

    def inner_points(count, margin_cells):
        pts = []
        for ax in (x1, x2, x3):
            mc = margin_cells if len(ax) >= 2 * (rd + margin_cells) + 2 else 0
            lo = ax[rd + mc]
            hi = ax[-1 - rd - mc]
            pts.append(rng.uniform(lo, hi, count))
        return np.stack(pts, axis=1)

    src = inner_points(nsrc, 2)
    rec = inner_points(nrec, 2)
    comp = (np.zeros(nsrc, dtype=np.int32) if src_comp is None
            else np.asarray(src_comp, dtype=np.int32))
    return Workload(f"small_s{seed}_{shape[0]}x{shape[1]}x{shape[2]}_r{rd}",
                    x1, x2, x3, r11, r22, r33, sources=src, receivers=rec,
                    freqs=np.asarray(freqs, dtype=np.float64), src_comp=comp,
                    rd=rd, nb=nb, ne=ne, f0=1.0, nt=nt)


# --------------------------------------------------------------------------
# Large marine grid: 400 x 400 x 200 nodes, 50 m horizontal, 10 m at the
# seafloor stretched to 100 m below, three seeded resistive bodies, 8th order.
# --------------------------------------------------------------------------
def large_z_axis() -> np.ndarray:
    n_grow = 48
    ratio = (100.0 / 10.0) ** (1.0 / (n_grow - 1))
    return grids.marine_z_axis(1000.0, 10.0, n_up=37, n_down=162,
                               down_ratio=ratio, down_cap=100.0, n_grow=n_grow)


def large_marine(nt: int = 0, rd: int = 4, nsrc: int = 1) -> Workload:
    rng = np.random.default_rng(2025)
    x = grids.centred_uniform_axis(400, 50.0)         # -9975 ... 9975
    z = large_z_axis()
    m = BlockModel(background=1.0)
    m.add_layer(-np.inf, 1000.0, 0.3125)
    for _ in range(3):
        sx, sy = rng.uniform(1000.0, 5000.0, 2)
        sz = rng.uniform(50.0, 300.0)
        cx, cy = rng.uniform(-5000.0, 5000.0, 2)
        top = rng.uniform(1200.0, 4000.0)
        rho = float(np.exp(rng.uniform(np.log(20.0), np.log(100.0))))
        m.add_box(cx - sx / 2, cx + sx / 2, cy - sy / 2, cy + sy / 2, top, top + sz, rho)
    r11, r22, r33 = _model_arrays(m, x, x, z)
    gx = -7600.0 + 800.0 * np.arange(20)
    gxx, gyy = np.meshgrid(gx, gx, indexing="xy")
    rec = np.stack([gxx.ravel(), gyy.ravel(), np.full(gxx.size, 1000.0)], axis=1)
    sx = -7000.0 + 2000.0 * np.arange(8)
    src = np.stack([sx, np.zeros(8), np.full(8, 950.0)], axis=1)[:nsrc]
    freqs = np.geomspace(0.1, 2.0, 5)
    return Workload("large_marine_400x400x200", x, x.copy(), z, r11, r22, r33,
                    sources=src, receivers=rec, freqs=freqs, rd=rd, nb=10,
                    ne=rd + 5, f0=1.0, nt=nt, dft_mode=1)


def uniform_cube(n: int, rd: int = 2, nt: int = 100) -> Workload:
    """Homogeneous n^3 cube for bandwidth sweeps (1 ohm-m, 50 m)."""
    x = grids.centred_uniform_axis(n, 50.0)
    r11, r22, r33 = _uniform_rho(n, n, n, 1.0)
    rec = np.array([[100.0, 0.0, 0.0], [400.0, 100.0, -50.0]])
    return Workload(f"uniform_cube_{n}", x, x.copy(), x.copy(), r11, r22, r33,
                    sources=np.array([[0.0, 0.0, 0.0]]), receivers=rec,
                    freqs=np.array([1.0]), rd=rd, nb=10, ne=rd + 5, nt=nt)


# --------------------------------------------------------------------------
# Stretched-axis pins of the injection control volume and the padding.
# --------------------------------------------------------------------------
def stretched_z_axis(ratio: float = 1.2, d0: float = 20.0, z_fine: float = -600.0,
                     n_down: int = 22, n_up: int = 20) -> np.ndarray:
    """z axis whose intervals grow geometrically by `ratio` away from a fine
    point z_fine (first interval d0 on each side).  Below z_fine every node
    has an interval below it `ratio` times the one above it, so the dual
    interval at a node, (h_{k-1} + h_k)/2, differs from the primal one below
    it by 2 ratio/(1 + ratio) (9 % at 1.2)."""
    down = grids.axis_from_intervals(z_fine, grids.geometric_intervals(d0, ratio, n_down))
    up = grids.axis_from_intervals(z_fine, -grids.geometric_intervals(d0, ratio, n_up))
    return np.concatenate([up[::-1], down[1:]])


def stretched_whole_space(comp: int = 0, ratio: float = 1.2, n: int = 60, d: float = 80.0,
                          nt: int = 0) -> Workload:
    """Homogeneous 1 ohm-m whole space on a uniform 80 m x, y grid and the
    strongly stretched z axis of `stretched_z_axis` (the source sits 600 m
    below the fine point, in cells of ~124 and ~149 m whose neighbours
    differ by `ratio`); a unit dipole along axis `comp` at the origin, 10
    receivers on the x axis at 400..2000 m on both sides, 1 Hz."""
    x = grids.centred_uniform_axis(n, d)
    z = stretched_z_axis(ratio)
    r11, r22, r33 = _uniform_rho(n, n, len(z), 1.0)
    off = np.array([400.0, 800.0, 1200.0, 1600.0, 2000.0])
    rx = np.concatenate([-off[::-1], off])
    rec = np.stack([rx, np.zeros_like(rx), np.zeros_like(rx)], axis=1)
    return Workload(f"stretched_whole_space_q{ratio:g}_c{comp}", x, x.copy(), z, r11, r22, r33,
                    sources=np.array([[0.0, 0.0, 0.0]]), receivers=rec,
                    freqs=np.array([1.0]), src_comp=np.array([comp], np.int32),
                    chan_mask=1 << comp, rd=2, nb=10, ne=7, f0=1.0, nt=nt)


def marine_reciprocity(n: int = 40, freq: float = 0.75, extend_z: int = 0) -> tuple:
    """The marine z axis (25 m at the seafloor, growing by ~1.047 up to the
    sea surface and by 1.05 down) under a 40 x 40 node, 100 m horizontal
    grid; 0.3125 ohm-m water over 1 ohm-m sediment; CPML on every face; Ex
    only.  Returns (workload, a, b): two points with different local
    stretching (50 m above the seafloor in the water, 500 m below it) for
    the swap G(b; a) = G(a; b).  extend_z > 0 continues the z axis by that
    many nodes at each end with the end intervals (a longer box of the same
    medium)."""
    x = grids.centred_uniform_axis(n, 100.0)
    z = marine_z_128x128x96()
    if extend_z > 0:
        h0, h1 = z[1] - z[0], z[-1] - z[-2]
        z = np.concatenate([z[0] - h0 * np.arange(extend_z, 0, -1), z,
                            z[-1] + h1 * np.arange(1, extend_z + 1)])
    m = BlockModel(background=1.0)
    m.add_layer(-np.inf, 1000.0, 0.3125)
    r11, r22, r33 = _model_arrays(m, x, x, z)
    a = np.array([-600.0, -150.0, 950.0])
    b = np.array([700.0, 250.0, 1500.0])
    w = Workload(f"marine_reciprocity_{n}x{n}x{len(z)}", x, x.copy(), z, r11, r22, r33,
                 sources=a[None, :], receivers=b[None, :], freqs=np.array([freq]),
                 chan_mask=1, rd=2, nb=10, ne=7, f0=1.0)
    return w, a, b
