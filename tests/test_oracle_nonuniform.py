"""Pins of the oracle on strongly non-uniform axes: the injection control
volume and the padding of a stretched axis.

The injection of a point dipole divides the interpolation weights (the
tensor product of 1-D Lagrange operators, Section 3.1) by the control volume
of each E node: the primal interval along the component times the dual
intervals across it.  On a uniform axis primal and dual intervals coincide,
so only stretched axes can tell a slip between them; likewise the padding
(Section 3.4: nb + ne extra layers per side, whose spacing the paper leaves
open) only matters where the axis is not uniform.  These tests hold the
oracle to what the physics fixes there:

* the analytic whole-space dipole (Section 2.1, closed form in
  oracle.analytic) on a z axis stretched by 1.2 around the source, for an x
  dipole (z across the component: dual intervals) and a z dipole (z along
  it: primal interval);
* source-receiver reciprocity G_xx(b; a) = G_xx(a; b) of the Green's
  function of a symmetric conductivity, on the marine z axis with CPML,
  between points of different local stretching;
* a padded box agrees with a longer box of the same medium (the padding and
  its CPML do not show in the interior).

Each mistake these pins are for is planted in the oracle (on the CPU) and
shown to fail the same check.
"""
import numpy as np
import pytest

from oracle import analytic as A
from oracle import forward as F
from oracle import tables as T
from workloads import configs

ANALYTIC_AMP = 0.03        # 400..2000 m offsets
ANALYTIC_PHASE_DEG = 2.0
ANALYTIC_FAR_AMP = 0.01    # >= 800 m offsets
RECIPROCITY_TOL = 1e-2     # stretched axis with CPML: the D+/D- pair is not exactly adjoint
PADDING_TOL = 1e-5


def _dipole_errors(comp):
    w = configs.stretched_whole_space(comp=comp)
    G, _ = F.forward(w)
    d = [0.0, 0.0, 0.0]
    d[comp] = 1.0
    E, _ = A.dipole_fields([0.0, 0.0, 0.0], d, w.receivers, 1.0, 1.0)
    ratio = G[0, :, 0, 0] / E[:, comp]
    off = np.abs(w.receivers[:, 0])
    return off, np.abs(ratio) - 1.0, np.degrees(np.angle(ratio))


def _analytic_ok(off, amp, ph):
    far = off >= 800.0
    return bool(np.max(np.abs(amp)) <= ANALYTIC_AMP and np.max(np.abs(ph)) <= ANALYTIC_PHASE_DEG
                and np.max(np.abs(amp[far])) <= ANALYTIC_FAR_AMP)


def _reciprocity_error():
    w, a, b = configs.marine_reciprocity()
    G_ab, _ = F.forward(w)
    G_ba, _ = F.forward(w.with_(sources=b[None, :], receivers=a[None, :]))
    return abs(G_ab.ravel()[0] / G_ba.ravel()[0] - 1.0)


def _padding_difference():
    w, _, _ = configs.marine_reciprocity()
    wl, _, _ = configs.marine_reciprocity(extend_z=30)
    G, _ = F.forward(w)
    G_long, _ = F.forward(wl)
    return abs(G.ravel()[0] / G_long.ravel()[0] - 1.0)


def _primal_everywhere(axes_pad, comp, base, r):
    """Planted slip: primal intervals across the component as well."""
    ext = []
    for a in range(3):
        idx = base[a] + np.arange(2 * r)
        ext.append(axes_pad[a][idx + 1] - axes_pad[a][idx])
    return ext[2][:, None, None] * ext[1][None, :, None] * ext[0][None, None, :]


def _dual_everywhere(axes_pad, comp, base, r):
    """Planted slip: dual intervals along the component as well."""
    ext = []
    for a in range(3):
        xh = T.half_nodes(axes_pad[a])
        idx = base[a] + np.arange(2 * r)
        ext.append(xh[idx] - xh[idx - 1])
    return ext[2][:, None, None] * ext[1][None, :, None] * ext[0][None, None, :]


def _swapped_ends(x, nbe):
    """Planted slip: each end padded with the other end's interval."""
    x = np.asarray(x, dtype=np.float64)
    lo = x[0] - (x[-1] - x[-2]) * np.arange(nbe, 0, -1)
    hi = x[-1] + (x[1] - x[0]) * np.arange(1, nbe + 1)
    return np.concatenate([lo, x, hi])


def test_stretched_axis_is_strongly_non_uniform_at_the_source():
    w = configs.stretched_whole_space()
    z = w.x3
    h = np.diff(z)
    k = int(np.searchsorted(z, 0.0))          # z[k-1] < 0 <= z[k]
    # every node of the 4-node z support of the source: its interval below is
    # 1.2 times the one above, so dual and primal intervals differ by >= 9 %
    for node in range(k - 2, k + 2):
        assert h[node] / h[node - 1] == pytest.approx(1.2, rel=1e-12)
        dual = 0.5 * (h[node - 1] + h[node])
        assert abs(h[node] / dual - 1.0) >= 0.09


def test_analytic_x_dipole_on_stretched_z():
    """Measured: amplitude 2.8 % at 400 m, <= 0.53 % from 800 m; phase
    <= 0.42 degree."""
    off, amp, ph = _dipole_errors(0)
    assert _analytic_ok(off, amp, ph), (amp, ph)


def test_analytic_z_dipole_on_stretched_z():
    """z is the component axis here (primal interval).  Measured: amplitude
    1.6 % at 400 m, <= 0.34 % from 800 m; phase <= 0.05 degree."""
    off, amp, ph = _dipole_errors(2)
    assert _analytic_ok(off, amp, ph), (amp, ph)


def test_planted_volume_slips_fail_the_analytic_pin(monkeypatch):
    """Primal intervals across the component bias the x dipole by ~9 %;
    dual intervals along it bias the z dipole by ~9 %."""
    monkeypatch.setattr(T, "dual_volume", _primal_everywhere)
    off, amp, ph = _dipole_errors(0)
    assert not _analytic_ok(off, amp, ph)
    assert np.min(np.abs(amp[off >= 800.0])) > 0.05
    monkeypatch.setattr(T, "dual_volume", _dual_everywhere)
    off, amp, ph = _dipole_errors(2)
    assert not _analytic_ok(off, amp, ph)
    assert np.min(np.abs(amp[off >= 800.0])) > 0.05


def test_reciprocity_on_marine_stretched_z_with_cpml():
    """Source 50 m above the seafloor in the water (intervals shrinking
    downwards by 1/1.047), receiver 500 m below it in the sediment
    (intervals growing by 1.05), CPML on every face.  Measured:
    |G(b; a)/G(a; b) - 1| = 5.2e-4."""
    err = _reciprocity_error()
    assert err <= RECIPROCITY_TOL, err


def test_planted_volume_slip_breaks_reciprocity(monkeypatch):
    """Primal intervals across the component scale the two injections by
    2q/(1+q) at their own local ratios q: 4.8e-2 apart here."""
    monkeypatch.setattr(T, "dual_volume", _primal_everywhere)
    assert _reciprocity_error() > RECIPROCITY_TOL


def test_padding_of_a_stretched_axis_does_not_show_in_the_interior():
    """The marine z axis (end intervals 69 m at the sea surface, 799 m at
    the bottom) padded by nb + ne layers with CPML, against the same medium
    on the axis continued by 30 more nodes at each end.  Measured:
    1.0e-7.  Only where the padding meets fields does its spacing matter;
    any padding whose CPML absorbs as well gives the same interior result
    (the choice of the end interval is a reading, held between the oracle
    and the library by the parity tests)."""
    assert _padding_difference() <= PADDING_TOL


def test_planted_padding_slip_shows_in_the_interior(monkeypatch):
    """Swapping the end intervals puts 69 m cells and a 690 m CPML under the
    deep end and 799 m cells right above the water column: 1.9e-3."""
    monkeypatch.setattr(T, "pad_axis", _swapped_ends)
    w, _, _ = configs.marine_reciprocity()
    G_bad, _ = F.forward(w)
    monkeypatch.undo()
    wl, _, _ = configs.marine_reciprocity(extend_z=30)
    G_long, _ = F.forward(wl)
    assert abs(G_bad.ravel()[0] / G_long.ravel()[0] - 1.0) > PADDING_TOL
