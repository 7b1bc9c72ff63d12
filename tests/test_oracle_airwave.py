"""Pins of the oracle's air boundary above the sea surface (Section 3.3).

* The ghost-plane fills are exact on fields that are harmonic in the air:
  single horizontal Fourier modes psi = cos(kx x + ky y + t) exp(|kappa| z)
  (z positive down) and their gradients, on the staggered positions of each
  component.  This fixes the decay sign and rate, the wavenumbers of the DFT
  bins, the i k/|kappa| relation between the horizontal and vertical H, the
  half-cell shifts of H1 and H2 and the heights of the ghost nodes.
* The time loop with the ghost fills equals the z-domain direct solve of the
  same spatially discrete system (oracle.brute with the fills as sparse
  maps), to truncation of the DTFT.
"""
import numpy as np
import pytest

from oracle import airwave as AW
from oracle import brute as B
from oracle import forward as F
from oracle import tables as T
from workloads import configs


def _axes(r=3, ks=5):
    x = -1150.0 + 100.0 * np.arange(24)
    y = 300.0 + 80.0 * np.arange(20)
    h = np.array([60.0, 55.0, 40.0, 30.0, 25.0, 25.0, 30.0, 40.0, 55.0])
    z = np.concatenate([[0.0], np.cumsum(h)])
    z = z - z[ks]                                    # surface node ks at z = 0
    return x, y, z, r, ks


def _modes(x, y):
    n1, n2 = len(x), len(y)
    dx, dy = x[1] - x[0], y[1] - y[0]
    out = []
    for px, py, amp, th in ((1, 0, 1.0, 0.3), (3, -2, 0.7, 1.1), (-5, 4, 0.4, -0.6), (0, 3, 0.9, 2.0)):
        kx, ky = 2 * np.pi * px / (n1 * dx), 2 * np.pi * py / (n2 * dy)
        out.append((kx, ky, np.hypot(kx, ky), amp, th))
    return out


def test_E_ghosts_are_exact_for_harmonic_fields():
    x, y, z, r, ks = _axes()
    ops = AW.make_ops((x, y, z), ks, r)
    xh, yh = x + 50.0, y + 40.0
    n3 = len(z)

    def field(xs, ys):            # [n3][n2][n1] of a sum of harmonic modes plus a constant
        F3 = np.full((n3, len(ys), len(xs)), 0.25)
        for kx, ky, kap, a, th in _modes(x, y):
            ph = kx * xs[None, None, :] + ky * ys[None, :, None] + th
            F3 += a * np.cos(ph) * np.exp(kap * z[:, None, None])
        return F3
    E1, E2 = field(xh, y), field(x, yh)              # E1 at (i+1/2, j), E2 at (i, j+1/2)
    ref1, ref2 = E1.copy(), E2.copy()
    E1[:ks], E2[:ks] = 0.0, 0.0
    AW.fill_E(E1, E2, ops)
    for m in range(1, r):
        assert np.max(np.abs(E1[ks - m] - ref1[ks - m])) < 1e-12
        assert np.max(np.abs(E2[ks - m] - ref2[ks - m])) < 1e-12
    assert np.all(E1[:ks - r + 1] == 0.0)           # nothing written beyond the ghost nodes


def test_H_ghosts_are_exact_for_potential_fields():
    x, y, z, r, ks = _axes()
    ops = AW.make_ops((x, y, z), ks, r)
    xh, yh = x + 50.0, y + 40.0
    zh = 0.5 * (z[:-1] + z[1:])                      # half nodes: index k <-> z_{k+1/2}
    n1, n2 = len(x), len(y)
    H3 = np.zeros((len(z), n2, n1))
    H1 = np.zeros_like(H3)
    H2 = np.zeros_like(H3)
    ref1 = np.zeros((len(zh), n2, n1))
    ref2 = np.zeros_like(ref1)
    for kx, ky, kap, a, th in _modes(x, y):
        # psi = a cos(kx x + ky y + th) exp(kap z); H = grad psi
        ph3 = kx * xh[None, :] + ky * yh[:, None] + th          # H3 at (i+1/2, j+1/2)
        H3[ks] += a * kap * np.cos(ph3)
        ph1 = kx * x[None, :] + ky * yh[:, None] + th           # H1 at (i, j+1/2)
        ph2 = kx * xh[None, :] + ky * y[:, None] + th           # H2 at (i+1/2, j)
        ez = np.exp(kap * zh)[:, None, None]
        ref1 += -a * kx * np.sin(ph1)[None] * ez
        ref2 += -a * ky * np.sin(ph2)[None] * ez
    AW.fill_H(H1, H2, H3, ops)
    scale = np.max(np.abs(H3))
    for m in range(1, r + 1):
        assert np.max(np.abs(H1[ks - m] - ref1[ks - m])) < 1e-12 * scale
        assert np.max(np.abs(H2[ks - m] - ref2[ks - m])) < 1e-12 * scale


def test_ghost_fill_rejects_non_uniform_horizontal_axes():
    x, y, z, r, ks = _axes()
    x2 = x.copy()
    x2[3] += 1.0
    with pytest.raises(ValueError):
        AW.make_ops((x2, y, z), ks, r)


@pytest.mark.parametrize("rd,ne,shape", [(2, 2, (12, 11, 10)), (3, 3, (11, 10, 9))])
def test_z_domain_identity_with_air(rd, ne, shape):
    w = configs.small_case(seed=5, shape=shape, rd=rd, nb=0, ne=ne, nrec=3, freqs=(2.0,),
                           nu_axes=(False, False, True)).with_(airwave=True)
    fp = T.peak_frequency(w.freqs, w.f0)
    st = F.make_setup(w, fp)
    nt = int(np.ceil(40.0 / (np.imag(T.omega_prime(w.freqs, st.omega0))[0] * st.dt)))
    acc, S, rc = F.run_source(st, nt, w.sources[0], 0, w.receivers, w.channels, w.freqs,
                              airwave=True)
    assert rc == 0
    bf = B.solve(st, w.freqs[0], w.sources[0], 0, w.receivers, w.channels, airwave=True)
    v = acc[:, :, 0] / S[0]
    assert np.max(np.abs(v - bf)) <= 1e-9 * np.max(np.abs(bf))
    # the air changes the answer (the boundary is live)
    bz = B.solve(st, w.freqs[0], w.sources[0], 0, w.receivers, w.channels)
    assert np.max(np.abs(bz - bf)) > 1e-3 * np.max(np.abs(bf))
