"""Whole-pipeline pins of the oracle.

* analytic whole-space electric dipole (Section 2.1 equations, closed form in
  oracle.analytic) on the 48^3 plain-forward workload: discretisation-level
  agreement, and refinement must reduce the error;
* the z-domain identity (oracle.brute): time loop + DTFT == sparse direct
  solve, with and without CPML, to truncation level;
* reciprocity on a uniform grid without CPML (D- = -(D+)^T there, injection
  = extraction / V);
* omega0 invariance of G and wavelet invariance of G (both exact for the
  discrete scheme up to DFT truncation);
* CPML absorbs: a small box with CPML agrees with a large box far better than
  the same small box with plain zero walls.
"""
import numpy as np
import pytest

from oracle import analytic as A
from oracle import brute as B
from oracle import forward as F
from oracle import tables as T
from workloads import configs, grids


def _errors(G, ref):
    return np.abs(G) / np.abs(ref) - 1.0, np.degrees(np.angle(G / ref))


@pytest.fixture(scope="module")
def plain():
    w = configs.plain_forward()
    # add off-axis receivers so every E and H component is non-trivial
    xs = np.array([-1800.0, -1200.0, -600.0, 600.0, 1200.0, 1800.0])
    off = np.stack([xs, np.full_like(xs, 450.0), np.full_like(xs, -350.0)], axis=1)
    w = w.with_(receivers=np.concatenate([w.receivers, off]))
    G, info = F.forward(w)
    return w, G, info


def test_plain_forward_info(plain):
    w, G, info = plain
    assert info["n_pad"] == (82, 82, 82)
    assert 200 <= info["nt"] <= 400
    assert not info["nonfinite"]


def test_analytic_whole_space_inline(plain):
    w, G, _ = plain
    keep = w.receivers[:21, 0] != 0.0           # the coincident receiver is excluded
    rec = w.receivers[:21][keep]
    E, _ = A.dipole_fields([0, 0, 0], [1, 0, 0], rec, 1.0, 1.0)
    off = np.abs(rec[:, 0])
    amp, ph = _errors(G[0, :21, 0, 0][keep], E[:, 0])
    far = off >= 600
    assert np.max(np.abs(amp[far])) < 0.01 and np.max(np.abs(ph[far])) < 0.5
    mid = off == 400
    assert np.max(np.abs(amp[mid])) < 0.035 and np.max(np.abs(ph[mid])) < 1.0
    # spot magnitudes of the closed form itself (inline: p e^{ikr}(1-ikr)/(2 pi sigma r^3))
    k = A.wavenumber(1.0, 1.0)
    r = 1000.0
    assert abs(E[off == r][0, 0]) == pytest.approx(
        abs(np.exp(1j * k * r) * (1 - 1j * k * r) / (2 * np.pi * r ** 3)), rel=1e-12)


def test_analytic_whole_space_all_components(plain):
    w, G, _ = plain
    rec = w.receivers[21:]
    E, H = A.dipole_fields([0, 0, 0], [1, 0, 0], rec, 1.0, 1.0)
    ref = np.concatenate([E, H], axis=1)          # [nrec][6]
    got = G[0, 21:, :, 0]
    for c in (0, 1, 2, 4, 5):                     # Hx vanishes for an x-dipole
        amp, ph = _errors(got[:, c], ref[:, c])
        assert np.max(np.abs(amp)) < 0.02, (c, amp)
        assert np.max(np.abs(ph)) < 1.0, (c, ph)
    assert np.max(np.abs(got[:, 3])) < 1e-6 * np.max(np.abs(got[:, 4]))


@pytest.mark.slow
def test_refinement_reduces_error():
    errs = []
    for d, n in ((100.0, 30), (50.0, 60)):
        x = grids.centred_uniform_axis(n, d)
        rho = np.ones((n, n, n), np.float32)
        rec = np.array([[600.0, 0, 0], [800.0, 0, 0], [1000.0, 0, 0]])
        w = configs.plain_forward().with_(x1=x, x2=x.copy(), x3=x.copy(), rho11=rho,
                                          rho22=rho, rho33=rho, receivers=rec)
        G, _ = F.forward(w)
        E, _ = A.dipole_fields([0, 0, 0], [1, 0, 0], rec, 1.0, 1.0)
        errs.append(np.max(np.abs(G[0, :, 0, 0] / E[:, 0] - 1.0)))
    assert errs[1] < 0.5 * errs[0], errs


@pytest.mark.parametrize("nb,ne,shape", [(0, 2, (10, 9, 8)), (3, 0, (8, 8, 7))])
def test_z_domain_identity(nb, ne, shape):
    w = configs.small_case(seed=3, shape=shape, rd=2, nb=nb, ne=ne, nrec=3, freqs=(2.0,),
                           nu_axes=(False, True, True))
    fp = T.peak_frequency(w.freqs, w.f0)
    st = F.make_setup(w, fp)
    nt = int(np.ceil(40.0 / (np.imag(T.omega_prime(w.freqs, st.omega0))[0] * st.dt)))
    acc, S, rc = F.run_source(st, nt, w.sources[0], 0, w.receivers, w.channels, w.freqs)
    bf = B.solve(st, w.freqs[0], w.sources[0], 0, w.receivers, w.channels)
    v = acc[:, :, 0] / S[0]
    assert np.max(np.abs(v - bf)) <= 1e-9 * np.max(np.abs(bf))


def test_z_domain_identity_other_source_components():
    w = configs.small_case(seed=4, shape=(9, 9, 8), rd=1, nb=0, ne=2, nrec=2, freqs=(1.0,))
    fp = T.peak_frequency(w.freqs, w.f0)
    st = F.make_setup(w, fp)
    nt = int(np.ceil(40.0 / (np.imag(T.omega_prime(w.freqs, st.omega0))[0] * st.dt)))
    for comp in (1, 2):
        acc, S, _ = F.run_source(st, nt, w.sources[0], comp, w.receivers, w.channels, w.freqs)
        bf = B.solve(st, w.freqs[0], w.sources[0], comp, w.receivers, w.channels)
        assert np.max(np.abs(acc[:, :, 0] / S[0] - bf)) <= 1e-9 * np.max(np.abs(bf))


def test_reciprocity_uniform_grid_without_cpml():
    n = 15
    x = grids.centred_uniform_axis(n, 100.0)
    rho = np.full((n, n, n), 2.0, np.float32)
    rho[:, :, 8:] = 0.5                          # heterogeneous: still reciprocal
    w = configs.small_case(seed=2, shape=(n, n, n), nb=0, ne=2, nt=2500, freqs=(1.0,))
    w = w.with_(x1=x, x2=x.copy(), x3=x.copy(), rho11=rho, rho22=rho.copy(),
                rho33=rho.copy(), chan_mask=1)
    s = np.array([[-213.0, 37.0, -58.0]])
    q = np.array([[188.0, -121.0, 77.0]])
    Gsr, _ = F.forward(w.with_(sources=s, receivers=q))
    Grs, _ = F.forward(w.with_(sources=q, receivers=s))
    assert abs(Gsr.ravel()[0] / Grs.ravel()[0] - 1.0) < 1e-9


def test_omega0_invariance():
    w = configs.small_case(seed=1, shape=(21, 19, 17), nt=0)
    G1, a = F.forward(w.with_(f0=0.7))
    G2, b = F.forward(w.with_(f0=1.9))
    assert a["nt"] == b["nt"]
    assert np.max(np.abs(G1 - G2)) <= 1e-10 * np.max(np.abs(G2))


def test_wavelet_invariance():
    w = configs.small_case(seed=2, shape=(15, 14, 13), nb=0, ne=2, nt=2500, freqs=(1.0, 2.0))
    Ga, _ = F.forward(w, fpeak=1.5)
    Gb, _ = F.forward(w, fpeak=4.0)
    assert np.max(np.abs(Ga - Gb)) <= 1e-10 * np.max(np.abs(Gb))


def test_cpml_absorbs():
    base = configs.plain_forward()

    def box(n, nb, ne):
        x = grids.centred_uniform_axis(n, 100.0)
        r = np.ones((n, n, n), np.float32)
        rec = np.array([[-1500.0, 0, 0], [1000.0, 0, 0], [1500.0, 1400.0, 1300.0]])
        return base.with_(x1=x, x2=x.copy(), x3=x.copy(), rho11=r, rho22=r, rho33=r,
                          receivers=rec, nb=nb, ne=ne, chan_mask=1)
    Gb, _ = F.forward(box(76, 10, 7), nt=300)
    Gc, _ = F.forward(box(36, 10, 7), nt=300)
    Gw, _ = F.forward(box(36, 0, 17), nt=300)
    err_c = np.abs(Gc - Gb) / np.abs(Gb)
    err_w = np.abs(Gw - Gb) / np.abs(Gb)
    assert np.max(err_c) < 2e-4
    assert np.max(err_c) < 0.1 * np.max(err_w)


def test_step_count_is_converged():
    w = configs.plain_forward()
    G1, info = F.forward(w)
    G2, _ = F.forward(w, nt=int(info["nt"] * 1.5))
    rel = np.abs(G1 - G2)[..., 0] / np.abs(G2)[..., 0]
    assert np.max(rel[0, :, 0]) < 1e-5
