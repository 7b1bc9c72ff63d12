"""Pins of the oracle's set-up quantities and of the shared input synthesis."""
import numpy as np
import pytest

from oracle import forward as F
from oracle import tables as T
from workloads import configs, grids
from workloads.models import BlockModel, homogenize


def test_time_step_closed_form_uniform_cube():
    """Section 3.2 on uniform cubic cells: D_d = 2 sum_l |c_l|/dx in every
    direction, so dt = 0.99 dx/(v sqrt(3) sum_l |c_l|), v = sqrt(2 w0 rho/mu0)."""
    w = configs.plain_forward()
    st = F.make_setup(w, fp=2.0)
    v = np.sqrt(2 * 2 * np.pi * 1.0 * 1.0 / T.MU0)
    expect = 0.99 * 100.0 / (v * np.sqrt(3.0) * (9 / 8 + 1 / 24))
    assert st.dt == pytest.approx(expect, rel=1e-13)
    assert st.dt == pytest.approx(0.0154927, rel=1e-5)


def test_time_step_uses_largest_resistivity_and_finest_spacing():
    w = configs.marine_layered()
    st = F.make_setup(w, fp=2.0)
    # the (homogenized) resistor sets v_max; the 25 m seafloor interval sets D_z
    rmax = max(float(a.max()) for a in (w.rho11, w.rho22, w.rho33))
    assert 50.0 < rmax <= 100.0
    v = np.sqrt(2 * 2 * np.pi * rmax / T.MU0)
    d = [2 * (9 / 8 + 1 / 24) / 100.0] * 2
    dz = max(np.abs(st.fd[2][0]).sum(axis=1).max(), np.abs(st.fd[2][1]).sum(axis=1).max())
    assert dz == pytest.approx(2 * (9 / 8 + 1 / 24) / 25.0, rel=0.05)
    eta = 0.5 * v * np.sqrt(d[0] ** 2 + d[1] ** 2 + dz ** 2)
    assert st.dt == pytest.approx(0.99 / eta, rel=1e-12)
    assert 6.0e-4 < st.dt < 7.5e-4


def test_cpml_tables_shape_and_limits():
    w = configs.small_case(seed=0)
    st = F.make_setup(w, fp=2.0)
    n = st.n_pad[0]
    a_i, b_i, a_h, b_h = st.cpml[0]
    inner = slice(st.nb, n - st.nb)
    assert not a_i[inner].any() and not b_i[inner].any()
    slab = np.r_[0:st.nb, n - st.nb:n - 1]
    # 0 < b < 1 and a = b - 1 when alpha = 0 at the outer face (d only)
    assert np.all((b_i[slab] > 0) & (b_i[slab] < 1)) and np.all(a_i[slab] < 0)
    assert a_i[0] == pytest.approx(b_i[0] - 1.0, rel=1e-12)
    # damping grows towards the outer faces
    assert np.all(np.diff(b_i[:st.nb]) > 0)
    assert np.all(np.diff(b_h[n - st.nb:n - 1]) < 0)
    # no CPML at all when nb = 0
    st0 = F.make_setup(w.with_(nb=0), fp=2.0)
    assert all(not np.any(t) for ax in st0.cpml for t in ax)


def test_create_nugrid_fixed_point():
    """Section 3.7: L = dx (q^n - 1)/(q - 1); geometric intervals."""
    q, x = grids.create_nugrid(23, 1000.0, 25.0)
    assert x[0] == 0.0 and x[-1] == pytest.approx(1000.0, rel=1e-12)
    assert 25.0 * (q ** 23 - 1) / (q - 1) == pytest.approx(1000.0, rel=1e-12)
    assert q == pytest.approx(1.0471760, abs=5e-7)
    h = np.diff(x)
    assert h[0] == pytest.approx(25.0, rel=1e-12)
    assert np.allclose(h[1:] / h[:-1], q, rtol=1e-10)
    q1, x1 = grids.create_nugrid(10, 100.0, 10.0)
    assert q1 == 1.0 and np.allclose(x1, np.arange(11) * 10.0)


def test_marine_axis_layout():
    z = configs.marine_z_128x128x96()
    assert len(z) == 96 and z[0] == 0.0
    assert np.all(np.diff(z) > 0)
    i = int(np.argmin(np.abs(z - 1000.0)))
    assert z[i] == pytest.approx(1000.0, abs=1e-9)
    assert z[i + 1] - z[i] == pytest.approx(25.0) and z[i] - z[i - 1] == pytest.approx(25.0)


def test_homogenization_series_and_parallel():
    """Section 3.6: a cell cut by a horizontal interface sees it in series
    for the normal (z) component and in parallel for tangential ones."""
    x = np.arange(4) * 10.0
    z = np.array([0.0, 10.0, 20.0, 30.0])
    m = BlockModel(background=1.0).add_layer(-np.inf, 14.0, 4.0)  # rho 4 above z=14
    r11, r22, r33 = homogenize(m, x, x, z)
    # rho33 at z-half cell [10, 20]: series -> arithmetic mean of rho
    assert r33[1, 1, 1] == pytest.approx(0.4 * 4.0 + 0.6 * 1.0)
    # rho11 at node z=10: dual z-cell [5, 15]: parallel -> harmonic of rho
    sig = 0.9 * 0.25 + 0.1 * 1.0
    assert r11[1, 1, 1] == pytest.approx(1.0 / sig)
    assert r22[1, 1, 1] == pytest.approx(1.0 / sig)
    # homogeneous regions are untouched
    assert r11[0, 2, 2] == pytest.approx(4.0) and r33[3, 0, 0] == pytest.approx(1.0)


def test_point_stencils():
    w = configs.plain_forward()
    st = F.make_setup(w, fp=2.0)
    # x = -2000 lies on an E1 half node: Kronecker weights in x
    b, wts = T.point_stencil(st.axes, (-2000.0, 0.0, 0.0), (1, 0, 0), 2)
    assert np.allclose(wts[0], [0, 1, 0, 0])
    xh = T.half_nodes(st.axes[0])
    assert xh[b[0] + 1] == -2000.0
    # off-node: partition of unity and symmetric bracketing
    b, wts = T.point_stencil(st.axes, (13.0, -27.0, 41.0), (0, 0, 1), 2)
    assert np.allclose(wts.sum(axis=1), 1.0)
    assert st.axes[0][b[0] + 1] <= 13.0 < st.axes[0][b[0] + 2]
    # dual volume of a uniform 100 m grid
    assert np.allclose(T.dual_volume(st.axes, 0, b, 2), 1e6)


def test_dft_phases_and_source_spectrum():
    dt, nt = 0.01, 50
    wp = T.omega_prime([0.5], 2 * np.pi)[0]
    phE, phH = T.dft_phases([0.5], 2 * np.pi, dt, nt)
    assert phE[0, 0] == pytest.approx(np.exp(1j * wp * dt))
    assert phH[3, 0] == pytest.approx(np.exp(1j * wp * 3.5 * dt))
    assert abs(phE[-1, 0]) < abs(phE[0, 0])          # Im w' > 0: decaying kernel
    s = np.zeros(nt)
    s[4] = 1.0
    assert T.source_spectrum(s, [0.5], 2 * np.pi, dt)[0] == pytest.approx(phH[4, 0])
    # w' = (1+i) sqrt(w w0) and (w/w')^2 = -i w/(2 w0)
    w = 2 * np.pi * 0.5
    assert (w / wp) ** 2 == pytest.approx(-1j * w / (2 * 2 * np.pi))
