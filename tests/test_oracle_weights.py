"""Pins of the oracle's weight builders (Section 3.1; appendix on dispersion).

Fornberg's recursion must reproduce, on a uniform staggered grid, the
standard staggered first-derivative coefficients that the paper's appendix
names (c_i^+ = -c_{-i+1}^+ = c_i^- = c_i/dx); on arbitrary nodes it must
differentiate every polynomial of degree <= 2r-1 exactly (2r nodes), and
must NOT be exact for degree 2r on a non-uniform grid (a check that the test
is not vacuous).  Interpolation rows: partition of unity, Kronecker delta on
nodes, polynomial reproduction.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import tables as T
from oracle.weights import derivative_weights, fornberg, lagrange_weights

# standard staggered-grid coefficients c_1..c_r (tabulated by Fornberg 1988)
STAGGERED = {
    1: [Fraction(1)],
    2: [Fraction(9, 8), Fraction(-1, 24)],
    3: [Fraction(75, 64), Fraction(-25, 384), Fraction(3, 640)],
    4: [Fraction(1225, 1024), Fraction(-245, 3072), Fraction(49, 5120), Fraction(-5, 7168)],
}


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_uniform_staggered_coefficients(r):
    dx = 7.0
    nodes = dx * (np.arange(2 * r) - r + 0.5)        # half nodes around 0
    c = derivative_weights(0.0, nodes) * dx
    expect = [float(v) for v in STAGGERED[r]]
    # c for node offsets +1/2, +3/2, ... equal c_1, c_2, ...; mirrored with sign
    for i in range(r):
        assert c[r + i] == pytest.approx(expect[i], rel=1e-12, abs=1e-14)
        assert c[r - 1 - i] == pytest.approx(-expect[i], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_polynomial_exactness_nonuniform(r):
    rng = np.random.default_rng(r)
    nodes = np.cumsum(rng.uniform(0.3, 2.0, 2 * r))
    z = rng.uniform(nodes[0], nodes[-1])
    c = derivative_weights(z, nodes)
    for deg in range(2 * r):
        assert c @ nodes ** deg == pytest.approx(deg * z ** (deg - 1) if deg else 0.0,
                                                 rel=1e-9, abs=1e-9)
    err = c @ nodes ** (2 * r) - 2 * r * z ** (2 * r - 1)
    assert abs(err) > 1e-6                      # degree 2r is not reproduced


def test_fornberg_higher_derivative_sanity():
    nodes = np.array([-1.0, 0.0, 1.0])
    c = fornberg(0.0, nodes, 2)
    assert np.allclose(c[:, 2], [1.0, -2.0, 1.0])   # textbook second difference
    assert np.allclose(c[:, 1], [-0.5, 0.0, 0.5])


def test_lagrange_rows():
    rng = np.random.default_rng(7)
    nodes = np.cumsum(rng.uniform(0.5, 1.5, 6))
    for z in rng.uniform(nodes[0], nodes[-1], 5):
        w = lagrange_weights(z, nodes)
        assert w.sum() == pytest.approx(1.0, abs=1e-12)
        for deg in range(6):
            assert w @ nodes ** deg == pytest.approx(z ** deg, rel=1e-10)
    for j, z in enumerate(nodes):
        assert np.allclose(lagrange_weights(z, nodes), np.eye(6)[j], atol=1e-15)


@pytest.mark.parametrize("r", [2, 4])
def test_fd_tables_rows_on_padded_nonuniform_axis(r):
    from workloads import configs
    x3 = configs.marine_z_128x128x96()
    xp = T.pad_axis(x3, 10 + r + 5)
    cm, cp = T.fd_tables(xp, r)
    xh = T.half_nodes(xp)
    n = len(xp)
    for i in range(r, n - r):
        sm = xh[i - r:i + r] - xp[i]
        sp_ = xp[i - r + 1:i + r + 1] - xh[i]
        assert abs(cm[i].sum()) < 1e-12 * np.abs(cm[i]).sum()
        assert cm[i] @ sm == pytest.approx(1.0, abs=1e-10)
        assert abs(cp[i].sum()) < 1e-12 * np.abs(cp[i]).sum()
        assert cp[i] @ sp_ == pytest.approx(1.0, abs=1e-10)
    assert not cm[:r].any() and not cm[n - r:].any()
