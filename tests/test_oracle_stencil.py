"""Pins of the oracle stepper's own stencil application (its C curl routines).

On a uniform grid the staggered operators have the symbol of the paper's
dispersion appendix: applied to exp(i k x) they multiply it by
(2i/dx) sum_l c_l sin((l - 1/2) k dx).  For a real cosine this gives
D cos(k x) = -(2/dx) S(k) sin(k x) at the derivative's own position, so a
wrong offset, a wrong staggering, a swapped table or a sign error in the curl
assembly fails here.  On a non-uniform grid the same curls must differentiate
cubic fields exactly (2r = 4 nodes).
"""
import numpy as np
import pytest

from oracle import forward as F
from oracle import tables as T
from workloads import configs, grids

STAG_E = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
STAG_H = ((0, 1, 1), (1, 0, 1), (1, 1, 0))


def _setup(w):
    return F.make_setup(w, fp=2.0)


def _coords(st, stag):
    """Broadcastable coordinate arrays (x, y, z) of a component on [z][y][x]."""
    out = []
    for a in range(3):
        xp = st.axes[a]
        c = np.concatenate([T.half_nodes(xp), [np.nan]]) if stag[a] else xp
        shape = [1, 1, 1]
        shape[2 - a] = len(c)
        out.append(c.reshape(shape))
    return out


def _update_mask(st):
    n1, n2, n3 = st.n_pad
    r = st.r
    m = np.zeros((n3, n2, n1), dtype=bool)
    m[r:n3 - r, r:n2 - r, r:n1 - r] = True
    return m


def _symbol(r, k, dx):
    from fractions import Fraction  # noqa: F401
    c = {1: [1.0], 2: [9 / 8, -1 / 24], 3: [75 / 64, -25 / 384, 3 / 640],
         4: [1225 / 1024, -245 / 3072, 49 / 5120, -5 / 7168]}[r]
    return sum(cl * np.sin((l + 0.5) * k * dx) for l, cl in enumerate(c))


@pytest.mark.parametrize("r", [1, 2, 4])
def test_plane_wave_symbol_curl_h_and_curl_e(r):
    n = 6 * r + 8
    d = (100.0, 70.0, 40.0)
    axes = [grids.uniform_axis(n, d[a], -0.5 * d[a] * (n - 1)) for a in range(3)]
    rho = np.ones((n, n, n), np.float32)
    w = configs.plain_forward().with_(x1=axes[0], x2=axes[1], x3=axes[2], rho11=rho,
                                      rho22=rho, rho33=rho, rd=r, nb=0, ne=r)
    st = _setup(w)
    k = [2 * np.pi / (7.3 * d[0]), 2 * np.pi / (5.1 * d[1]), 2 * np.pi / (9.7 * d[2])]
    S = [2.0 / d[a] * _symbol(r, k[a], d[a]) for a in range(3)]
    mask = _update_mask(st)

    # curl H: fields on the H grid
    X = [_coords(st, s) for s in STAG_H]
    cosf = lambda comp, a: np.cos(k[a] * X[comp][a])
    H1 = cosf(0, 1) + cosf(0, 2) + 0 * X[0][0]
    H2 = cosf(1, 0) + cosf(1, 2) + 0 * X[1][1]
    H3 = cosf(2, 0) + cosf(2, 1) + 0 * X[2][2]
    c1, c2, c3 = F.curl_apply(st, "H", *(np.nan_to_num(a) for a in (H1, H2, H3)))
    Y = [_coords(st, s) for s in STAG_E]
    sinf = lambda comp, a: np.sin(k[a] * Y[comp][a])
    e1 = -S[1] * sinf(0, 1) + S[2] * sinf(0, 2)     # D-y H3 - D-z H2
    e2 = -S[2] * sinf(1, 2) + S[0] * sinf(1, 0)     # D-z H1 - D-x H3
    e3 = -S[0] * sinf(2, 0) + S[1] * sinf(2, 1)     # D-x H2 - D-y H1
    for got, exp in ((c1, e1), (c2, e2), (c3, e3)):
        exp = np.broadcast_to(exp, got.shape)
        assert np.max(np.abs(got[mask] - exp[mask])) < 1e-12 * max(S)

    # curl E: fields on the E grid
    E1 = np.cos(k[1] * Y[0][1]) + np.cos(k[2] * Y[0][2]) + 0 * Y[0][0]
    E2 = np.cos(k[0] * Y[1][0]) + np.cos(k[2] * Y[1][2]) + 0 * Y[1][1]
    E3 = np.cos(k[0] * Y[2][0]) + np.cos(k[1] * Y[2][1]) + 0 * Y[2][2]
    c1, c2, c3 = F.curl_apply(st, "E", *(np.nan_to_num(a) for a in (E1, E2, E3)))
    s_ = lambda comp, a: np.sin(k[a] * X[comp][a])
    h1 = -S[1] * s_(0, 1) + S[2] * s_(0, 2)        # D+y E3 - D+z E2
    h2 = -S[2] * s_(1, 2) + S[0] * s_(1, 0)        # D+z E1 - D+x E3
    h3 = -S[0] * s_(2, 0) + S[1] * s_(2, 1)        # D+x E2 - D+y E1
    for got, exp in ((c1, h1), (c2, h2), (c3, h3)):
        exp = np.broadcast_to(exp, got.shape)
        assert np.max(np.abs(got[mask] - exp[mask])) < 1e-12 * max(S)


def test_nonuniform_cubic_fields_are_differentiated_exactly():
    w = configs.small_case(seed=5, shape=(13, 12, 11), rd=2, nb=0, ne=2,
                           nu_axes=(True, True, True))
    st = _setup(w)
    mask = _update_mask(st)
    X = [_coords(st, s) for s in STAG_H]
    Y = [_coords(st, s) for s in STAG_E]
    s = 1e-3
    # H3 = (s x)^3 + (s y)^3  ->  curlH2 = -3 s^3 x^2 at E2, curlH1 = 3 s^3 y^2 at E1
    H3 = np.nan_to_num((s * X[2][0]) ** 3 + (s * X[2][1]) ** 3 + 0 * X[2][2])
    z = np.zeros_like(H3)
    c1, c2, c3 = F.curl_apply(st, "H", z, z, H3)
    e1 = np.broadcast_to(3 * s ** 3 * Y[0][1] ** 2, c1.shape)
    e2 = np.broadcast_to(-3 * s ** 3 * Y[1][0] ** 2, c2.shape)
    assert np.allclose(c1[mask], e1[mask], rtol=1e-9, atol=1e-15)
    assert np.allclose(c2[mask], e2[mask], rtol=1e-9, atol=1e-15)
    assert np.max(np.abs(c3[mask])) < 1e-15
    # E2 = (s z)^3  ->  curlE1 = -D+z E2 = -3 s^3 z^2 at H1, curlE3 = D+x E2 = 0
    E2 = np.nan_to_num((s * Y[1][2]) ** 3 + 0 * Y[1][0] + 0 * Y[1][1])
    c1, c2, c3 = F.curl_apply(st, "E", z, E2, z)
    h1 = np.broadcast_to(-3 * s ** 3 * X[0][2] ** 2, c1.shape)
    assert np.allclose(c1[mask], h1[mask], rtol=1e-9, atol=1e-15)
    assert np.max(np.abs(c3[mask])) < 1e-15
