"""Pin of the oracle's discrete adjoint (the gradient of the misfit
chi = 1/2 sum |log(G/G_obs)|^2 with respect to log sigma of every cell):
central finite differences of the FP64 forward, with dt, the step count and
the CPML tables held at the reference model's values, on a non-uniform grid
with CPML, E and H data at two frequencies, cells in the interior and on the
model faces (whose values are replicated into the padding), all three
staggered conductivity arrays."""
import numpy as np
import pytest

from oracle import forward as F
from workloads import configs


@pytest.fixture(scope="module")
def case():
    w = configs.small_case(seed=31, shape=(17, 16, 15), nb=4, ne=3, nt=300, nrec=5,
                           freqs=(0.5, 1.5), nu_axes=(False, True, True))
    st = F.make_setup(w, 2.0 * np.sqrt(1.5))
    s = np.float32(1.3)
    wo = w.with_(rho11=w.rho11 * s, rho22=w.rho22 * s, rho33=w.rho33 * s)
    G_obs, _ = F.forward(wo, dt_override=st.dt)
    chi, g, _ = F.misfit_gradient(w, G_obs, frozen=st, ckpt=37)
    return w, st, G_obs, chi, g


CELLS = [(1, 7, 12, 16), (0, 2, 13, 16), (0, 4, 13, 7), (0, 12, 4, 6), (1, 8, 1, 0),
         (2, 11, 13, 9), (2, 0, 5, 5), (1, 14, 15, 3)]


@pytest.mark.parametrize("cell", CELLS)
def test_adjoint_matches_central_differences(case, cell):
    w, st, G_obs, chi, g = case
    c, k, j, i = cell
    rho = [w.rho11, w.rho22, w.rho33]
    h = 1e-3
    vals = []
    for sgn in (+1, -1):
        r2 = [a.copy() for a in rho]
        r2[c][k, j, i] = np.float32(rho[c][k, j, i] * np.exp(-sgn * h))   # log sigma +/- h
        chi_s = F.misfit_gradient(w.with_(rho11=r2[0], rho22=r2[1], rho33=r2[2]), G_obs,
                                  frozen=st, with_gradient=False)[0]
        vals.append((r2[c][k, j, i], chi_s))
    (rp, cp), (rm, cm) = vals
    fd = (cp - cm) / (np.log(rm) - np.log(rp))
    assert abs(g[c, k, j, i] - fd) <= 2e-5 * abs(fd) + 1e-12 * chi, (g[c, k, j, i], fd)


def test_gradient_vanishes_at_zero_residual(case):
    w, st, _, _, _ = case
    G, _ = F.forward(w)
    chi, g, _ = F.misfit_gradient(w, G, frozen=st)
    assert chi < 1e-20 and np.max(np.abs(g)) < 1e-12


def test_fold_padding_is_the_adjoint_of_replication():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 4, 6))
    y = rng.normal(size=(5 + 6, 4 + 6, 6 + 6))
    lhs = np.sum(np.pad(x, 3, mode="edge") * y)
    rhs = np.sum(x * F.fold_padding(y, 3))
    assert lhs == pytest.approx(rhs, rel=1e-12)
