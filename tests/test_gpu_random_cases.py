"""Seeded random small cases through the C ABI against the FP64 oracle:
grid sizes, stencil order, CPML thickness, stretched axes, sources (count
and dipole direction), receivers, frequencies and the launch options (tile
width, z chunk, compact dt/eps, nontemporal hints, source order, graph
replays, DTFT accumulators) drawn together, so that combinations no
hand-written case names still meet the tolerance: forwards, misfit
gradients and forwards with the air boundary."""
import numpy as np
import pytest

from oracle import forward as F
from tests.parity import compare
from workloads import configs

pytestmark = pytest.mark.gpu


def _draw(i):
    rng = np.random.default_rng(20260 + i)
    rd = int(rng.integers(1, 5))
    shape = tuple(int(v) for v in rng.integers(14, 46, 3))
    nsrc = int(rng.integers(1, 4))
    w = configs.small_case(
        seed=300 + i, shape=shape, rd=rd, nb=int(rng.choice([0, 3, 6, 8])),
        nt=int(rng.integers(200, 401)), nu_axes=tuple(bool(b) for b in rng.integers(0, 2, 3)),
        nsrc=nsrc, nrec=int(rng.integers(3, 10)),
        freqs=tuple(np.sort(np.exp(rng.uniform(np.log(0.2), np.log(3.0), int(rng.integers(1, 5)))))),
        src_comp=tuple(int(c) for c in rng.integers(0, 3, nsrc)))
    opt = dict(tile_x=int(rng.choice([32, 64])), tile_kz=int(rng.choice([0, 3, 7, 1000])),
               ce_table=int(rng.integers(0, 2)), nontemporal=int(rng.integers(0, 2)),
               src_order=int(rng.integers(0, 2)), graph_steps=int(rng.choice([0, 16, 64])))
    return w.with_(dft_mode=int(rng.integers(0, 2))), opt


@pytest.fixture(scope="module")
def emm():
    from paper_2304_00233_amd import emm as E
    return E


@pytest.mark.parametrize("i", range(12))
def test_random_case_matches_oracle(emm, i):
    w, opt = _draw(i)
    print(f"[gpu] random case {i}: {w.name} nb={w.nb} sources={len(w.sources)} "
          f"comp={list(w.src_comp)} freqs={len(w.freqs)} dft_mode={w.dft_mode} {opt}", flush=True)
    G_o, info_o = F.forward(w)
    G_g, info_g = emm.forward_workload(w, **opt)
    assert info_g["dt"] == pytest.approx(info_o["dt"], rel=1e-12)
    rep = compare(G_g, G_o, w.channels)
    print(f"[parity] random case {i}: {rep}", flush=True)
    assert rep["ok"], rep


def _draw_gradient(i):
    rng = np.random.default_rng(20360 + i)
    rd = int(rng.integers(1, 5))
    nsrc = int(rng.integers(1, 3))
    w = configs.small_case(
        seed=400 + i, shape=tuple(int(v) for v in rng.integers(14, 30, 3)), rd=rd,
        nb=int(rng.choice([0, 3, 5])), ne=rd + 1, nt=int(rng.integers(250, 401)),
        nu_axes=(False, True, True), nsrc=nsrc, nrec=5, freqs=(0.5, 1.5),
        src_comp=tuple(int(c) for c in rng.integers(0, 3, nsrc)))
    opt = dict(tile_x=int(rng.choice([32, 64])), checkpoint_every=int(rng.choice([0, 23, 50])))
    return w, opt


@pytest.mark.parametrize("i", range(6))
def test_random_gradient_matches_oracle(emm, i):
    """The misfit gradient of seeded random cases (data from the model with
    every resistivity times 1.3) against the oracle's adjoint: relative L2
    within 1e-4, or within three times the gradient's own FP32 rounding
    noise where that is larger.  The noise is the larger change of the GPU
    gradient when every resistivity is nudged by +2^-20 or -2^-20 (exact
    changes of ~1e-6; one nudge alone can land an order of magnitude under
    the noise: 1.2e-5 and 1.2e-4 on case 4).  A draw whose noise exceeds
    1e-2 is skipped, since no comparison can hold it (case 5: 0.19)."""
    w, opt = _draw_gradient(i)
    print(f"[gpu] random gradient case {i}: {w.name} nb={w.nb} sources={len(w.sources)} {opt}",
          flush=True)
    s = np.float32(1.3)
    st = F.make_setup(w, 2.0 * np.sqrt(max(w.freqs)))
    G_obs, _ = F.forward(w.with_(rho11=w.rho11 * s, rho22=w.rho22 * s, rho33=w.rho33 * s),
                         dt_override=st.dt)
    chi_o, g_o, _ = F.misfit_gradient(w, G_obs, frozen=st)
    with emm.Model(w, **opt) as m:
        dt = m.info()["dt"]
        g, _, chi = m.gradient(g_obs=G_obs)
    noise = 0.0
    for e in (1.0 + 2.0 ** -20, 1.0 - 2.0 ** -20):
        e = np.float32(e)
        with emm.Model(w.with_(rho11=w.rho11 * e, rho22=w.rho22 * e, rho33=w.rho33 * e),
                       dt_override=dt, **opt) as m:
            gn, _, _ = m.gradient(g_obs=G_obs)
        noise = max(noise, np.linalg.norm(gn - g) / np.linalg.norm(g))
    err = np.linalg.norm(g - g_o) / np.linalg.norm(g_o)
    print(f"[adjoint] random case {i}: rel L2 {err:.2e}, rounding noise {noise:.2e}, "
          f"chi {chi:.6e} oracle {chi_o:.6e}", flush=True)
    if noise > 1e-2:
        pytest.skip(f"ill-conditioned draw: FP32 rounding noise of the gradient {noise:.1e}")
    # chi sums |log(G/G_obs)|^2 over data down to ~1e-7 of the largest |G|
    # (FP32 fields): 1.3e-4 relative on case 0
    assert chi == pytest.approx(chi_o, rel=1e-3)
    assert err <= max(1e-4, 3.0 * noise)


def _draw_air(i):
    rng = np.random.default_rng(20460 + i)
    rd = int(rng.integers(1, 5))
    nsrc = int(rng.integers(1, 3))
    w = configs.small_case(
        seed=500 + i, shape=tuple(int(v) for v in rng.integers(16, 40, 3)), rd=rd,
        nb=int(rng.choice([3, 5, 6])), ne=rd + 2, nt=int(rng.integers(300, 501)),
        nu_axes=(False, False, bool(rng.integers(0, 2))), nsrc=nsrc, nrec=int(rng.integers(3, 8)),
        freqs=tuple(np.sort(np.exp(rng.uniform(np.log(0.3), np.log(2.0), int(rng.integers(1, 4)))))),
        src_comp=tuple(int(c) for c in rng.integers(0, 3, nsrc))).with_(airwave=True)
    opt = dict(airwave=int(rng.choice([2, 3])), tile_x=int(rng.choice([32, 64])),
               graph_steps=int(rng.choice([0, 16])), src_order=int(rng.integers(0, 2)))
    return w, opt


@pytest.mark.parametrize("i", range(4))
def test_random_air_case_matches_oracle(emm, i):
    """Seeded random cases with the air boundary (either ghost-fill
    transform) against the oracle."""
    w, opt = _draw_air(i)
    print(f"[gpu] random air case {i}: {w.name} nb={w.nb} sources={len(w.sources)} "
          f"comp={list(w.src_comp)} freqs={len(w.freqs)} {opt}", flush=True)
    G_o, info_o = F.forward(w)
    G_g, info_g = emm.forward_workload(w, **opt)
    assert info_g["dt"] == pytest.approx(info_o["dt"], rel=1e-12)
    rep = compare(G_g, G_o, w.channels)
    print(f"[parity] random air case {i}: {rep}", flush=True)
    assert rep["ok"], rep
