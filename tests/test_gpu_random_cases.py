"""Seeded random small cases through the C ABI against the FP64 oracle:
grid sizes, stencil order, CPML thickness, stretched axes, sources (count
and dipole direction), receivers, frequencies and the launch options (tile
width, z chunk, compact dt/eps, nontemporal hints, source order, graph
replays, DTFT accumulators) drawn together, so that combinations no
hand-written case names still meet the tolerance."""
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
