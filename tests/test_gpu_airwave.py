"""The air boundary above the sea surface (Section 3.3) on the GPU, through
the C ABI, against the FP64 oracle (whose ghost fills are pinned in
tests/test_oracle_airwave.py): small ragged cases at r = 1 to 4 (r - 1 E
ghost planes, r H ghost half planes), several sources in one
launch bitwise equal to one at a time, with either form of the ghost-fill
transforms (hipFFT or the direct kernels), the entry points that
refuse the air boundary, and the full-size shallow-water workload against
a stored oracle result."""
import json
import os

import numpy as np
import pytest

from oracle import forward as F
from tests.parity import compare
from workloads import configs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "shallow_marine_air_oracle.json")


@pytest.fixture(scope="module")
def emm():
    from paper_2304_00233_amd import emm as E
    return E


def _air_case(seed, shape, rd, nb, nsrc=1, nt=500):
    return configs.small_case(seed=seed, shape=shape, rd=rd, nb=nb, ne=rd + 2, nt=nt, nsrc=nsrc,
                              nu_axes=(False, False, True)).with_(airwave=True)


# the ghost-fill transforms: 2 = hipFFT, 3 = the direct kernels (planes up
# to 512 points per axis, each split once as n = f m; the padded planes
# here: 57 x 49 = (3 x 19) x (7 x 7), 52 x 49 = (4 x 13) x (7 x 7),
# 40 x 84 = (5 x 8) x (7 x 12), 46 x 44 = (2 x 23) x (4 x 11) and, at
# r = 3, 52 x 47 = (4 x 13) x 47 (prime: whole-line sums))
AIR = [2, 3]


@pytest.mark.parametrize("air", AIR, ids=["fft", "direct"])
@pytest.mark.parametrize("seed,shape,rd,nb", [(50, (37, 29, 23), 2, 6), (51, (30, 27, 25), 4, 5),
                                              (52, (26, 70, 19), 1, 4), (53, (32, 27, 24), 3, 5)],
                         ids=["r2", "r4", "r1_ragged", "r3"])
def test_air_boundary_matches_oracle(emm, seed, shape, rd, nb, air):
    w = _air_case(seed, shape, rd, nb)
    G_o, info_o = F.forward(w)
    print(f"[gpu] air {w.name} rd={rd} nt={w.nt} transforms {air}", flush=True)
    G_g, info_g = emm.forward_workload(w, airwave=air)
    rep = compare(G_g, G_o, w.channels)
    print(f"[parity] air r={rd} transforms {air}: {rep}", flush=True)
    assert info_g["air_transform"] == air - 1
    assert info_g["dt"] == pytest.approx(info_o["dt"], rel=1e-12)
    assert rep["ok"], rep
    if rd == 2:
        # the boundary is live here (the r = 4 case's receivers hardly see the
        # top within its 500 steps): without it the answer differs
        G_n, _ = emm.forward_workload(w.with_(airwave=False))
        assert np.max(np.abs(G_n - G_g)) > 1e-3 * np.max(np.abs(G_g))


def test_air_transform_chosen_by_plane_size(emm):
    """Option 1 picks the FP64 direct kernels while both padded horizontal
    axes have at most 512 points (here 57 x 49) and hipFFT above (533)."""
    w = _air_case(50, (37, 29, 23), 2, 6, nt=20)
    _, i = emm.forward_workload(w)
    assert i["air_transform"] == 2
    w2 = _air_case(57, (513, 29, 23), 2, 6, nt=20)
    _, i2 = emm.forward_workload(w2)
    assert i2["air_transform"] == 1
    with pytest.raises(emm.EmmError):
        emm.forward_workload(w2, airwave=3)


def test_wide_plane_fp64_fills(emm):
    """A 137 x 49 plane (137 prime: the direct sums run over whole rows) with
    the source near one end: the surface field spans orders of magnitude
    along x, and a transform's rounding is relative to the plane's largest
    value.  The FP64 direct fills keep every result within the tolerance;
    hipFFT's FP32 transforms were measured at 2.0e-4 in amplitude on this
    case (reported here, held only to 1e-3)."""
    w = _air_case(56, (117, 29, 23), 2, 6, nt=300)
    G_o, _ = F.forward(w)
    G_d, i_d = emm.forward_workload(w)
    assert i_d["air_transform"] == 2
    rep = compare(G_d, G_o, w.channels)
    print(f"[parity] air 137 x 49, FP64 direct fills: {rep}", flush=True)
    assert rep["ok"], rep
    G_f, _ = emm.forward_workload(w, airwave=2)
    rep_f = compare(G_f, G_o, w.channels)
    print(f"[parity] air 137 x 49, hipFFT fills: {rep_f}", flush=True)
    assert rep_f["amp_max"] <= 1e-3, rep_f


@pytest.mark.parametrize("air", AIR, ids=["fft", "direct"])
def test_air_boundary_batched_sources_bitwise(emm, air):
    w = _air_case(53, (28, 26, 22), 2, 5, nsrc=3, nt=200)
    Gb, _ = emm.forward_workload(w, airwave=air)
    for s in range(3):
        Gs, _ = emm.forward_workload(w.with_(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1]),
                                     airwave=air)
        assert np.array_equal(Gb[s:s + 1], Gs)


def test_air_boundary_source_groups_bitwise(emm):
    """Three sources in groups of 2 + 1 (the ghost-fill plans are rebuilt when
    the group size changes) give the one-loop batch bit for bit."""
    w = _air_case(54, (28, 26, 22), 2, 5, nsrc=3, nt=200)
    G1, i1 = emm.forward_workload(w, src_group=-1)
    G2, i2 = emm.forward_workload(w, src_group=2, graph_steps=16)
    assert (i1["src_group"], i2["src_group"]) == (3, 2)
    assert np.array_equal(G1, G2)


@pytest.mark.parametrize("air", AIR, ids=["fft", "direct"])
def test_air_boundary_graph_replays_are_bitwise_identical(emm, air):
    """The ghost fills (hipFFT transforms and spectral kernels, or the direct
    transform kernels) captured in the step graphs and replayed 12 times per
    forward give the direct launches' result bit for bit, twice in a row."""
    w = _air_case(55, (28, 26, 22), 2, 5, nt=200)
    G0, i0 = emm.forward_workload(w, airwave=air)
    with emm.Model(w, graph_steps=16, airwave=air) as m:
        G1 = m.forward()
        G2 = m.forward()
    assert np.array_equal(G0, G1) and np.array_equal(G0, G2)


def test_air_direct_fills_with_every_tile_shape_are_bitwise(emm):
    """The FP64 direct fills with the stencils on 32- and 64-wide tiles,
    register-blocked tiles, another z chunking and graph replays, two
    sources in one launch: the same bits."""
    w = _air_case(58, (41, 29, 23), 2, 6, nsrc=2, nt=200)
    G0, i0 = emm.forward_workload(w, airwave=3, tile_x=32)
    assert i0["air_transform"] == 2
    for kw in (dict(tile_x=64), dict(tile_rows=2), dict(tile_rows=4), dict(tile_x=32, graph_steps=16),
               dict(tile_x=64, tile_kz=5)):
        G, _ = emm.forward_workload(w, airwave=3, **kw)
        assert np.array_equal(G0, G), kw


def test_air_boundary_refused_by_gradient_and_batch(emm):
    w = _air_case(54, (21, 20, 19), 2, 4, nt=50)
    with emm.Model(w) as m:
        G = m.forward()
        with pytest.raises(emm.EmmError) as e:
            m.gradient(g_obs=G)
        assert e.value.status == -1
        with pytest.raises(emm.EmmError):
            emm.forward_models([m])


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="shallow-water oracle result not generated")
def test_shallow_marine_full_size_vs_stored_oracle(emm):
    g = json.load(open(GOLDEN))
    G_o = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    w = configs.shallow_marine(nt=g["nt"])
    print(f"[gpu] {w.name} nt={g['nt']}", flush=True)
    for air in (1, 2):
        G_g, info = emm.forward_workload(w, tile_kz=-1, graph_steps=64, airwave=air)
        assert info["dt"] == pytest.approx(g["dt"], rel=1e-12)
        assert info["air_transform"] == (2 if air == 1 else 1)
        rep = compare(G_g, G_o, g["channels"])
        print(f"[parity] shallow_marine_air full size, transforms {info['air_transform']}: {rep}",
              flush=True)
        assert rep["ok"], rep
