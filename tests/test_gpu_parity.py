"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Every case runs the same seeded synthetic inputs through both and applies
the rule of tests/parity.py: <= 1e-4 relative amplitude and <= 0.1 degree
phase for every result above the floor.  Cases span several 64 x 4 tiles
and z chunks with ragged tails, r = 1..4, non-uniform axes, CPML on and
off, all three source components in one batched launch, all six receiver
channels, both accumulator modes; plus run-to-run and tile-shape bitwise
determinism, the full-size marine layered workload against a stored oracle
result, and the error paths that need a device.
"""
import json
import os

import numpy as np
import pytest

from oracle import analytic as A
from oracle import forward as F
from tests.parity import compare
from workloads import configs

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "marine_layered_oracle.json")
LARGE_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_marine_oracle.json")


@pytest.fixture(scope="module")
def emm():
    from paper_2304_00233_amd import emm as E
    return E


def _run(emm, w, **opt):
    print(f"[gpu] {w.name} nsrc={len(w.sources)} nrec={len(w.receivers)} rd={w.rd} "
          f"nt={w.nt} opts={opt}", flush=True)
    G, info = emm.forward_workload(w, **opt)
    return G, info


def _check(emm, w, label, **opt):
    G_o, info_o = F.forward(w)
    G_g, info_g = _run(emm, w.with_(nt=info_o["nt"]), **opt)
    rep = compare(G_g, G_o, w.channels)
    print(f"[parity] {label}: {rep}", flush=True)
    assert info_g["dt"] == pytest.approx(info_o["dt"], rel=1e-12)
    assert (info_g["n1pad"], info_g["n2pad"], info_g["n3pad"]) == tuple(info_o["n_pad"])
    assert info_g["nt"] == info_o["nt"]
    if opt.get("ce_table") == 1:
        assert info_g["ce_table"] == 1
    assert rep["ok"], rep
    return G_g, G_o, rep


def test_plain_forward_48cube(emm):
    w = configs.plain_forward_offaxis()
    G_g, _, _ = _check(emm, w, "plain_forward_48cube")
    # the GPU result is also close to the analytic whole-space dipole
    rec = w.receivers[21:]
    E, _ = A.dipole_fields([0, 0, 0], [1, 0, 0], rec, 1.0, 1.0)
    assert np.max(np.abs(G_g[0, 21:, 0, 0] / E[:, 0] - 1)) < 0.02


SMALL = [
    dict(seed=0),
    dict(seed=1, rd=1, shape=(30, 27, 25), nu_axes=(True, True, True)),
    dict(seed=2, rd=3, shape=(33, 31, 29), nu_axes=(False, True, True)),
    dict(seed=3, rd=4, shape=(41, 35, 33), nb=8),
    dict(seed=4, shape=(70, 13, 11), nb=4, nrec=9),                  # two x tiles, ragged
    dict(seed=5, shape=(23, 22, 21), nb=0, ne=3, nt=400),            # no CPML
    dict(seed=6, nsrc=3, src_comp=(0, 1, 2), shape=(31, 30, 26)),    # batched sources
    dict(seed=7, rd=2, shape=(26, 24, 40), freqs=(0.3, 0.9, 2.7, 5.0)),
]


@pytest.mark.parametrize("kw", SMALL, ids=[f"s{c['seed']}" for c in SMALL])
def test_small_cases(emm, kw):
    # r = 2, 3, 4 and the batched sources read dt/eps in the compact form,
    # the rest the FP32 arrays
    w = configs.small_case(**kw)
    _check(emm, w, w.name, ce_table=1 if kw["seed"] in (0, 2, 3, 6) else 0)


def test_kahan_fp32_accumulators(emm):
    w = configs.small_case(seed=8, shape=(29, 27, 25), nt=300)
    _, _, rep = _check(emm, w, "kahan", dft_mode=1)


@pytest.mark.parametrize("rd", [1, 2, 3, 4])
def test_bitwise_determinism_runs_and_tiles(emm, rd):
    """Runs, z chunks, both tile widths (64 x 4 and 32 x 8 columns) and both
    dt/eps forms give the same results bit for bit, at every stencil order."""
    w = configs.small_case(seed=9, shape=(40, 30, 37), nt=200, rd=rd)
    G1, _ = _run(emm, w)
    G2, _ = _run(emm, w)
    G3, i3 = _run(emm, w, tile_kz=3)
    G4, i4 = _run(emm, w, tile_x=32, tile_kz=7, ce_table=1)
    G5, i5 = _run(emm, w, tile_x=64, ce_table=0)
    G6, i6 = _run(emm, w, tile_x=32, ce_table=0, nontemporal=1)
    # register-blocked 64 x 8 and 64 x 16 tiles (two and four rows per wavefront;
    # the 30-row y extent leaves a ragged last tile of each)
    G7, i7 = _run(emm, w, tile_rows=2, ce_table=1, tile_kz=5)
    G8, i8 = _run(emm, w, tile_rows=4, ce_table=0, nontemporal=1)
    G9, i9 = _run(emm, w, tile_rows=4, ce_table=1)
    # one z chunk per column (a request beyond the depth is clamped to it)
    G10, i10 = _run(emm, w, tile_kz=1000, tile_x=32)
    assert i10["tile_kz"] == i10["n3pad"] - 2 * rd
    assert i3["tile_kz"] == 3 and (i4["tile_x"], i5["tile_x"], i6["tile_x"]) == (32, 64, 32)
    assert (i4["ce_table"], i5["ce_table"], i6["ce_table"]) == (1, 0, 0)
    assert (i7["tile_rows"], i8["tile_rows"], i9["tile_rows"]) == (2, 4, 4)
    assert (i7["tile_x"], i8["tile_x"], i9["tile_x"]) == (64, 64, 64)
    for G in (G2, G3, G4, G5, G6, G7, G8, G9, G10):
        assert np.array_equal(G1, G)


def test_batched_equals_single_sources(emm):
    w = configs.small_case(seed=10, nsrc=4, shape=(28, 26, 24), nt=200)
    Gb, ib = _run(emm, w)
    # the blocks of the four sources in either order within the launches
    Gs1, is1 = _run(emm, w, src_order=1)
    assert (ib["src_order"], is1["src_order"]) == (0, 1)
    assert np.array_equal(Gb, Gs1)
    for s in range(4):
        Gs, _ = _run(emm, w.with_(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1]))
        assert np.array_equal(Gb[s:s + 1], Gs)


def test_source_groups_equal_one_loop(emm):
    """emm_forward running the sources in groups (2 + 2 + 1 time loops, one
    after another) gives the one-loop batch bit for bit, and checks every
    source before it runs the first group."""
    w = configs.small_case(seed=14, nsrc=5, src_comp=(0, 1, 2, 0, 2), shape=(28, 26, 24), nt=160)
    G1, i1 = _run(emm, w, src_group=-1)
    G2, i2 = _run(emm, w, src_group=2, profile=1)
    G3, i3 = _run(emm, w)                  # automatic: this small grid fits all five
    assert (i1["src_group"], i2["src_group"], i3["src_group"]) == (5, 2, 5)
    assert np.array_equal(G1, G2) and np.array_equal(G1, G3)
    assert i2["e_launches"] > 0 and i2["forward_ms"] > 0
    bad = w.sources.copy()
    bad[4] = [1e6, 0.0, 0.0]
    with emm.Model(w, src_group=2) as m:
        with pytest.raises(emm.EmmError) as e:
            m.forward(sources=bad)
        assert e.value.status == -4


def test_convergence_stop_matches_oracle(emm):
    """The lowest-frequency convergence stop: the GPU stops at the same
    check as the oracle (measure 1.6e-4 at step 1100, 2.4e-5 at 1200 for
    tolerance 1e-4), with direct launches and with graphs of 50 steps, and
    the stopped run equals a fixed run of that many steps bitwise."""
    w = configs.small_case(seed=61, shape=(24, 22, 20), nb=5, nt=6000, nrec=4, freqs=(0.5, 1.5))
    G_o, info_o = F.forward(w, converge_tol=1e-4, converge_every=100)
    for graph in (0, 50):
        G_g, info = _run(emm, w, converge_tol=1e-4, converge_every=100, graph_steps=graph)
        assert info["converged"] == 1 and info["nt"] == info_o["nt_done"][0]
        rep = compare(G_g, G_o, w.channels)
        print(f"[parity] convergence stop at {info['nt']} (graph {graph}): {rep}", flush=True)
        assert rep["ok"], rep
    G_f, info_f = _run(emm, w.with_(nt=info["nt"]))
    assert info_f["converged"] == 0
    assert np.array_equal(G_g, G_f)


@pytest.mark.parametrize("kw", [dict(seed=70, shape=(37, 29, 23)),
                                dict(seed=71, rd=1, shape=(70, 13, 11), nb=4),
                                dict(seed=72, rd=4, shape=(30, 27, 25), nb=5),
                                dict(seed=73, rd=3, nsrc=3, shape=(33, 31, 24))],
                         ids=["r2", "r1_ragged", "r4", "r3_three_sources"])
def test_fused_step_equals_half_steps(emm, kw):
    """One launch per time step (E recomputed on the halo, ping-pong
    buffers, lagged E-channel DTFT) gives the two half-step kernels' results
    bit for bit: direct launches, graph replays and another z chunk."""
    w = configs.small_case(nt=230, **kw)
    G0, i0 = _run(emm, w)
    G1, i1 = _run(emm, w, fused=1)
    G2, i2 = _run(emm, w, fused=1, graph_steps=16, tile_kz=5)
    assert (i0["fused"], i1["fused"], i2["fused"]) == (0, 1, 1)
    assert np.array_equal(G0, G1)
    assert np.array_equal(G0, G2)
    if len(w.sources) > 1:                    # one fused time loop per source
        G3, i3 = _run(emm, w, fused=1, src_group=1)
        assert i3["src_group"] == 1 and np.array_equal(G0, G3)


def test_nontemporal_hint_is_bitwise_neutral(emm):
    w = configs.small_case(seed=12, shape=(30, 26, 22), nt=120)
    G0, i0 = _run(emm, w, nontemporal=0)
    G1, i1 = _run(emm, w, nontemporal=1)
    assert (i0["nontemporal"], i1["nontemporal"]) == (0, 1)
    assert np.array_equal(G0, G1)


@pytest.mark.parametrize("nval", [256, 257])
def test_compact_dt_eps_is_bitwise_neutral(emm, nval):
    """The E step reading dt/eps as per-cell byte indices into a table of the
    model's distinct values gives the FP32 arrays' results bit for bit.  The
    three components draw every cell's resistivity from one pool of nval
    values, each used at least once: at 256, the table size, the compact
    form is used (ce_table = 1); at 257 the model has only the FP32 arrays.
    The automatic choice (autotuned or by size) gives the same results."""
    w = configs.small_case(seed=13, shape=(30, 26, 22), nt=120)
    rng = np.random.default_rng(nval)
    n = w.rho11.size
    vals = np.exp(rng.uniform(np.log(0.5), np.log(5.0), nval)).astype(np.float32)
    assert len(np.unique(vals)) == nval

    def draw(all_values):
        idx = rng.integers(0, nval, n)
        if all_values:
            idx[:nval] = np.arange(nval)
        return np.ascontiguousarray(vals[rng.permutation(idx)].reshape(w.rho11.shape))

    w = w.with_(rho11=draw(True), rho22=draw(False), rho33=draw(False))
    G0, i0 = _run(emm, w, ce_table=0)
    G1, i1 = _run(emm, w, ce_table=1)
    G2, _ = _run(emm, w, tile_kz=-1)
    assert (i0["ce_table"], i1["ce_table"]) == (0, int(nval <= 256))
    if nval <= 256:
        assert i1["e_bytes"] < i0["e_bytes"]
    assert np.array_equal(G0, G1)
    assert np.array_equal(G0, G2)


def test_multi_model_batch_equals_single_forwards(emm):
    """Models of uneven sizes, step counts and source counts in one hipGraph
    (32 steps per block: every job ends with a ragged remainder, and the
    graph is re-captured as jobs finish) give bitwise the results of their
    own forwards; the middle job is also held against the oracle."""
    ws = [configs.small_case(seed=40, shape=(30, 26, 22), nt=150),
          configs.small_case(seed=41, shape=(37, 29, 23), nt=230, nsrc=2),
          configs.small_case(seed=42, shape=(24, 22, 20), nt=100, rd=1)]
    singles = [_run(emm, w)[0] for w in ws]
    models = [emm.Model(w) for w in ws]
    one = emm.Model(ws[0], src_group=1)      # as the first job: one job per graph
    try:
        print("[gpu] forward_models of 3 models", flush=True)
        outs = emm.forward_models(models, graph_steps=32)
        infos = [m.info() for m in models]
        print("[gpu] forward_models of 3 models, one graph each", flush=True)
        outs1 = emm.forward_models([one] + models[1:], graph_steps=32)
        infos1 = [m.info() for m in [one] + models[1:]]
    finally:
        for m in models + [one]:
            m.close()
    for a, b, c in zip(outs, singles, outs1):
        assert np.array_equal(a, b) and np.array_equal(c, b)
    assert [i["nt"] for i in infos] == [150, 230, 100]
    assert [i["src_group"] for i in infos] == [3, 3, 3]      # small grids share one group
    assert [i["src_group"] for i in infos1] == [1, 1, 1]
    # graphs of 200 steps: two jobs are shorter (direct launches only)
    models = [emm.Model(w) for w in ws]
    try:
        print("[gpu] forward_models of 3 models, 200-step graphs", flush=True)
        outs2 = emm.forward_models(models, graph_steps=200)
    finally:
        for m in models:
            m.close()
    for a, b in zip(outs2, singles):
        assert np.array_equal(a, b)
    G_o, _ = F.forward(ws[1])
    rep = compare(outs[1], G_o, ws[1].channels)
    print(f"[parity] multi-model job 1: {rep}", flush=True)
    assert rep["ok"], rep


def test_more_frequencies_than_lanes(emm):
    """70 frequencies: lane l of a DTFT wavefront updates frequencies l and
    l + 64; both accumulator modes against the oracle."""
    freqs = tuple(np.geomspace(0.2, 5.0, 70))
    w = configs.small_case(seed=15, shape=(24, 22, 20), nt=300, freqs=freqs, nrec=4)
    G_o, info_o = F.forward(w)
    for mode in (0, 1):
        G_g, _ = _run(emm, w.with_(nt=info_o["nt"], dft_mode=mode))
        rep = compare(G_g, G_o, w.channels)
        print(f"[parity] 70 frequencies dft_mode={mode}: {rep}", flush=True)
        assert rep["ok"], rep
        assert np.all(np.abs(G_g[..., 64:]) > 0)


@pytest.mark.parametrize("comp", [0, 2])
def test_stretched_whole_space(emm, comp):
    """The z axis stretched by 1.2 around the source (injection control
    volume on a non-uniform axis): GPU against the oracle, and the GPU result
    against the analytic whole-space dipole."""
    w = configs.stretched_whole_space(comp=comp)
    G_g, _, _ = _check(emm, w, f"stretched whole space, dipole along axis {comp}")
    d = [0.0, 0.0, 0.0]
    d[comp] = 1.0
    E, _ = A.dipole_fields([0.0, 0.0, 0.0], d, w.receivers, 1.0, 1.0)
    ratio = G_g[0, :, 0, 0] / E[:, comp]
    assert np.max(np.abs(np.abs(ratio) - 1.0)) <= 0.03
    assert np.max(np.abs(np.degrees(np.angle(ratio)))) <= 2.0


def test_reciprocity_marine_stretched_z(emm):
    """Source and receiver swapped between a point in the water and one 500 m
    into the sediment on the marine z axis with CPML: each run against the
    oracle, and the GPU pair reciprocal to the oracle's level (5.2e-4)."""
    w, a, b = configs.marine_reciprocity()
    G_ab, _, _ = _check(emm, w, "marine reciprocity a -> b")
    G_ba, _, _ = _check(emm, w.with_(sources=b[None, :], receivers=a[None, :]),
                        "marine reciprocity b -> a")
    err = abs(G_ab.ravel()[0] / G_ba.ravel()[0] - 1.0)
    print(f"[parity] GPU reciprocity on the stretched marine axis: {err:.3e}", flush=True)
    assert err <= 1e-2


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="marine oracle result not generated")
def test_marine_layered_full_size_vs_stored_oracle(emm):
    g = json.load(open(GOLDEN))
    G_o = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    w = configs.marine_layered(nt=g["nt"])
    # the benchmark's launch configuration: autotuned tiles and hint, 64-step
    # graph replays, sampled timing launches
    G_g, info = _run(emm, w, tile_kz=-1, graph_steps=64, profile=1)
    assert info["dt"] == pytest.approx(g["dt"], rel=1e-12)
    rep = compare(G_g, G_o, g["channels"])
    print(f"[parity] marine_layered_128x128x96 full size: {rep}", flush=True)
    assert rep["ok"], rep


@pytest.mark.slow
def test_large_marine_full_size_r4_batched(emm):
    """The 400 x 400 x 200 grid (438 x 438 x 238 padded cells) at 8th order
    with all 8 sources in one batched launch, the compensated FP32 DTFT,
    autotuned tiles and graph replays, as the large-grid benchmark runs it.
    The run is cut to 160 steps with a 25 Hz wavelet peak (pulse centre at
    step 124) so the FP64 oracle finishes in about a minute; source 3 is
    held against it."""
    nt, fp, s = 160, 25.0, 3
    w = configs.large_marine(nt=nt, rd=4, nsrc=8)
    G, info = _run(emm, w, tile_kz=-1, graph_steps=64, wavelet_fpeak=fp)
    G_o, info_o = F.forward(w.with_(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1]),
                            threads=min(16, os.cpu_count() or 1), nt=nt, fpeak=fp)
    assert info["dt"] == pytest.approx(info_o["dt"], rel=1e-12)
    rep = compare(G[s:s + 1], G_o, w.channels)
    print(f"[parity] large_marine r=4 8 sources, source {s}: {rep}", flush=True)
    assert rep["ok"], rep


@pytest.mark.skipif(not os.path.exists(LARGE_GOLDEN), reason="large-grid oracle result not generated")
@pytest.mark.timeout(900)
def test_large_marine_full_length_vs_stored_oracle(emm):
    """One source of the 400 x 400 x 200 grid at 8th order over the full
    automatic step count with the default wavelet, against the stored FP64
    oracle result: batched with a second source in the large-grid
    benchmark's launch configuration (58 planes per block, 32 x 8 tiles,
    source-slowest order, no nontemporal hints, compact dt/eps, compensated
    FP32 DTFT, 64-step graph replays with sampled timing launches), then
    alone with FP64 accumulators.  Most results are above the noise floor
    at this length, and both runs hold every one of them to the tolerance."""
    g = json.load(open(LARGE_GOLDEN))
    G_o = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    s = g["source_index"]
    w = configs.large_marine(rd=4, nsrc=g["sources_in_workload"]).with_(nt=g["nt"])
    pair = [s, (s + 1) % len(w.sources)]
    w2 = w.with_(sources=w.sources[pair], src_comp=w.src_comp[pair])
    G2, info = _run(emm, w2, tile_kz=58, tile_x=32, src_order=1, nontemporal=0, ce_table=1,
                    graph_steps=64, profile=1)
    assert info["dt"] == pytest.approx(g["dt"], rel=1e-12) and info["nt"] == g["nt"]
    rep = compare(G2[0:1], G_o, g["channels"])
    print(f"[parity] large_marine full length, source {s}, Kahan FP32 DTFT, batched: {rep}", flush=True)
    assert rep["compared"] >= 0.5 * G_o.size, rep
    assert rep["ok"], rep
    w1 = w.with_(sources=w.sources[s:s + 1], src_comp=w.src_comp[s:s + 1], dft_mode=0)
    G1, _ = _run(emm, w1, tile_kz=-1, graph_steps=64)
    rep64 = compare(G1, G_o, g["channels"])
    print(f"[parity] large_marine full length, source {s}, FP64 DTFT: {rep64}", flush=True)
    assert rep64["compared"] >= 0.5 * G_o.size, rep64
    assert rep64["ok"], rep64


def test_error_paths_on_device(emm):
    w = configs.small_case(seed=11, shape=(21, 20, 19), nt=50)
    with emm.Model(w) as m:
        with pytest.raises(emm.EmmError) as e:
            m.forward(receivers=np.array([[1e6, 0.0, 0.0]]))
        assert e.value.status == -4
        with pytest.raises(emm.EmmError) as e:
            m.forward(freqs=np.array([-1.0]))
        assert e.value.status == -5
        with pytest.raises(emm.EmmError) as e:
            m.forward(chan_mask=0)
        assert e.value.status == -1
        # empty acquisitions: no receiver, no source, no frequency
        with pytest.raises(emm.EmmError) as e:
            m.forward(receivers=np.zeros((0, 3)))
        assert e.value.status == -1
        with pytest.raises(emm.EmmError) as e:
            m.forward(sources=np.zeros((0, 3)), src_comp=np.zeros(0, dtype=np.int32))
        assert e.value.status == -1
        with pytest.raises(emm.EmmError) as e:
            m.forward(freqs=np.zeros(0))
        assert e.value.status == -5
        G = m.forward()                     # the model is still usable
        assert np.all(np.isfinite(G))
    # an unstable time step (forced from the host) ends non-finite, reported as such
    probe = emm.Model(w)
    dt = probe.info()["dt"]
    probe.close()
    with emm.Model(w.with_(nt=400), dt_override=3.0 * dt / 0.99, allow_unstable=1) as m:
        with pytest.raises(emm.EmmError) as e:
            m.forward()
        assert e.value.status == -7


def test_profile_counters(emm):
    w = configs.small_case(seed=12, shape=(30, 28, 26), nt=120)
    G, info = _run(emm, w, profile=1)
    assert info["e_launches"] == 120 // 16 + 1 and info["h_launches"] == info["e_launches"]
    assert 0 < info["e_kernel_ms"] < info["forward_ms"]
    assert 0 < info["h_kernel_ms"] < info["forward_ms"]
    G2, info2 = _run(emm, w, profile=1, graph_steps=16)     # events inside the graphs
    assert np.array_equal(G, G2)
    # 7 blocks of 16: block 0 direct with 4 timed steps, then a tail of 8 with 1
    assert info2["e_launches"] == 4 + 1 and info2["e_kernel_ms"] > 0


def test_autotuned_tiles_are_bitwise_identical(emm):
    w = configs.small_case(seed=13, shape=(44, 30, 61), nt=120, nsrc=2)
    G0, i0 = _run(emm, w)
    G1, i1 = _run(emm, w, tile_kz=-1)
    assert i1["tile_kz"] > 0
    assert np.array_equal(G0, G1)


def test_graph_replays_are_bitwise_identical(emm):
    """K steps captured in one hipGraph and replayed (device step counter),
    plus a tail of direct launches; every replay is checked through the
    final result against direct launches, twice in a row."""
    w = configs.small_case(seed=14, shape=(33, 29, 27), nt=120)
    G0, _ = _run(emm, w)
    with emm.Model(w, graph_steps=16) as m:
        G1 = m.forward()
        G2 = m.forward()
    assert np.array_equal(G0, G1) and np.array_equal(G0, G2)


def test_roofline_bytes_follow_the_algorithmic_count(emm):
    """The bytes the roofline divides by: per launch of one source, the E step
    reads H and E and writes E (36 B per padded cell) plus dt/eps (12 B as
    three FP32 arrays, 4 B in the compact form), the H step 36 B, both + 16 B
    per CPML slab cell per axis (two memory variables read and written);
    for S sources the benchmark's count reads the FP32 dt/eps once:
    (36 S + 12) N and 36 S N.  Recomputed here from the padded grid."""
    import bench
    w = configs.small_case(seed=16, shape=(27, 23, 21), nb=6, nsrc=3, nt=40)
    for ce in (0, 1):
        _, info = _run(emm, w, ce_table=ce)
        n = (info["n1pad"], info["n2pad"], info["n3pad"])
        N = float(n[0] * n[1] * n[2])
        ncpml = sum(2.0 * w.nb * N / na for na in n)
        assert info["ce_table"] == ce
        assert info["cells"] == N
        assert info["e_bytes"] == (40.0 if ce else 48.0) * N + 16.0 * ncpml
        assert info["h_bytes"] == 36.0 * N + 16.0 * ncpml
        kb = bench.kernel_bytes(info, 3)
        assert kb["e_8d"] == pytest.approx((36.0 * 3 + 12.0) * N + 16.0 * 3 * ncpml, rel=1e-12)
        assert kb["e_moved"] == pytest.approx((36.0 * 3 + (4.0 if ce else 12.0)) * N + 16.0 * 3 * ncpml,
                                              rel=1e-12)
        assert kb["h"] == pytest.approx(3 * (36.0 * N + 16.0 * ncpml), rel=1e-12)
