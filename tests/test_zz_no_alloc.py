"""emm_forward_noalloc (every per-call device buffer in the library's static
128 MiB workspace; no hipMalloc, no events, no graphs) against emm_forward,
through the C ABI: two calls in a row, the second with a smaller input (fewer
sources, receivers and frequencies), each equal bit for bit to emm_forward on
the same model (the same kernels and launch shape, direct launches), the
first also against the FP64 oracle; a forward too large for the workspace is
refused with EMM_ERR_OOM and leaves the model usable."""
import numpy as np
import pytest

from oracle import forward as F
from tests.parity import compare
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emm():
    from paper_2304_00233_amd import emm as E
    return E


def test_noalloc_forward_matches_forward(emm):
    w = configs.small_case(seed=50, shape=(34, 30, 28), nt=220, nsrc=3, src_comp=(0, 1, 2),
                           nrec=6, freqs=(0.4, 1.1, 2.3))
    print(f"[gpu] no-alloc forward, {w.name}, 3 sources", flush=True)
    with emm.Model(w) as m:
        G1 = m.forward(noalloc=True)
        G_ref = m.forward()
        assert np.array_equal(G1, G_ref)
        # the second call: one source, 3 receivers, 1 frequency; the workspace
        # still holds the first call's (larger) contents
        kw = dict(sources=w.sources[1:2], src_comp=w.src_comp[1:2], receivers=w.receivers[:3],
                  freqs=w.freqs[1:2])
        print("[gpu] no-alloc forward, second call, 1 source", flush=True)
        G2 = m.forward(noalloc=True, **kw)
        G2_ref = m.forward(**kw)
        assert G2.shape == (1, 3, 6, 1)
        assert np.array_equal(G2, G2_ref)
        # and the first input again after the smaller one
        G3 = m.forward(noalloc=True)
        assert np.array_equal(G3, G_ref)
    G_o, _ = F.forward(w)
    rep = compare(G1, G_o, w.channels)
    print(f"[parity] no-alloc forward vs oracle: {rep}", flush=True)
    assert rep["ok"], rep


def test_noalloc_refuses_what_does_not_fit(emm):
    """A 150^3 grid (184^3 padded cells, rows padded to 192): its fields alone
    are 156 MB, beyond the 128 MiB workspace."""
    w = configs.uniform_cube(150, nt=8)
    print(f"[gpu] no-alloc size limit, {w.name}", flush=True)
    with emm.Model(w) as m:
        with pytest.raises(emm.EmmError) as e:
            m.forward(noalloc=True)
        assert e.value.status == -8 and "static workspace" in str(e.value)
        G = m.forward()                 # the model is still usable
        assert np.all(np.isfinite(G))
    wa = configs.small_case(seed=51, shape=(20, 19, 18), nt=20).with_(airwave=True)
    with emm.Model(wa) as m:
        with pytest.raises(emm.EmmError) as e:
            m.forward(noalloc=True)
        assert e.value.status == -1
