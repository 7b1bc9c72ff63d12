"""Pins of the oracle's lowest-frequency convergence stop (Sections 3.5 and
4.1: the run ends once the lowest frequency's DTFT at the corners of the
interior stops changing between checks).

* Stopping is a truncation of the same time loop: the stopped run's Green's
  functions equal those of a fixed-length run of the reported step count,
  to the last bit.
* The reported step is the first check whose measure (largest corner change
  over largest corner magnitude) is at or below the tolerance.
* A tight tolerance reproduces a much longer run to about that tolerance.
"""
import numpy as np

from oracle import forward as F
from workloads import configs


def _case():
    return configs.small_case(seed=61, shape=(24, 22, 20), nb=5, nt=6000, nrec=4, freqs=(0.5, 1.5))


def test_stop_is_a_truncation_of_the_same_loop():
    w = _case()
    G_c, info = F.forward(w, converge_tol=1e-4, converge_every=100)
    nd = info["nt_done"][0]
    assert nd % 100 == 0 and nd < w.nt
    G_f, _ = F.forward(w.with_(nt=nd))
    assert np.array_equal(G_c, G_f)


def test_reported_step_is_the_first_check_below_tolerance():
    w = _case()
    st = F.make_setup(w, 2.0 * np.sqrt(1.5 * w.f0))
    rep = {}
    F.run_source(st, w.nt, w.sources[0], 0, w.receivers, w.channels, w.freqs,
                 converge_tol=1e-4, converge_every=100, report=rep)
    m = rep["measure"]
    assert len(m) == rep["nt_done"] // 100
    assert np.all(m[:-1] > 1e-4) and m[-1] <= 1e-4


def test_tight_tolerance_matches_a_long_run():
    w = _case()
    G_c, info = F.forward(w, converge_tol=1e-8, converge_every=100)
    G_l, _ = F.forward(w.with_(nt=info["nt_done"][0] + 2000))
    assert np.max(np.abs(G_c - G_l)) <= 1e-5 * np.max(np.abs(G_l))
