"""The stored plain-forward 48^3 result that the benchmark compares the GPU
against (tests/golden/plain_forward_48cube_oracle.json) is what the oracle
computes now: the same step count, dt and Green's functions."""
import json
import os

import numpy as np

from oracle import forward as F
from workloads import configs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "plain_forward_48cube_oracle.json")


def test_plain_golden_is_current():
    g = json.load(open(GOLDEN))
    G, info = F.forward(configs.plain_forward_offaxis())
    assert info["nt"] == g["nt"] and info["dt"] == g["dt"]
    G_s = (np.array(g["re"]) + 1j * np.array(g["im"])).reshape(g["shape"])
    assert np.allclose(G, G_s, rtol=1e-12, atol=0.0)
