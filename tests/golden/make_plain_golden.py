"""Write the FP64 oracle's Green's functions for the plain-forward 48^3 model
(1 ohm-m whole space, 100 m cells, x-dipole at the origin, 21 inline and 6
off-axis receivers, 1 Hz, all six channels) to
plain_forward_48cube_oracle.json, with the analytic whole-space dipole
fields at the same receivers (the receiver on the source has none).  Calls only oracle/ and the shared
input synthesis; the HIP path is compared against this file on the GPU."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import analytic as A  # noqa: E402
from oracle import forward as F  # noqa: E402
from workloads import configs   # noqa: E402


def main(threads=None):
    w = configs.plain_forward_offaxis()
    t = time.time()
    G, info = F.forward(w, threads=threads)
    secs = time.time() - t
    src = w.sources[0]
    r = np.linalg.norm(w.receivers - src, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):     # the receiver on the source
        E, H = A.dipole_fields(src, [1.0, 0.0, 0.0], w.receivers, float(w.freqs[0]), 1.0)
    E[r == 0] = np.nan
    H[r == 0] = np.nan
    an = np.concatenate([E, H], axis=1)               # [nrec][6]: Ex Ey Ez Hx Hy Hz
    out = {
        "workload": w.name,
        "source": "oracle.forward (FP64) and oracle.analytic.dipole_fields, written by "
                  "tests/golden/make_plain_golden.py",
        "nt": int(info["nt"]), "dt": float(info["dt"]), "n_pad": list(info["n_pad"]),
        "freqs": [float(f) for f in w.freqs], "channels": w.channels,
        "shape": list(G.shape),
        "re": [float(v) for v in G.real.ravel()],
        "im": [float(v) for v in G.imag.ravel()],
        "receiver_distance_m": [float(v) for v in r],
        "analytic_re": [None if np.isnan(v) else float(v) for v in an.real.ravel()],
        "analytic_im": [None if np.isnan(v) else float(v) for v in an.imag.ravel()],
        "oracle_seconds": secs,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plain_forward_48cube_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, info, secs)


if __name__ == "__main__":
    main()
