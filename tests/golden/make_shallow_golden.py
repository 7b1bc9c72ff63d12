"""Write the FP64 oracle's Green's functions for the full-size shallow-water
workload with the air above the sea surface (128 x 128 x 80 nodes, 3
frequencies, 101 receivers, all six channels) to
shallow_marine_air_oracle.json.  Calls only oracle/ and the shared input
synthesis; the HIP path is compared against this file on the GPU."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import forward as F  # noqa: E402
from workloads import configs   # noqa: E402


def main(threads=None):
    w = configs.shallow_marine()
    t = time.time()
    G, info = F.forward(w, threads=threads)
    out = {
        "workload": w.name,
        "source": "oracle.forward (FP64), written by tests/golden/make_shallow_golden.py",
        "nt": int(info["nt"]), "dt": float(info["dt"]), "n_pad": list(info["n_pad"]),
        "freqs": [float(f) for f in w.freqs], "channels": w.channels,
        "shape": list(G.shape),
        "re": [float(v) for v in G.real.ravel()],
        "im": [float(v) for v in G.imag.ravel()],
        "oracle_seconds": time.time() - t,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shallow_marine_air_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, info, out["oracle_seconds"])


if __name__ == "__main__":
    main()
