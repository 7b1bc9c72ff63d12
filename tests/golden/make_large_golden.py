"""Write the FP64 oracle's Green's functions for one source of the large
marine workload (400 x 400 x 200 nodes, 438 x 438 x 238 padded cells, 8th
order, 400 seafloor receivers, all six channels, 5 frequencies 0.1..2 Hz) at
its full automatic step count with the default wavelet, to
large_marine_oracle.json.  Calls only oracle/ and the shared input
synthesis; the HIP path (all 8 sources batched) is compared against this
file on the GPU.  Takes hours of CPU time (FP64, ~8 GB of memory)."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import forward as F  # noqa: E402
from workloads import configs   # noqa: E402

SOURCE = 3          # x = -1000 m on the towline of 8


def main(threads=None):
    w = configs.large_marine(rd=4, nsrc=8)
    w1 = w.with_(sources=w.sources[SOURCE:SOURCE + 1], src_comp=w.src_comp[SOURCE:SOURCE + 1])
    t = time.time()
    G, info = F.forward(w1, threads=threads)
    out = {
        "workload": w.name, "source_index": SOURCE, "sources_in_workload": len(w.sources),
        "source": "oracle.forward (FP64), written by tests/golden/make_large_golden.py",
        "nt": int(info["nt"]), "dt": float(info["dt"]), "n_pad": list(info["n_pad"]),
        "rd": w.rd, "freqs": [float(f) for f in w.freqs], "channels": w.channels,
        "shape": list(G.shape),
        "re": [float(v) for v in G.real.ravel()],
        "im": [float(v) for v in G.imag.ravel()],
        "oracle_seconds": time.time() - t, "threads": threads,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_marine_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(path, info, out["oracle_seconds"])


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else None)
