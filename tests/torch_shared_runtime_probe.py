"""Run in a fresh process by tests/test_gpu_torch.py: torch first, then the
autograd Function (which loads libemm onto torch's HIP runtime); the
Function's forward and backward with the model on the GPU (cuda:0, torch's
current stream) against the same gradient through the host path; prints one
JSON line."""
import json
import os
import sys

import torch  # noqa: F401  (first: libemm then shares torch's HIP runtime)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import forward as F  # noqa: E402
from paper_2304_00233_amd import autograd as AG  # noqa: E402
from paper_2304_00233_amd import emm  # noqa: E402
from workloads import configs  # noqa: E402


def main():
    w = configs.small_case(seed=38, shape=(21, 19, 17), rd=2, nb=4, ne=3, nt=200, nrec=5,
                           freqs=(0.5, 1.5), nu_axes=(False, True, True))
    s = np.float32(1.3)
    G_obs, _ = F.forward(w.with_(rho11=w.rho11 * s, rho22=w.rho22 * s, rho33=w.rho33 * s))
    with emm.Model(w) as m:
        dt = m.info()["dt"]
        g_ref, _, chi_ref = m.gradient(g_obs=G_obs)
    dev = torch.device("cuda:0")
    ls = AG.log_sigma_of(w).to(dev).requires_grad_(True)
    G = AG.green(ls, w, dt_override=dt, checkpoint_every=40)
    r = torch.log(G / torch.from_numpy(G_obs).to(dev))        # the misfit on the GPU
    loss = 0.5 * torch.sum(r.real ** 2 + r.imag ** 2)
    loss.backward()
    torch.cuda.synchronize()
    g = ls.grad.cpu().numpy()
    out = {"runtimes": emm.hip_runtimes(), "G_device": str(G.device),
           "grad_device": str(ls.grad.device), "loss": float(loss), "chi_ref": chi_ref,
           "grad_max_rel_diff": float(np.max(np.abs(g - g_ref)) / np.max(np.abs(g_ref)))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
