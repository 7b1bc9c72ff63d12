"""torch and libemm in one process on the GPU: with torch imported first,
libemm binds to torch's HIP runtime (one runtime mapped), the autograd
Function takes log-sigma as a cuda tensor, runs on torch's current stream,
returns G and the gradient as cuda tensors, and its gradient equals the one
of the host path (emm_gradient with the same misfit) to rounding.  Runs in a
fresh process, since this test process may have loaded libemm before torch."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def test_autograd_function_with_cuda_tensors_in_one_runtime():
    print("[gpu] torch + libemm in one process (subprocess)", flush=True)
    res = subprocess.run([sys.executable, os.path.join(HERE, "torch_shared_runtime_probe.py")],
                         capture_output=True, text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-3000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    print(f"[torch] {out}", flush=True)
    assert len(out["runtimes"]) == 1
    assert out["G_device"] == "cuda:0" and out["grad_device"] == "cuda:0"
    assert out["loss"] == pytest.approx(out["chi_ref"], rel=1e-9)
    assert out["grad_max_rel_diff"] <= 1e-9
