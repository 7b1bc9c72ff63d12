"""torch.autograd.Function around the forward modelling and its discrete
adjoint.

    G = green(log_sigma, workload)     # complex128 [nsrc][nrec][nchan][nfreq]

log_sigma is a float64 tensor [3][n3][n2][n1] (log conductivity behind
rho11, rho22, rho33), on the CPU or on the GPU.  Backward hands torch's
complex cotangent (dL/dRe G + i dL/dIm G, torch's convention for real
losses) to emm_gradient, which runs the hand-written adjoint kernels on the
GPU from the checkpoints the forward kept.  dt is frozen at the value of the
model the Function was first built for (pass dt_override) because it depends
on the largest resistivity; the CPML profile likewise depends on the face
resistivities.  torch is used for the tensors, the stream and the autograd
graph only; all numerics run in libemm.

Device tensors: this module imports torch before libemm, so a process that
imports it (or torch) first holds one HIP runtime, torch's, which libemm
shares; then the library runs on torch's current stream of the tensor's
device and G and the gradient come back as tensors on that device.  The
model itself crosses the C boundary as host arrays (emm_create validates and
uploads it), and G, the cotangent and the gradient cross it as host arrays
of the acquisition's and the model's size.
"""
from __future__ import annotations

import numpy as np
import torch

from . import emm


def _library_stream(device: torch.device):
    """The hipStream_t of torch's current stream on `device` (None on the
    CPU); refuses a process where libemm and torch hold different HIP
    runtimes (libemm imported before torch)."""
    if device.type != "cuda":
        return None
    rt = emm.hip_runtimes()
    if len(rt) != 1:
        raise RuntimeError("libemm and torch run on different HIP runtimes in this process "
                           f"({rt}): import torch before paper_2304_00233_amd.emm")
    return torch.cuda.current_stream(device).cuda_stream


class GreenFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, log_sigma: torch.Tensor, w, dt_override: float, checkpoint_every: int):
        stream = _library_stream(log_sigma.device)
        rho = np.exp(-log_sigma.detach().cpu().numpy()).astype(np.float32)
        wm = w.with_(rho11=rho[0], rho22=rho[1], rho33=rho[2])
        model = emm.Model(wm, dt_override=dt_override, checkpoint_every=checkpoint_every,
                          allow_unstable=0)
        G = model.forward(stream=stream)
        ctx.model = model
        ctx.device = log_sigma.device
        ctx.stream = stream
        return torch.from_numpy(G).to(log_sigma.device)

    @staticmethod
    def backward(ctx, gG: torch.Tensor):
        model = ctx.model
        g, _, _ = model.gradient(g_bar=gG.detach().cpu().numpy(), stream=ctx.stream)
        model.close()
        return torch.from_numpy(g).to(ctx.device), None, None, None


def green(log_sigma: torch.Tensor, w, dt_override: float = 0.0, checkpoint_every: int = 50):
    return GreenFunction.apply(log_sigma, w, dt_override, checkpoint_every)


def log_sigma_of(w) -> torch.Tensor:
    """The workload's conductivity as the [3][n3][n2][n1] log-sigma tensor."""
    return torch.from_numpy(-np.log(np.stack([w.rho11, w.rho22, w.rho33]).astype(np.float64)))
