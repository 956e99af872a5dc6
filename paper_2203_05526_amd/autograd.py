"""torch.autograd.Function whose backward is the library's reverse RK4 sweep.

``expectation_of_params(theta, spec)`` returns Re <psi0| A(T) |psi0> as a
torch scalar that depends on theta = (K[N], chi[i<j], Delta[N], gamma1[N],
gamma_phi[N]); its gradient comes from hgf_grad (discrete adjoint kernels),
not from autograd tracing.
"""

from __future__ import annotations

import numpy as np
import torch

from . import hgf


def _system_from_theta(theta: np.ndarray, spec: dict) -> hgf.System:
    cutoff = spec["cutoff"]
    n = len(cutoff)
    kerr = theta[:n]
    npair = n * (n - 1) // 2
    chi = np.zeros((n, n))
    q = n
    for i in range(n):
        for j in range(i + 1, n):
            chi[i, j] = chi[j, i] = theta[q]
            q += 1
    det = theta[n + npair:2 * n + npair]
    g1 = theta[2 * n + npair:3 * n + npair]
    gphi = theta[3 * n + npair:4 * n + npair]
    return hgf.System(cutoff, det, kerr, chi, g1, gphi, spec["n_th"])


class HgfExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, spec: dict):
        th = theta.detach().cpu().double().numpy()
        system = _system_from_theta(th, spec)
        value, g = hgf.grad(system, spec["state"], spec["t_total"], spec["dt"], factors=spec.get("factors"),
                            sparse=spec.get("sparse"), checkpoint_every=spec.get("checkpoint_every", 100))
        ctx.save_for_backward(torch.from_numpy(g.real.copy()).to(theta.dtype))
        return torch.tensor(value.real, dtype=theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None


def expectation_of_params(theta: torch.Tensor, spec: dict) -> torch.Tensor:
    return HgfExpectation.apply(theta, spec)
