"""torch.autograd.Function whose backward is the library's reverse RK4 sweep.

``expectation_of_params(theta, spec)`` returns Re <psi0| A(T) |psi0> as a
torch scalar that depends on theta = (K[N], chi[i<j], Delta[N], gamma1[N],
gamma_phi[N]); its gradient comes from hgf_grad (discrete adjoint kernels),
not from autograd tracing.  The value and the gradient are real for a
Hermitian observable; an imaginary part above ``imag_tol`` (relative to the
largest magnitude) raises, since the real part alone would then not be the
caller's expectation value.

``spec`` holds the system shape and the operator: ``cutoff``, ``n_th``,
``state``, ``t_total``, ``dt``, ``factors`` or ``sparse``, and optionally
``checkpoint_every`` (default 100) and ``imag_tol`` (default 1e-12).
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


def _real_part(z, scale: float, tol: float, what: str):
    im = float(np.max(np.abs(np.imag(z)))) if np.size(z) else 0.0
    if im > tol * max(scale, 1e-300):
        raise ValueError(f"{what} has an imaginary part {im:.3e} (the observable is not Hermitian); "
                         "expectation_of_params returns real values only")
    return np.real(z)


class HgfExpectation(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, spec: dict):
        th = theta.detach().cpu().double().numpy()
        system = _system_from_theta(th, spec)
        tol = float(spec.get("imag_tol", 1e-12))
        if ctx.needs_input_grad[0]:
            value, g = hgf.grad(system, spec["state"], spec["t_total"], spec["dt"], factors=spec.get("factors"),
                                sparse=spec.get("sparse"), checkpoint_every=spec.get("checkpoint_every", 100))
            gr = _real_part(g, float(np.max(np.abs(g))) if g.size else 0.0, tol, "dJ/dtheta")
            ctx.save_for_backward(torch.as_tensor(np.ascontiguousarray(gr), dtype=theta.dtype, device=theta.device))
        else:
            # no gradient requested: the forward evolve alone (FP64, as hgf_grad)
            op = hgf.map_operator(system, factors=spec.get("factors"), sparse=spec.get("sparse"), precision="fp64")
            hgf.evolve(op, spec["t_total"], spec["dt"])
            value = hgf.expectation(op, spec["state"])
        v = float(_real_part(value, abs(value), tol, "the expectation value"))
        return torch.tensor(v, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None


def expectation_of_params(theta: torch.Tensor, spec: dict) -> torch.Tensor:
    return HgfExpectation.apply(theta, spec)
