"""torch.autograd wrapper: eigenvalues of the damped-wave QEP as a
differentiable function of the per-element damping field.

forward : c_e (ne x ne, float64, on the device) -> lam (nev, complex128)
          through assemble + factor + Krylov-Schur in libriga
backward: dL/dc_e from riga_adjoint (the element-wise formula
          d lam/d c_e = -lam u^T M_e u / u^T (2 lam M + C) u); no finite differences.
"""
from __future__ import annotations

import numpy as np
import torch

from . import riga


class QEPEigenvalues(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c_elem, problem, sigma, nev, m, alpha, beta, seed):
        problem.assemble(alpha, beta, c_elem.detach())
        problem.factor(sigma)
        lam, X, eta, nconv, st = problem.eigs(nev, m, block=2, seed=seed)
        if nconv < nev:
            raise riga.RigaError(riga.RIGA_WARN_NOT_CONVERGED, "QEPEigenvalues.forward")
        ctx.problem = problem
        ctx.lam = lam
        ctx.save_for_backward(torch.view_as_real(X).contiguous())
        return torch.as_tensor(lam, dtype=torch.complex128, device=c_elem.device)

    @staticmethod
    def backward(ctx, grad_lam):
        (Xr,) = ctx.saved_tensors
        # torch's convention for a real loss of complex outputs: grad = dL/dRe + i dL/dIm
        g = grad_lam.detach().cpu().numpy().astype(np.complex128)
        grad_c = ctx.problem.adjoint(ctx.lam, torch.view_as_complex(Xr), g)
        return grad_c, None, None, None, None, None, None, None


def qep_eigenvalues(c_elem, problem, sigma, nev, m=0, alpha=0.0, beta=0.0, seed=0):
    """The nev eigenvalues nearest sigma (canonical order), differentiable in c_elem."""
    return QEPEigenvalues.apply(c_elem, problem, sigma, nev, m, alpha, beta, seed)
