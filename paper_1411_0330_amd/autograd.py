"""The homogenised matrix as a differentiable function of per-voxel moduli.

``homogenized_gram(coef, ctx, loads)`` returns G_lm = p_l . A*_h p_m for the
loads p_l (rows of ``loads``) of the medium given by the per-voxel isotropic
coefficients ``coef`` (a, or (K, mu)).  The forward pass is one batched solve
of eq. (13) in the HIP library; the backward pass is ``lsh_gradient``: the
operator of eq. (13) is symmetric, so dG_lm/dA_beta = (1/V) sym(eps_l (x) eps_m)
with the strain estimates eps = p - Gamma tau of the solved loads, and no
adjoint solve is needed.  Everything upstream of ``coef`` (a parametrisation
such as E = 1 + 9 sigmoid(theta)) is ordinary torch autograd.
"""
from __future__ import annotations

import numpy as np
import torch


class HomogenizedGram(torch.autograd.Function):
    @staticmethod
    def forward(fctx, coef, lsh_ctx, loads, solver, tol, maxit):
        lsh_ctx.set_voxel_moduli(coef.detach())
        report = lsh_ctx.solve(loads, solver=solver, tol=tol, maxit=maxit)
        S = lsh_ctx.effective()                      # rows A*_h p_l
        G = loads @ S.T                              # G_lm = p_l . A*_h p_m
        fctx.lsh = lsh_ctx
        fctx.stamp = lsh_ctx.solves
        fctx.report = report
        fctx.coef_meta = (coef.dtype, coef.device)
        return torch.tensor(G, dtype=torch.float64, device=coef.device)

    @staticmethod
    def backward(fctx, gG):
        if fctx.lsh.solves != fctx.stamp:
            raise RuntimeError("the solver context was used again after this forward pass; "
                               "its solution no longer matches the graph")
        W = gG.detach().to("cpu", torch.float64).numpy()
        g = fctx.lsh.gradient(W)
        dtype, device = fctx.coef_meta
        return g.to(device=device, dtype=dtype), None, None, None, None, None


def homogenized_gram(coef, ctx, loads, solver="cg", tol=1e-10, maxit=2000):
    """G (nload x nload, float64, on coef's device) with autograd support."""
    loads = np.ascontiguousarray(np.atleast_2d(loads), dtype=np.float64)
    return HomogenizedGram.apply(coef, ctx, loads, solver, tol, maxit)


def young_to_bulk_shear(E, nu):
    """(K, mu) of an isotropic medium from Young's modulus and Poisson's ratio."""
    return E / (3.0 * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))
