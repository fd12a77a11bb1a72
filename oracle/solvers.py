"""Iterative solvers of the discrete system eq. (13) (oracle).

Both follow textbook definitions.  The paper cites conjugate gradients
(its Section 5 choice, valid when A0 is softer than every phase so that the
system is positive definite) and the fixed-point scheme of Moulinec and
Suquet, which it does not write out.
"""
from __future__ import annotations

import math

import numpy as np

from . import operator as op


def cg(pb: op.Problem, p, tol: float = 1e-10, maxit: int = 1000, history=None):
    """Hestenes--Stiefel conjugate gradients on L tau = b, tau_0 = 0.

    Euclidean inner product over voxels and components (Mandel in
    elasticity); stops when the recursive residual satisfies
    ||r||_2 <= tol ||b||_2.  Returns a dict with the solution, the number of
    operator applications and the relative true residual of the result.
    ``history`` (a list) receives the relative recursive residual after each
    iteration."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return {"tau": x, "iters": 0, "rel_res": 0.0}
    r = b.copy()
    pdir = r.copy()
    rr = op.dot(r, r)
    it = 0
    while it < maxit:
        q = op.apply(pb, pdir)
        it += 1
        alpha = rr / op.dot(pdir, q)
        x += alpha * pdir
        r -= alpha * q
        rr_new = op.dot(r, r)
        if history is not None:
            history.append(math.sqrt(rr_new) / bnorm)
        if math.sqrt(rr_new) <= tol * bnorm:
            break
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
    true_r = b - op.apply(pb, x)
    return {"tau": x, "iters": it, "rel_res": math.sqrt(op.dot(true_r, true_r)) / bnorm}


def basic(pb: op.Problem, p, tol: float = 1e-10, maxit: int = 10000, history=None):
    """Basic fixed-point scheme: tau_{k+1} = (A - A0)(p - Gamma tau_k) on I0,
    tau_0 = 0, i.e. the fixed point of eq. (13) written as
    tau = (A - A0)(p - Gamma tau).

    The residual of iterate k is b - L tau_k = (A - A0)^{-1}(tau_{k+1} - tau_k)
    on I0; the loop stops once its norm is at most tol ||b|| and returns
    tau_{k+1}.  ``iters`` counts applications of Gamma."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    m = op.mask(pb)
    tau = np.zeros_like(b)
    if bnorm == 0.0:
        return {"tau": tau, "iters": 0, "rel_res": 0.0}
    pcol = np.asarray(p, dtype=np.float64).reshape((-1,) + (1,) * pb.d)
    it = 0
    rel = math.inf
    while it < maxit:
        g = op.gamma_apply(pb, tau)
        it += 1
        new = m * op.local_apply(pb, pcol - g, which="direct")
        res = m * (op.local_apply(pb, new) - op.local_apply(pb, tau))
        rel = math.sqrt(op.dot(res, res)) / bnorm
        tau = new
        if history is not None:
            history.append(rel)
        if rel <= tol:
            break
    return {"tau": tau, "iters": it, "rel_res": rel}
