"""Iterative solvers of the discrete system eq. (13) (oracle).

Each follows its textbook definition.  The paper cites conjugate gradients
(its Section 5 choice, valid when A0 is softer than every phase so that the
system is positive definite), SYMMLQ beside it (Section 1), and the
fixed-point scheme of Moulinec and Suquet, which it does not write out.
MINRES (the other Lanczos solver of symmetric indefinite systems) and the
Eyre--Milton scheme complete the set.
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


def minres(pb: op.Problem, p, tol: float = 1e-10, maxit: int = 1000, history=None):
    """MINRES of Paige and Saunders (1975) on L tau = b, tau_0 = 0, for the
    symmetric but possibly indefinite system that eq. (13) becomes when A0 is
    not softer than every phase.

    Lanczos vectors v_k (v_1 = b/||b||) tridiagonalise L; Givens rotations
    (c_k, s_k) reduce the tridiagonal matrix to upper bidiagonal form, and the
    iterate minimises ||b - L tau||_2 over the Krylov space.  With the
    rotation of the previous step applied to the new column (beta_k, alpha_k,
    beta_{k+1}):
        delta2_k = c_{k-1} delta1_k + s_{k-1} alpha_k
        gamma1_k = s_{k-1} delta1_k - c_{k-1} alpha_k
        eps_{k+1} = s_{k-1} beta_{k+1},  delta1_{k+1} = -c_{k-1} beta_{k+1}
        gamma2_k = hypot(gamma1_k, beta_{k+1}),  c_k = gamma1_k/gamma2_k,
        s_k = beta_{k+1}/gamma2_k,  t_k = c_k phi_{k-1},  phi_k = s_k phi_{k-1}
        w_k = (v_k - delta2_k w_{k-1} - eps_k w_{k-2}) / gamma2_k,
        tau_k = tau_{k-1} + t_k w_k,
    starting from c_0 = -1, s_0 = 0, delta1_1 = 0, phi_0 = ||b||; phi_k is the
    residual norm ||b - L tau_k||_2, which never increases.  ``history``
    receives phi_k / ||b|| after each iteration."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return {"tau": x, "iters": 0, "rel_res": 0.0}
    v_prev = np.zeros_like(b)
    v = b / bnorm
    w1 = np.zeros_like(b)      # w_{k-1}
    w2 = np.zeros_like(b)      # w_{k-2}
    beta = 0.0                 # beta_k (beta_1 v_0 = 0)
    c_prev, s_prev = -1.0, 0.0
    delta1 = 0.0
    eps = 0.0                  # eps_k
    phi = bnorm
    it = 0
    while it < maxit:
        q = op.apply(pb, v)
        it += 1
        alpha = op.dot(v, q)
        q = q - alpha * v - beta * v_prev
        beta_next = math.sqrt(op.dot(q, q))
        delta2 = c_prev * delta1 + s_prev * alpha
        gamma1 = s_prev * delta1 - c_prev * alpha
        eps_next = s_prev * beta_next
        delta1_next = -c_prev * beta_next
        gamma2 = math.hypot(gamma1, beta_next)
        if gamma2 == 0.0:
            break
        c, s = gamma1 / gamma2, beta_next / gamma2
        t = c * phi
        phi = s * phi
        w = (v - delta2 * w1 - eps * w2) / gamma2
        x += t * w
        if history is not None:
            history.append(abs(phi) / bnorm)
        if abs(phi) <= tol * bnorm or beta_next == 0.0:
            break
        v_prev, v = v, q / beta_next
        w2, w1 = w1, w
        beta, delta1, eps = beta_next, delta1_next, eps_next
        c_prev, s_prev = c, s
    true_r = b - op.apply(pb, x)
    return {"tau": x, "iters": it, "rel_res": math.sqrt(op.dot(true_r, true_r)) / bnorm}


def eyre_milton(pb: op.Problem, p, tol: float = 1e-10, maxit: int = 10000, history=None):
    """Eyre--Milton scheme (Eyre and Milton, 1999) in polarisation form.

    Adding (A - A0)^{-1} tau to both sides of eq. (13) after multiplication
    by 2 A0 shows that its solution is the fixed point of
        tau_{k+1} = (A - A0)(A + A0)^{-1} [tau_k + 2 A0 (p - Gamma tau_k)]
    on I0 (tau = 0 elsewhere), tau_0 = 0.  With 0 <= A0^{1/2} Gamma A0^{1/2}
    <= Id (truncated, filtered and consistent operators) the bracket is a
    reflection-like map of norm at most one, so the iteration contracts by
    max |(a - a0)/(a + a0)| (scalar, A0 = a0 Id) for any a0 > 0.  The residual
    of iterate k is (p - Gamma tau_k) - (A - A0)^{-1} tau_k on I0; the loop
    stops once its norm is at most tol ||b|| and returns tau_{k+1}."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    m = op.mask(pb)
    tau = np.zeros_like(b)
    if bnorm == 0.0:
        return {"tau": tau, "iters": 0, "rel_res": 0.0}
    delta, _, in_i0 = op.voxel_tables(pb)
    A0 = np.asarray(pb.A0, dtype=np.float64)
    M = np.zeros_like(delta)
    M[in_i0] = delta[in_i0] @ np.linalg.inv(delta[in_i0] + 2.0 * A0)
    pcol = np.asarray(p, dtype=np.float64).reshape((-1,) + (1,) * pb.d)
    c = pb.c
    it = 0
    rel = math.inf
    while it < maxit:
        u = pcol - op.gamma_apply(pb, tau)
        it += 1
        res = m * (u - op.local_apply(pb, tau))
        rel = math.sqrt(op.dot(res, res)) / bnorm
        y = (tau + 2.0 * np.einsum("ij,j...->i...", A0, u)).reshape(c, -1)
        tau = m * np.einsum("vij,jv->iv", M, y).reshape(tau.shape)
        if history is not None:
            history.append(rel)
        if rel <= tol:
            break
    return {"tau": tau, "iters": it, "rel_res": rel}


def symmlq(pb: op.Problem, p, tol: float = 1e-10, maxit: int = 1000, history=None, iterates=None):
    """SYMMLQ of Paige and Saunders (1975) on L tau = b, tau_0 = 0: the Krylov
    solver named beside CG in Section 1, for the symmetric indefinite system
    that eq. (13) becomes when A0 lies between the phases.

    The Lanczos process is that of MINRES.  An LQ factorisation T_k = Lbar_k Q_k
    of the tridiagonal matrix, by reflectors [c s; s -c] acting on columns
    (k, k+1), has the recurrences of MINRES's QR (T_k is symmetric):
        delta_k   = c_{k-1} dbar_k + s_{k-1} alpha_k
        gbar_k    = s_{k-1} dbar_k - c_{k-1} alpha_k
        eps_{k+1} = s_{k-1} beta_{k+1},  dbar_{k+1} = -c_{k-1} beta_{k+1}
        gamma_k   = hypot(gbar_k, beta_{k+1}),  c_k = gbar_k / gamma_k,
        s_k       = beta_{k+1} / gamma_k,
    from c_0 = -1, s_0 = 0, dbar_1 = 0.  Forward substitution in
    L z = ||b|| e_1 with num_k = [k = 1] ||b|| - delta_k z_{k-1} - eps_k z_{k-2}
    gives z_k = num_k / gamma_k and, with the last diagonal unrotated,
    zbar_k = num_k / gbar_k.  The rotated Lanczos vectors are
        w_k = c_k wbar_k + s_k v_{k+1},  wbar_{k+1} = s_k wbar_k - c_k v_{k+1},
    wbar_1 = v_1.  The SYMMLQ iterate x^L_k = x^L_{k-1} + z_k w_k has the
    least error ||tau* - x|| over x in L K_k(L, b); the CG point
    x^C_k = x^L_{k-1} + zbar_k wbar_k (Galerkin over K_k, defined when
    gbar_k != 0) has the residual |beta_{k+1}| |s_{k-1} z_{k-1} - c_{k-1} zbar_k|.

    The loop stops once that residual is at most tol ||b|| and returns the CG
    point; after maxit steps it returns the CG point of the last step (x^L_k if
    gbar_k = 0).  ``history`` receives the CG-point residual / ||b|| after each
    step; ``iterates`` (a list) receives (x^L_k, x^C_k or None) after each step
    that was not the last."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return {"tau": x, "iters": 0, "rel_res": 0.0}
    v_prev = np.zeros_like(b)
    v = b / bnorm
    wbar = v.copy()
    beta = 0.0
    c_prev, s_prev = -1.0, 0.0
    dbar, eps = 0.0, 0.0
    z1 = z2 = 0.0                      # z_{k-1}, z_{k-2}
    first = bnorm                      # right-hand side entry of this row
    out = None
    it = 0
    while it < maxit:
        q = op.apply(pb, v)
        it += 1
        alpha = op.dot(v, q)
        q = q - alpha * v - beta * v_prev
        bn = math.sqrt(op.dot(q, q))
        delta = c_prev * dbar + s_prev * alpha
        gbar = s_prev * dbar - c_prev * alpha
        eps_next, dbar_next = s_prev * bn, -c_prev * bn
        num = first - delta * z1 - eps * z2
        if gbar != 0.0:
            zbar = num / gbar
            xc = x + zbar * wbar
            rc = bn * abs(s_prev * z1 - c_prev * zbar)
        else:
            xc, rc = None, math.inf
        if history is not None:
            history.append(rc / bnorm)
        if rc <= tol * bnorm:
            out = xc
            break
        gamma = math.hypot(gbar, bn)
        if gamma == 0.0:               # beta_{k+1} = gbar_k = 0: singular on the Krylov space
            out = x
            break
        c, s = gbar / gamma, bn / gamma
        z = num / gamma
        vn = q / bn
        w = c * wbar + s * vn
        wbar = s * wbar - c * vn
        x = x + z * w
        if it == maxit:
            out = xc if xc is not None else x
            break
        if iterates is not None:
            iterates.append((x.copy(), None if xc is None else xc.copy()))
        v_prev, v = v, vn
        beta, dbar, eps = bn, dbar_next, eps_next
        c_prev, s_prev = c, s
        z2, z1 = z1, z
        first = 0.0
    if out is None:
        out = x
    true_r = b - op.apply(pb, out)
    return {"tau": out, "iters": it, "rel_res": math.sqrt(op.dot(true_r, true_r)) / bnorm}
