"""Derivative of the discrete homogenised matrix with respect to the local
moduli (oracle).

Write eq. (13) as M tau_p = p on I0 with M = (A - A0)^{-1} + Gamma, a
symmetric operator (the Green table is real, symmetric and even in k).  The
estimate of Theorem 4 gives, for two loads p and q,

    q . A*_h p = q . A0 p + (1/V) sum_beta q . tau_p,beta .

Only the block (A_beta - A0)^{-1} of M depends on A_beta, and its derivative
is -(A_beta - A0)^{-1} dA_beta (A_beta - A0)^{-1}, so differentiating
M^{-1} gives

    d(q . A*_h p) / dA_beta = (1/V) eps_q,beta (x) eps_p,beta   (symmetrised),

with eps = (A_beta - A0)^{-1} tau_beta, which equals the strain estimate
p - (Gamma tau)_beta at the solution (Section 2.2.2).  The oracle uses the
strain estimate on every voxel.  For a weighted sum J = sum_lm W_lm
p_l . A*_h p_m over solved loads the per-voxel tensor is
(1/V) sum_lm W_lm sym(eps_l (x) eps_m).

Isotropic coefficients: scalar A_beta = a_beta I gives dJ/da = tr G; elastic
C = K m m^T + 2 mu (I - m m^T / 3) in Mandel form (m = (1,1,1,0,0,0)) gives
dJ/dK = m^T G m and dJ/dmu = 2 (tr G - m^T G m / 3).
"""
from __future__ import annotations

import numpy as np

from . import operator as op

_M = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])


def strain_fields(pb: op.Problem, loads, taus):
    """p_l - Gamma tau_l for every load, each of shape (c, *grid)."""
    return [op.strain(pb, p, t) for p, t in zip(np.atleast_2d(loads), taus)]


def tensor_gradient(pb: op.Problem, W, loads, taus) -> np.ndarray:
    """dJ/dA_beta for J = sum_lm W_lm p_l . A*_h p_m: array (*grid, c, c)."""
    W = np.asarray(W, dtype=np.float64)
    eps = strain_fields(pb, loads, taus)
    c = pb.c
    G = np.zeros((c, c) + tuple(pb.shape))
    for l in range(len(eps)):
        for m in range(len(eps)):
            if W[l, m] != 0.0:
                G += W[l, m] * 0.5 * (eps[l][:, None] * eps[m][None, :] + eps[m][:, None] * eps[l][None, :])
    G /= pb.nvox
    return np.moveaxis(G, (0, 1), (-2, -1))


def isotropic_gradient(pb: op.Problem, G: np.ndarray) -> np.ndarray:
    """Contract the tensor gradient with the isotropic parametrisation:
    (1, *grid) = dJ/da (scalar) or (2, *grid) = (dJ/dK, dJ/dmu) (elastic)."""
    tr = np.trace(G, axis1=-2, axis2=-1)
    if pb.physics == "scalar":
        return tr[None]
    mGm = np.einsum("i,...ij,j->...", _M, G, _M)
    return np.stack([mGm, 2.0 * (tr - mGm / 3.0)])


def isotropic_moduli(physics: str, coef: np.ndarray, d: int = 3) -> np.ndarray:
    """Per-voxel moduli (*grid, c, c) from isotropic coefficients: a (scalar,
    shape (1, *grid)) or bulk and shear moduli (K, mu) (elastic, (2, *grid))."""
    coef = np.asarray(coef, dtype=np.float64)
    shape = coef.shape[1:]
    if physics == "scalar":
        return coef[0][..., None, None] * np.eye(d)
    K, mu = coef[0][..., None, None], coef[1][..., None, None]
    mm = np.outer(_M, _M)
    return K * mm + 2.0 * mu * (np.eye(6) - mm / 3.0)
