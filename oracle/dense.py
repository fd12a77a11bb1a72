"""Dense real-space assembly of eq. (12) (oracle, tiny grids only).

Eq. (12) writes the discrete system as
(A_beta - A0)^{-1} tau_beta + sum_gamma Gamma_{beta-gamma} tau_gamma = p on I0,
where Gamma_beta is the inverse DFT of the Green table.  Here Gamma_beta is
summed directly, N^{-d} sum_k Gamma_hat_k cos(2 pi sum_a beta_a k_a / N_a)
(the table is even in k so the sine part cancels), without any FFT, the
block-circulant matrix is assembled on I0 x I0 and solved with LAPACK.
This is independent of the FFT route of ``oracle.operator`` and of any
iterative solver.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import green as _green
from . import operator as op


def real_space_kernel(pb: op.Problem) -> np.ndarray:
    """Gamma_beta for every beta of the grid: array (*grid, c, c)."""
    G = _green.table(pb.shape, pb.physics, pb.A0, pb.green, nmax=pb.series)
    shape = pb.shape
    d = len(shape)
    idx = np.array(list(itertools.product(*[range(n) for n in shape])))   # array-axis order
    phase = np.zeros((idx.shape[0], idx.shape[0]))
    for ax in range(d):
        phase += np.outer(idx[:, ax], idx[:, ax]) / shape[ax]
    E = np.exp(2j * math.pi * phase)           # rows beta, cols k
    Gf = G.reshape(idx.shape[0], pb.c, pb.c)
    K = np.einsum("bk,kij->bij", E, Gf) / idx.shape[0]
    if np.max(np.abs(K.imag)) > 1e-12 * max(1.0, np.max(np.abs(K.real))):
        raise AssertionError("real-space kernel is not real")
    return K.real.reshape(tuple(shape) + (pb.c, pb.c))


def assemble(pb: op.Problem):
    """Matrix of eq. (12) on the unknowns (beta in I0, component).

    Returns (M, voxel flat indices of I0)."""
    K = real_space_kernel(pb)
    shape = pb.shape
    c = pb.c
    _, dinv, in_i0 = op.voxel_tables(pb)
    i0 = np.nonzero(in_i0)[0]
    coords = np.array(np.unravel_index(i0, shape)).T
    n = i0.size
    M = np.zeros((n * c, n * c))
    for a, ca in enumerate(coords):
        diff = (ca[None, :] - coords) % np.array(shape)[None, :]
        blocks = K[tuple(diff.T)]                 # (n, c, c): Gamma_{beta_a - gamma}
        M[a * c:(a + 1) * c, :] = blocks.transpose(1, 0, 2).reshape(c, n * c)
        M[a * c:(a + 1) * c, a * c:(a + 1) * c] += dinv[i0[a]]
    return M, i0


def solve(pb: op.Problem, p) -> np.ndarray:
    """Exact solution tau of eq. (12) (zero outside I0), shape (c, *grid)."""
    M, i0 = assemble(pb)
    c = pb.c
    rhs = np.tile(np.asarray(p, dtype=np.float64), i0.size)
    sol = np.linalg.solve(M, rhs) if i0.size else np.zeros(0)
    tau = np.zeros((c, pb.nvox))
    tau[:, i0] = sol.reshape(i0.size, c).T
    return tau.reshape((c,) + tuple(pb.shape))
