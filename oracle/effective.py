"""Homogenised matrix from the polarisation (oracle).

Theorem 4 (error analysis) defines the discrete estimate through
A*_h p = A0 p + integral over Q of tau^h_p, the discrete analogue of
eq. (tau_Astar).  With piecewise-constant tau^h the integral is the voxel
mean.  Sums use math.fsum.
"""
from __future__ import annotations

import math

import numpy as np


def mean_stress(A0: np.ndarray, p, tau: np.ndarray) -> np.ndarray:
    """A0 p + mean over voxels of tau (shape (c, *grid)) -> c-vector."""
    c = tau.shape[0]
    nvox = tau[0].size
    m = np.array([math.fsum(tau[i].ravel().tolist()) / nvox for i in range(c)])
    return np.asarray(A0) @ np.asarray(p, dtype=np.float64) + m


def effective_matrix(A0: np.ndarray, loads: np.ndarray, taus) -> np.ndarray:
    """Columns A*_h p_l for the loads p_l (rows of ``loads``).  With the c
    unit loads this is the c x c homogenised matrix (Mandel in elasticity)."""
    cols = [mean_stress(A0, p, t) for p, t in zip(loads, taus)]
    return np.stack(cols, axis=1)
