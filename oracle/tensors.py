"""Mandel notation for symmetric second-order tensors (oracle-private).

The orthonormal basis E_J of symmetric 3x3 tensors is
E_0 = e1e1, E_1 = e2e2, E_2 = e3e3, E_3 = (e2e3+e3e2)/sqrt2,
E_4 = (e1e3+e3e1)/sqrt2, E_5 = (e1e2+e2e1)/sqrt2.  The Mandel vector of a
symmetric tensor t is v_J = E_J : t, so that v.w = t:s.
"""
import math

import numpy as np

_S = 1.0 / math.sqrt(2.0)


def mandel_basis() -> np.ndarray:
    E = np.zeros((6, 3, 3))
    E[0, 0, 0] = 1.0
    E[1, 1, 1] = 1.0
    E[2, 2, 2] = 1.0
    E[3, 1, 2] = E[3, 2, 1] = _S
    E[4, 0, 2] = E[4, 2, 0] = _S
    E[5, 0, 1] = E[5, 1, 0] = _S
    return E


def to_mandel(t: np.ndarray) -> np.ndarray:
    """(..., 3, 3) symmetric tensors -> (..., 6) Mandel vectors."""
    return np.einsum("Jij,...ij->...J", mandel_basis(), t)


def from_mandel(v: np.ndarray) -> np.ndarray:
    """(..., 6) Mandel vectors -> (..., 3, 3) tensors."""
    return np.einsum("Jij,...J->...ij", mandel_basis(), v)


def stiffness_tensor(M: np.ndarray) -> np.ndarray:
    """6x6 Mandel matrix -> fourth-order tensor C_ijkl acting on symmetric tensors."""
    E = mandel_basis()
    return np.einsum("IJ,Iij,Jkl->ijkl", M, E, E)
