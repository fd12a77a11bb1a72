"""The discrete Lippmann--Schwinger operator of eq. (13) (oracle).

For a polarisation tau (one c-vector per voxel, zero outside I0), eq. (13)
applies on every voxel beta of I0

    (L tau)_beta = (A_beta - A0)^{-1} tau_beta + DFT^{-1}_beta[ Gamma_hat_k DFT_k[tau] ]

and the system L tau = p holds on I0 (the right-hand side of eq. 9 is p on
every voxel of I0).  The forward DFT is unnormalised and DFT^{-1} carries the
1/N^d factor (Section 3.1).  A voxel is outside I0 when its phase has
A_beta = A0 exactly (hypothesis (2)); the polarisation and the operator output
vanish there.

This oracle uses full complex FFTs (scipy.fft, a library primitive) over the
whole grid, a per-voxel generic matrix inverse for (A_beta - A0)^{-1}, and
the Green tables of ``oracle.green``.  A problem is given either by a phase
map with one modulus per phase or by one modulus per voxel (``voxel``).  The real part of the inverse transform
is returned after checking the imaginary part is at rounding level.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

from . import green as _green


@dataclass
class Problem:
    phase: np.ndarray      # uint8, (NY,NX) or (NZ,NY,NX)
    moduli: np.ndarray     # (nphase, c, c) phase stiffness/conductivity
    A0: np.ndarray         # (c, c) reference medium
    physics: str           # "scalar" | "elastic"
    green: str = "filtered"
    series: int = 8        # consistent operator: alias cut nmax
    voxel: np.ndarray | None = None   # (*grid, c, c) per-voxel moduli; replaces phase/moduli

    @property
    def shape(self):
        return self.phase.shape

    @property
    def d(self):
        return self.phase.ndim

    @property
    def c(self):
        return _green.components(self.physics, self.d)

    @property
    def nvox(self):
        return int(np.prod(self.shape))


def phase_tables(pb: Problem):
    """Per phase: delta = A_phase - A0, its inverse, and membership of I0.

    A phase belongs to I0 unless A_phase equals A0 exactly.  Hypothesis (2)
    asks A_phase - A0 to be definite (of either sign) on I0; a singular or
    indefinite difference raises."""
    nph = pb.moduli.shape[0]
    c = pb.c
    delta = np.zeros((nph, c, c))
    dinv = np.zeros((nph, c, c))
    in_i0 = np.zeros(nph, dtype=bool)
    for p in range(nph):
        D = pb.moduli[p] - pb.A0
        if np.all(D == 0.0):
            continue
        ev = np.linalg.eigvalsh(0.5 * (D + D.T))
        if not (np.all(ev > 0) or np.all(ev < 0)):
            raise ValueError(f"phase {p}: A - A0 is not definite (hypothesis (2))")
        delta[p] = D
        dinv[p] = np.linalg.inv(D)
        in_i0[p] = True
    return delta, dinv, in_i0


def voxel_tables(pb: Problem):
    """Per voxel (flattened grid order): delta = A_beta - A0, its inverse
    (zero outside I0) and membership of I0, with the checks of
    ``phase_tables`` applied voxel by voxel."""
    c = pb.c
    if pb.voxel is None:
        delta, dinv, in_i0 = phase_tables(pb)
        ph = pb.phase.ravel()
        return delta[ph], dinv[ph], in_i0[ph]
    D = np.asarray(pb.voxel, dtype=np.float64).reshape(-1, c, c) - np.asarray(pb.A0)
    in_i0 = np.any(D != 0.0, axis=(1, 2))
    ev = np.linalg.eigvalsh(0.5 * (D + D.transpose(0, 2, 1)))
    definite = np.all(ev > 0, axis=1) | np.all(ev < 0, axis=1)
    bad = np.nonzero(in_i0 & ~definite)[0]
    if bad.size:
        raise ValueError(f"voxel {bad[0]}: A - A0 is not definite (hypothesis (2))")
    dinv = np.zeros_like(D)
    dinv[in_i0] = np.linalg.inv(D[in_i0])
    return D, dinv, in_i0


def mask(pb: Problem) -> np.ndarray:
    """Indicator of I0 on the grid."""
    if pb.voxel is not None:
        return voxel_tables(pb)[2].reshape(pb.shape)
    _, _, in_i0 = phase_tables(pb)
    return in_i0[pb.phase]


def _fft_axes(pb):
    return tuple(range(1, pb.d + 1))


_TABLE_CACHE = {}
_CACHE_LIMIT = 2.0e8   # table entries kept in memory (doubles)


def _slab_table(pb, sl):
    key = (pb.shape, pb.physics, np.asarray(pb.A0).tobytes(), pb.green, pb.series)
    full = _TABLE_CACHE.get(key)
    if full is not None:
        return full[sl]
    if pb.nvox * pb.c * pb.c <= _CACHE_LIMIT:
        if len(_TABLE_CACHE) > 8:
            _TABLE_CACHE.clear()
        full = _green.table(pb.shape, pb.physics, pb.A0, pb.green, nmax=pb.series)
        _TABLE_CACHE[key] = full
        return full[sl]
    return _green.table(pb.shape, pb.physics, pb.A0, pb.green, a_slice=sl, nmax=pb.series)


def gamma_apply(pb: Problem, tau: np.ndarray, slab: int = 16) -> np.ndarray:
    """DFT^{-1}[Gamma_hat_k DFT_k[tau]] for tau of shape (c, *grid).

    The Green table is evaluated once per problem when it fits in memory, and
    slab by slab along the slowest array axis otherwise."""
    axes = _fft_axes(pb)
    th = sfft.fftn(tau, axes=axes, workers=-1)
    out = np.empty_like(th)
    n0 = pb.shape[0]
    for s in range(0, n0, slab):
        sl = slice(s, min(s + slab, n0))
        G = _slab_table(pb, sl)
        # G: (n, ..., c, c);  th[:, sl]: (c, n, ...)
        out[:, sl] = np.einsum("...ij,j...->i...", G, th[:, sl])
    res = sfft.ifftn(out, axes=axes, workers=-1)
    scale = max(1.0, float(np.max(np.abs(res.real))))
    if np.max(np.abs(res.imag)) > 1e-10 * scale:
        raise AssertionError("Green operator output is not real: Gamma_hat is not even in k")
    return res.real


def local_apply(pb: Problem, tau: np.ndarray, which: str = "inverse") -> np.ndarray:
    """Per-voxel (A_beta - A0)^{-1} tau_beta (``inverse``) or (A_beta - A0) tau_beta."""
    if pb.voxel is not None:
        delta, dinv, _ = voxel_tables(pb)
        M = dinv if which == "inverse" else delta
        t = tau.reshape(pb.c, -1)
        return np.einsum("vij,jv->iv", M, t).reshape(tau.shape)
    delta, dinv, _ = phase_tables(pb)
    M = dinv if which == "inverse" else delta
    return np.einsum("...ij,j...->i...", M[pb.phase], tau)


def apply(pb: Problem, tau: np.ndarray) -> np.ndarray:
    """L tau of eq. (13), restricted to I0 (zero elsewhere)."""
    m = mask(pb)
    t = tau * m
    return m * (local_apply(pb, t) + gamma_apply(pb, t))


def rhs(pb: Problem, p: np.ndarray) -> np.ndarray:
    """Right-hand side of eq. (13): the macroscopic load p on every voxel of I0."""
    m = mask(pb).astype(np.float64)
    return np.asarray(p, dtype=np.float64).reshape((-1,) + (1,) * pb.d) * m


def strain(pb: Problem, p: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Estimate of p + grad w_p: p - Gamma tau on every voxel (Section 2.2.2,
    the proof of the equivalence lemma)."""
    return np.asarray(p, dtype=np.float64).reshape((-1,) + (1,) * pb.d) - gamma_apply(pb, tau)


def dot(a: np.ndarray, b: np.ndarray) -> float:
    """Euclidean product over voxels and components (NumPy pairwise sum)."""
    return float(np.sum(a * b, dtype=np.float64))
