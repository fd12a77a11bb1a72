"""Periodic Green operator and its discrete approximations (oracle).

Section 2.2.1 defines, for a constant symmetric positive definite A0,
Gamma0_hat(k) = (k^T A0 k)^{-1} k k^T for k != 0 and 0 at k = 0.  It is
homogeneous of degree 0, so only the direction of k matters.

For isotropic elasticity (Section 5 says the approach carries over but prints
no formula) the same object is read off its defining problem
-div(C0 eps(u) + tau) = 0, eps(u) = -Gamma0 * tau: in Fourier space
Gamma0_hat(xi) tau = sym(xi (x) K0(xi)^{-1} (tau xi)) with the acoustic tensor
K0(xi)_ik = C0_ijkl xi_j xi_l.  The oracle evaluates this generic form (no
isotropic closed form) and returns it as a 6x6 Mandel matrix.

Frequencies.  A grid has N_a voxels along physical axis a and the DFT index
k_a runs over {0, ..., N_a-1}.  The *physical* frequency of alias n is
k_a + n_a N_a (the unit cell is (0,1)^d); for a cubic grid this is N times
the k/N + n of Sections 3.1-3.2, and Gamma0_hat is blind to that factor.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .tensors import mandel_basis, stiffness_tensor


def components(physics: str, d: int) -> int:
    return d if physics == "scalar" else 6


# --------------------------------------------------------------------------
# continuous operator
# --------------------------------------------------------------------------
def gamma0(xi: np.ndarray, physics: str, A0: np.ndarray) -> np.ndarray:
    """Gamma0_hat at frequency vectors ``xi`` of shape (..., d); returns (..., c, c).

    Scalar: the formula of Section 2.2.1.  Elastic: the generic acoustic
    tensor form described in the module docstring (d = 3)."""
    xi = np.asarray(xi, dtype=np.float64)
    d = xi.shape[-1]
    c = components(physics, d)
    out = np.zeros(xi.shape[:-1] + (c, c))
    n2 = np.einsum("...i,...i->...", xi, xi)
    nz = n2 > 0.0
    x = xi[nz]
    if physics == "scalar":
        den = np.einsum("...i,ij,...j->...", x, A0, x)
        out[nz] = x[:, :, None] * x[:, None, :] / den[:, None, None]
        return out
    if d != 3:
        raise ValueError("elasticity is three-dimensional")
    C = stiffness_tensor(A0)
    K = np.einsum("ijkl,nj,nl->nik", C, x, x)
    Kinv = np.linalg.inv(K)
    E = mandel_basis()
    tx = np.einsum("Jij,nj->nJi", E, x)            # tau xi for each basis tensor
    u = np.einsum("nki,nJi->nJk", Kinv, tx)         # K0^{-1} (tau xi)
    eps = 0.5 * (x[:, None, :, None] * u[:, :, None, :] + x[:, None, None, :] * u[:, :, :, None])
    out[nz] = np.einsum("Iab,nJab->nIJ", E, eps)
    return out


def reference_compliance(A0: np.ndarray) -> np.ndarray:
    """A0^{-1} (scalar) or the compliance C0^{-1} on symmetric tensors (Mandel)."""
    return np.linalg.inv(A0)


# --------------------------------------------------------------------------
# frequency grids
# --------------------------------------------------------------------------
def _axis_indices(shape, a_slice=None):
    """DFT indices per *physical* axis, broadcastable over the array shape
    (array axis d-1-a holds physical axis a).  ``a_slice`` optionally restricts
    array axis 0 to a range (a slab of planes)."""
    d = len(shape)
    out = []
    for a in range(d):
        ax = d - 1 - a
        k = np.arange(shape[ax])
        if ax == 0 and a_slice is not None:
            k = k[a_slice]
        view = [1] * d
        view[ax] = k.size
        out.append(k.reshape(view))
    return out


def _grid_shape(shape, a_slice):
    if a_slice is None:
        return tuple(shape)
    n0 = len(range(*a_slice.indices(shape[0])))
    return (n0,) + tuple(shape[1:])


# --------------------------------------------------------------------------
# discrete Green operators
# --------------------------------------------------------------------------
def truncated(shape, physics, A0, a_slice=None) -> np.ndarray:
    """Truncated operator of Moulinec and Suquet, eqs. (14)/(15).

    Each index is mapped to its centred representative in {-M+1..M} (N = 2M)
    or {-M..M} (N = 2M+1) and Gamma0_hat is evaluated there.  For even N, any
    frequency with a component equal to M is replaced by A0^{-1} (the
    Nyquist rule closing Section 3.2.1); this reading applies the rule when
    *any* component sits at M.  Returns (*grid, c, c)."""
    d = len(shape)
    ks = _axis_indices(shape, a_slice)
    gshape = _grid_shape(shape, a_slice)
    xi = np.zeros(gshape + (d,))
    nyq = np.zeros(gshape, dtype=bool)
    for a in range(d):
        n = shape[d - 1 - a]
        k = ks[a]
        kc = np.where(k <= n // 2, k, k - n)
        xi[..., a] = np.broadcast_to(kc, gshape)
        if n % 2 == 0:
            nyq |= np.broadcast_to(k == n // 2, gshape)
    G = gamma0(xi, physics, A0)
    G[nyq] = reference_compliance(A0)
    return G


def filter_weights(k, n):
    """Per-axis weights of the filtered operator for DFT index k in [0, n):
    (cos^2(pi k/(2n)), sin^2(pi k/(2n))) for the aliases k/n and k/n - 1."""
    t = math.pi * np.asarray(k, dtype=np.float64) / (2.0 * n)
    return np.cos(t) ** 2, np.sin(t) ** 2


def filtered(shape, physics, A0, a_slice=None) -> np.ndarray:
    """Filtered operator of Section 3.2.2.

    Sum over n in {-1,0}^d of prod_a cos^2(pi (k_a/N_a + n_a)/2) times
    Gamma0_hat at the alias k + n N.  The index k is taken in {0..N-1} (the
    formula is not N-periodic as printed; this reading extends it
    periodically from that fundamental range)."""
    d = len(shape)
    ks = _axis_indices(shape, a_slice)
    gshape = _grid_shape(shape, a_slice)
    c = components(physics, d)
    out = np.zeros(gshape + (c, c))
    w_axes = [filter_weights(ks[a], shape[d - 1 - a]) for a in range(d)]
    for ns in itertools.product((0, -1), repeat=d):
        xi = np.zeros(gshape + (d,))
        w = np.ones(gshape)
        for a in range(d):
            n = shape[d - 1 - a]
            xi[..., a] = np.broadcast_to(ks[a] + ns[a] * n, gshape)
            w = w * np.broadcast_to(w_axes[a][0] if ns[a] == 0 else w_axes[a][1], gshape)
        out += w[..., None, None] * gamma0(xi, physics, A0)
    return out


def consistent(shape, physics, A0, nmax=8, a_slice=None) -> np.ndarray:
    """Consistent operator of eq. (11), with the lattice series cut to the
    aliases whose reduced frequency k_a/N_a + n_a lies in
    [-(nmax + 1/2), nmax + 1/2] on every axis (a cut symmetric in k, so the
    truncated series stays even).  F(K) = prod sin(K_a/2)/(K_a/2) at
    K = 2 pi (k/N + n)."""
    d = len(shape)
    ks = _axis_indices(shape, a_slice)
    gshape = _grid_shape(shape, a_slice)
    c = components(physics, d)
    out = np.zeros(gshape + (c, c))
    rng = range(-nmax - 1, nmax + 2)
    for ns in itertools.product(rng, repeat=d):
        xi = np.zeros(gshape + (d,))
        w = np.ones(gshape)
        for a in range(d):
            n = shape[d - 1 - a]
            frac = np.broadcast_to(ks[a] / n + ns[a], gshape)
            xi[..., a] = frac * n
            w = w * np.sinc(frac) ** 2 * (np.abs(frac) <= nmax + 0.5)   # sinc(x) = sin(pi x)/(pi x)
        out += w[..., None, None] * gamma0(xi, physics, A0)
    return out


def finite_difference(shape, A0, a_slice=None) -> np.ndarray:
    """Finite-difference operator of Section 3.2.3 (scalar problems):
    V V^H / (V^H A0 V) with V_a = (exp(2 i pi k_a/N_a) - 1) N_a.  Complex
    Hermitian; zero at k = 0."""
    d = len(shape)
    ks = _axis_indices(shape, a_slice)
    gshape = _grid_shape(shape, a_slice)
    V = np.zeros(gshape + (d,), dtype=np.complex128)
    for a in range(d):
        n = shape[d - 1 - a]
        V[..., a] = np.broadcast_to((np.exp(2j * math.pi * ks[a] / n) - 1.0) * n, gshape)
    den = np.einsum("...i,ij,...j->...", V.conj(), A0, V).real
    out = np.zeros(gshape + (d, d), dtype=np.complex128)
    nz = den > 0
    out[nz] = V[nz][:, :, None] * V[nz].conj()[:, None, :] / den[nz][:, None, None]
    return out


def at(shape, physics, A0, variant, kidx, nmax=8) -> np.ndarray:
    """Table entries at the DFT index vectors ``kidx`` (rows of physical-axis
    indices (kx, ky[, kz])), evaluated by the same definitions on a
    one-point view of the grid.  Returns (n, c, c)."""
    kidx = np.atleast_2d(np.asarray(kidx, dtype=np.int64))
    d = len(shape)
    out = []
    for k in kidx:
        # the entry of the full table at array index reversed(k)
        sl = slice(int(k[d - 1]), int(k[d - 1]) + 1)
        T = table(shape, physics, A0, variant, a_slice=sl, nmax=nmax)
        idx = (0,) + tuple(int(k[d - 1 - ax]) for ax in range(1, d))
        out.append(T[idx])
    return np.stack(out)


def table(shape, physics, A0, variant, a_slice=None, nmax=8) -> np.ndarray:
    if variant == "truncated":
        return truncated(shape, physics, A0, a_slice)
    if variant == "filtered":
        return filtered(shape, physics, A0, a_slice)
    if variant == "consistent":
        return consistent(shape, physics, A0, nmax=nmax, a_slice=a_slice)
    if variant == "fd":
        if physics != "scalar":
            raise ValueError("the finite-difference operator is scalar-only")
        return finite_difference(shape, A0, a_slice)
    raise ValueError(f"unknown Green operator {variant!r}")
