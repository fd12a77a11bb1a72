"""Pins of the oracle's Green operators against closed values and identities.

Section 2.2.1 gives Gamma0_hat(k) = (k^T A0 k)^{-1} k k^T (0 at k = 0);
Section 3.2.1 the truncated operator and its Nyquist rule; Section 3.2.2 the
filtered operator; eq. (11) the consistent one; Section 3.2.3 the
finite-difference one.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import green
from paper_1411_0330_amd import inputs as I


def _spd(rng, c):
    M = rng.standard_normal((c, c))
    return M @ M.T + c * np.eye(c)


def test_gamma0_scalar_closed_values():
    a0 = 2.5
    A0 = a0 * np.eye(2)
    G = green.gamma0(np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 0.0], [0.0, -3.0]]), "scalar", A0)
    np.testing.assert_allclose(G[0], [[1 / a0, 0], [0, 0]], atol=1e-16)
    np.testing.assert_allclose(G[1], np.ones((2, 2)) / (2 * a0), atol=1e-16)
    np.testing.assert_array_equal(G[2], np.zeros((2, 2)))
    np.testing.assert_allclose(G[3], [[0, 0], [0, 1 / a0]], atol=1e-16)
    # anisotropic A0: along e1 the denominator is A0_11
    A = np.array([[3.0, 1.0], [1.0, 2.0]])
    np.testing.assert_allclose(green.gamma0(np.array([1.0, 0.0]), "scalar", A), [[1 / 3, 0], [0, 0]])


def test_truncated_nyquist_and_centring():
    a0 = 4.0
    A0 = a0 * np.eye(2)
    T = green.truncated((8, 8), "scalar", A0)           # array (y, x)
    # index (kx, ky) = (4, 1): kx at N/2 -> A0^{-1}
    np.testing.assert_allclose(T[1, 4], np.eye(2) / a0)
    np.testing.assert_allclose(T[4, 3], np.eye(2) / a0)
    # index kx = 5 is the centred frequency -3 -> same direction as e1
    np.testing.assert_allclose(T[0, 5], [[1 / a0, 0], [0, 0]])
    np.testing.assert_array_equal(T[0, 0], np.zeros((2, 2)))
    # odd N: no Nyquist rule, index 4 of N=7 is frequency -3
    T7 = green.truncated((7, 7), "scalar", A0)
    np.testing.assert_allclose(T7[4, 4], np.ones((2, 2)) / (2 * a0))


@pytest.mark.parametrize("variant", ["truncated", "filtered", "consistent"])
def test_even_in_k(variant):
    rng = np.random.default_rng(0)
    shape = (6, 8)
    A0 = _spd(rng, 2)
    T = green.table(shape, "scalar", A0, variant)
    neg = T[(-np.arange(6)) % 6][:, (-np.arange(8)) % 8]
    np.testing.assert_allclose(T, neg, atol=1e-15)


def test_projector_trace_and_bounds_scalar():
    rng = np.random.default_rng(1)
    for d in (2, 3):
        A0 = _spd(rng, d)
        xi = rng.standard_normal((50, d))
        G = green.gamma0(xi, "scalar", A0)
        for g in G:
            np.testing.assert_allclose(g @ A0 @ g, g, atol=1e-14)
            assert abs(np.trace(A0 @ g) - 1.0) < 1e-14
        for variant in ("truncated", "filtered"):
            # odd sizes for the truncated operator: its Nyquist entries are
            # A0^{-1} (trace d), checked separately
            if variant == "truncated":
                shape = (5, 7) if d == 2 else (3, 5, 7)
            else:
                shape = (5, 6) if d == 2 else (4, 5, 6)
            T = green.table(shape, "scalar", A0, variant).reshape(-1, d, d)
            L = np.linalg.cholesky(A0)
            for i, g in enumerate(T):
                if i == 0:
                    np.testing.assert_array_equal(g, 0)
                    continue
                ev = np.linalg.eigvalsh(L.T @ g @ L)
                assert ev.min() > -1e-13 and ev.max() < 1 + 1e-13
                assert abs(np.trace(A0 @ g) - 1.0) < 1e-13


def _iso_elastic_closed(n, lam0, mu0):
    """Isotropic elastic Gamma0_hat as a Mandel matrix from the closed form
    (delta_ik n_j n_l + delta_il n_j n_k + delta_jk n_i n_l + delta_jl n_i n_k)/(4 mu0)
    - (lam0 + mu0)/(mu0 (lam0 + 2 mu0)) n_i n_j n_k n_l."""
    from oracle.tensors import mandel_basis
    dlt = np.eye(3)
    G4 = (np.einsum("ik,j,l->ijkl", dlt, n, n) + np.einsum("il,j,k->ijkl", dlt, n, n)
          + np.einsum("jk,i,l->ijkl", dlt, n, n) + np.einsum("jl,i,k->ijkl", dlt, n, n)) / (4 * mu0)
    G4 -= (lam0 + mu0) / (mu0 * (lam0 + 2 * mu0)) * np.einsum("i,j,k,l->ijkl", n, n, n, n)
    E = mandel_basis()
    return np.einsum("Iij,ijkl,Jkl->IJ", E, G4, E)


def test_elastic_generic_matches_isotropic_closed_form():
    rng = np.random.default_rng(2)
    lam0, mu0 = 0.7, 0.35
    C0 = I.elastic_isotropic_mandel(lam0, mu0)
    xi = rng.standard_normal((40, 3))
    G = green.gamma0(xi, "elastic", C0)
    S0 = np.linalg.inv(C0)
    L = np.linalg.cholesky(C0)
    for x, g in zip(xi, G):
        n = x / np.linalg.norm(x)
        np.testing.assert_allclose(g, _iso_elastic_closed(n, lam0, mu0), atol=1e-13)
        np.testing.assert_allclose(g @ C0 @ g, g, atol=1e-13)       # projector in the C0 metric
        assert abs(np.trace(C0 @ g) - 3.0) < 1e-13                  # rank d
        ev = np.linalg.eigvalsh(L.T @ g @ L)
        assert ev.min() > -1e-13 and ev.max() < 1 + 1e-13           # 0 <= Gamma <= C0^{-1}
    T = green.truncated((4, 4, 4), "elastic", C0)
    np.testing.assert_allclose(T[0, 0, 2], S0, atol=1e-15)         # kx = N/2 -> C0^{-1}


def test_filter_weights_partition_of_unity():
    for n in (3, 8, 64, 256):
        k = np.arange(n)
        c2, s2 = green.filter_weights(k, n)
        np.testing.assert_allclose(c2 + s2, 1.0, atol=1e-16)
        assert c2[0] == 1.0 and s2[0] == 0.0


def test_filtered_single_axis_frequency_is_exact_direction():
    # for k = (k1, 0, 0) every alias with non-zero weight points along e1
    C0 = I.elastic_isotropic_mandel(0.5, 0.3)
    T = green.filtered((4, 4, 8), "elastic", C0)
    for k1 in range(1, 8):
        np.testing.assert_allclose(T[0, 0, k1], green.gamma0(np.array([1.0, 0, 0]), "elastic", C0), atol=1e-14)


def test_consistent_series_partition():
    # sum over aliases of sinc^2 is 1, so the trace identity holds up to the cut series
    A0 = 1.7 * np.eye(2)
    T = green.consistent((6, 6), "scalar", A0, nmax=30).reshape(-1, 2, 2)
    tr = np.array([np.trace(A0 @ g) for g in T[1:]])
    assert np.all(np.abs(tr - 1.0) < 0.02)
    np.testing.assert_allclose(T[0], 0, atol=1e-25)     # sinc^2 vanishes at the non-zero integers


def test_fd_operator_projector():
    rng = np.random.default_rng(3)
    A0 = _spd(rng, 3)
    T = green.finite_difference((4, 5, 6), A0).reshape(-1, 3, 3)
    np.testing.assert_array_equal(T[0], 0)
    for g in T[1:]:
        np.testing.assert_allclose(g, g.conj().T, atol=1e-15)
        np.testing.assert_allclose(g @ A0 @ g, g, atol=1e-13)
