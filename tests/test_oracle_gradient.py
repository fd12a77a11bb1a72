"""Pins of the oracle's derivative of A*_h with respect to per-voxel moduli.

* Brute force: central finite differences of J = sum_lm W_lm p_l . A*_h p_m
  with every A*_h from the exact dense solve of eq. (12), at single voxels and
  along a random direction; scalar 2D and elastic 3D, truncated and filtered.
* Euler's identity for the truncated operator: A*_h does not depend on A0
  (Table 1), hence is homogeneous of degree one in the local moduli, and
  sum_beta A_beta : dJ/dA_beta = J exactly.  The filtered operator depends on
  A0 and must miss this identity (guard).
"""
import numpy as np
import pytest

from oracle import dense, effective, gradient, solvers
from oracle import operator as op
from paper_1411_0330_amd import inputs as I


def _coef(physics, shape, seed):
    rng = np.random.default_rng(seed)
    if physics == "scalar":
        return rng.uniform(1.0, 10.0, size=(1,) + shape)
    K = rng.uniform(1.0, 6.0, size=shape)
    mu = rng.uniform(0.5, 3.0, size=shape)
    return np.stack([K, mu])


def _A0(physics, d):
    if physics == "scalar":
        return 0.5 * np.eye(d)
    mu0, nu0 = 0.25, 0.3
    return I.elastic_isotropic_mandel(2 * mu0 * nu0 / (1 - 2 * nu0), mu0)


def _problem(physics, shape, coef, green):
    d = len(shape)
    vox = gradient.isotropic_moduli(physics, coef, d)
    A0 = _A0(physics, d)
    c = vox.shape[-1]
    return op.Problem(np.zeros(shape, np.uint8), np.zeros((1, c, c)), A0, physics, green, voxel=vox)


def _J(pb, W, loads, solve):
    taus = [solve(pb, p) for p in loads]
    A = effective.effective_matrix(pb.A0, loads, taus)     # columns A* p_l
    return float(np.sum(W * (loads @ A))), taus


def _dense(pb, p):
    return dense.solve(pb, p)


CASES = [("scalar", (6, 6), "truncated"), ("scalar", (5, 7), "filtered"),
         ("elastic", (3, 4, 4), "filtered"), ("elastic", (4, 2, 4), "truncated")]


@pytest.mark.parametrize("physics,shape,green", CASES)
def test_gradient_matches_finite_differences_of_dense_solves(physics, shape, green):
    _fd_check(physics, shape, green)


def _fd_check(physics, shape, green):
    coef = _coef(physics, shape, seed=3)
    pb = _problem(physics, shape, coef, green)
    rng = np.random.default_rng(5)
    loads = rng.standard_normal((2, pb.c))
    W = np.array([[1.0, 0.3], [0.3, -0.7]])
    J0, taus = _J(pb, W, loads, _dense)
    g = gradient.isotropic_gradient(pb, gradient.tensor_gradient(pb, W, loads, taus))
    assert g.shape == coef.shape
    flat = [(i, v) for i in range(coef.shape[0]) for v in rng.choice(pb.nvox, 3, replace=False)]
    for i, v in flat:
        idx = (i,) + np.unravel_index(v, shape)
        h = 1e-4 * coef[idx]
        Jp = _J(_problem(physics, shape, _bump(coef, idx, h), green), W, loads, _dense)[0]
        Jm = _J(_problem(physics, shape, _bump(coef, idx, -h), green), W, loads, _dense)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * np.abs(g).max(), (idx, fd, g[idx])
    # a random direction over every voxel and coefficient
    dirn = rng.standard_normal(coef.shape)
    h = 1e-5
    Jp = _J(_problem(physics, shape, coef + h * dirn, green), W, loads, _dense)[0]
    Jm = _J(_problem(physics, shape, coef - h * dirn, green), W, loads, _dense)[0]
    assert abs((Jp - Jm) / (2 * h) - np.sum(g * dirn)) <= 1e-6 * abs(np.sum(np.abs(g * dirn)))


def _bump(coef, idx, h):
    c2 = coef.copy()
    c2[idx] += h
    return c2


@pytest.mark.parametrize("physics,shape", [("scalar", (16, 16)), ("elastic", (8, 8, 8))])
def test_euler_identity_truncated_and_its_failure_when_filtered(physics, shape):
    coef = _coef(physics, shape, seed=8)
    loads = np.eye(op.Problem(np.zeros(shape, np.uint8), np.zeros((1, 1, 1)), np.eye(1), physics).c)[:2]
    W = np.array([[1.0, 0.0], [0.0, 0.5]])
    gaps = {}
    for green in ("truncated", "filtered"):
        pb = _problem(physics, shape, coef, green)
        J, taus = _J(pb, W, loads, lambda pb_, p: solvers.cg(pb_, p, tol=1e-13, maxit=3000)["tau"])
        g = gradient.isotropic_gradient(pb, gradient.tensor_gradient(pb, W, loads, taus))
        gaps[green] = abs(np.sum(g * coef) - J) / abs(J)
    assert gaps["truncated"] <= 1e-10
    assert gaps["filtered"] >= 1e-6


def test_isotropic_moduli_and_contraction_are_consistent():
    # dJ/dK and dJ/dmu are the contractions of G with dC/dK and dC/dmu
    rng = np.random.default_rng(1)
    G = rng.standard_normal((6, 6))
    G = 0.5 * (G + G.T)
    pb = op.Problem(np.zeros((1, 1, 1), np.uint8), np.zeros((1, 6, 6)), np.eye(6), "elastic")
    g = gradient.isotropic_gradient(pb, G[None, None, None])[:, 0, 0, 0]
    h = 1e-6
    for i in range(2):
        e = np.zeros((2, 1, 1, 1))
        e[i] = h
        base = np.array([2.0, 1.0]).reshape(2, 1, 1, 1)
        dC = (gradient.isotropic_moduli("elastic", base + e) - gradient.isotropic_moduli("elastic", base - e))[0, 0, 0]
        assert abs(np.sum(G * dC) / (2 * h) - g[i]) <= 1e-8


_ORIG_STRAIN = gradient.strain_fields
_ORIG_TENSOR = gradient.tensor_gradient
_ORIG_ISO = gradient.isotropic_gradient


def _tau_for_strain(pb, loads, taus):
    return list(taus)


def _no_volume(pb, W, loads, taus):
    return _ORIG_TENSOR(pb, W, loads, taus) * pb.nvox


def _diagonal_only(pb, W, loads, taus):
    return _ORIG_TENSOR(pb, np.diag(np.diag(np.asarray(W))), loads, taus)


def _shear_factor(pb, G):
    g = _ORIG_ISO(pb, G)
    if pb.physics == "elastic":
        g = g.copy()
        g[1] *= 0.5
    return g


@pytest.mark.parametrize("attr,fake", [("strain_fields", _tau_for_strain), ("tensor_gradient", _no_volume),
                                       ("tensor_gradient", _diagonal_only), ("isotropic_gradient", _shear_factor)])
def test_planted_gradient_mistake_is_caught(monkeypatch, attr, fake):
    monkeypatch.setattr(gradient, attr, fake)
    caught = 0
    for physics, shape, green in (CASES[0], CASES[2]):
        try:
            _fd_check(physics, shape, green)
        except AssertionError:
            caught += 1
    assert caught >= 1


@pytest.mark.parametrize("physics,shape", [("scalar", (8, 6)), ("elastic", (4, 4, 2))])
def test_voxel_moduli_reproduce_the_phase_map(physics, shape):
    # the same medium given per phase and per voxel: identical operator and mask
    d = len(shape)
    ph = I.random_phases(shape, 3, seed=2)
    if physics == "scalar":
        mods = np.stack([a * np.eye(d) for a in (1.0, 0.5, 7.0)])     # phase 1 equals A0
    else:
        mods = np.stack([I.elastic_from_young(1.0, 0.3), _A0("elastic", 3), I.elastic_from_young(9.0, 0.2)])
    A0 = _A0(physics, d)
    pb_ph = op.Problem(ph, mods, A0, physics, "filtered")
    pb_vx = op.Problem(np.zeros(shape, np.uint8), np.zeros((1,) + mods.shape[1:]), A0, physics, "filtered",
                       voxel=mods[ph])
    assert np.array_equal(op.mask(pb_ph), op.mask(pb_vx))
    tau = I.random_field(shape, pb_ph.c, 1, seed=4)[0] * op.mask(pb_ph)
    assert np.array_equal(op.apply(pb_ph, tau), op.apply(pb_vx, tau))


def test_voxel_hypothesis_two_is_checked():
    shape = (4, 4)
    vox = np.broadcast_to(2.0 * np.eye(2), shape + (2, 2)).copy()
    vox[1, 2] = np.diag([2.0, 0.1])          # A - A0 = diag(1.5, -0.4): indefinite
    pb = op.Problem(np.zeros(shape, np.uint8), np.zeros((1, 2, 2)), 0.5 * np.eye(2), "scalar", voxel=vox)
    with pytest.raises(ValueError):
        op.mask(pb)
