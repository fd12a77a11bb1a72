"""Planted mistakes in the oracle must be caught by its pins.

Each case monkeypatches one plausible error into ``oracle`` (on the CPU
only) and checks that the battery of closed-form pins rejects it.
"""
import numpy as np
import pytest

from oracle import effective, green
from oracle import operator as op
from oracle import solvers
from paper_1411_0330_amd import inputs as I

from . import closed_forms as cf


def _battery():
    """Return the list of failed pins (empty when the oracle is sound)."""
    op._TABLE_CACHE.clear()      # tables must come from the (possibly planted) code
    failed = []
    mod2 = np.stack([I.scalar_isotropic(1.0, 2), I.scalar_isotropic(10.0, 2)])
    harm, arith = cf.scalar_laminate([12 / 16, 4 / 16], [1.0, 10.0])
    for variant in ("truncated", "filtered"):
        ph = I.laminate((8, 16), 0, [(1, 4), (0, 12)])
        pb = op.Problem(ph, mod2, 0.5 * np.eye(2), "scalar", variant)
        try:
            A = effective.effective_matrix(pb.A0, np.eye(2),
                                           [solvers.cg(pb, p, tol=1e-12, maxit=300)["tau"] for p in np.eye(2)])
            if not np.allclose(A, [[harm, 0], [0, arith]], atol=1e-8):
                failed.append(f"laminate-{variant}")
        except (AssertionError, np.linalg.LinAlgError, ValueError):
            failed.append(f"laminate-{variant}-raised")
    # homogeneous medium
    pb = op.Problem(np.zeros((4, 4), np.uint8), np.stack([3.0 * np.eye(2)]), np.eye(2), "scalar", "filtered")
    try:
        tau = solvers.cg(pb, [1.0, 0.0], tol=1e-12)["tau"]
        if not np.allclose(effective.mean_stress(pb.A0, [1, 0], tau), [3.0, 0.0], atol=1e-10):
            failed.append("homogeneous")
    except (AssertionError, ValueError):
        failed.append("homogeneous-raised")
    # zero correction with a partially masked grid
    ph = I.random_phases((4, 4), 2, seed=1)
    pb = op.Problem(ph, np.stack([np.eye(2), 4.0 * np.eye(2)]), np.eye(2), "scalar", "truncated")
    try:
        tau = solvers.cg(pb, [1.0, 0.0], tol=1e-12)["tau"]
        if np.any(tau[:, ph == 0] != 0):
            failed.append("mask")
    except (AssertionError, ValueError):
        failed.append("mask-raised")
    # elastic laminate
    ph = I.laminate((2, 2, 8), 0, [(1, 2), (0, 6)])
    Cm, Ci = I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)
    C0 = I.elastic_isotropic_mandel(0.2, 0.15)
    pb = op.Problem(ph, np.stack([Cm, Ci]), C0, "elastic", "filtered")
    try:
        C = effective.effective_matrix(C0, np.eye(6), [solvers.cg(pb, p, tol=1e-12, maxit=300)["tau"] for p in np.eye(6)])
        if not np.allclose(C, cf.elastic_laminate([6 / 8, 2 / 8], [Cm, Ci]), atol=1e-8):
            failed.append("elastic-laminate")
    except (AssertionError, np.linalg.LinAlgError, ValueError):
        failed.append("elastic-laminate-raised")
    # symmetry of the bilinear form on a random elastic microstructure
    ph = I.random_phases((4, 4, 4), 2, seed=2)
    pb = op.Problem(ph, np.stack([Cm, Ci]), C0, "elastic", "filtered")
    s_, t_ = I.random_field((4, 4, 4), 6, 2, seed=3)
    try:
        lhs, rhs = op.dot(s_, op.apply(pb, t_)), op.dot(op.apply(pb, s_), t_)
        if abs(lhs - rhs) > 1e-10 * abs(lhs):
            failed.append("symmetry")
    except (AssertionError, ValueError):
        failed.append("symmetry-raised")
    return failed


def test_battery_passes_on_sound_oracle():
    assert _battery() == []


def _no_nyquist(shape, physics, A0, a_slice=None):
    d = len(shape)
    ks = green._axis_indices(shape, a_slice)
    gshape = green._grid_shape(shape, a_slice)
    xi = np.zeros(gshape + (d,))
    for a in range(d):
        n = shape[d - 1 - a]
        xi[..., a] = np.broadcast_to(np.where(ks[a] <= n // 2, ks[a], ks[a] - n), gshape)
    return green.gamma0(xi, physics, A0)


def _swapped_weights(k, n):
    c2, s2 = _ORIG_WEIGHTS(k, n)
    return s2, c2


_ORIG_WEIGHTS = green.filter_weights
_ORIG_GAMMA0 = green.gamma0
_ORIG_TABLES = op.phase_tables
_ORIG_AXES = green._axis_indices


def _neg_gamma0(xi, physics, A0):
    return -_ORIG_GAMMA0(xi, physics, A0)


def _unsym_gamma0(xi, physics, A0):
    G = _ORIG_GAMMA0(xi, physics, A0)
    if physics == "elastic":
        G = G + 0.25 * (G - np.swapaxes(G, -1, -2)) + 0.1 * np.tril(G, -1)
    return G


def _direct_instead_of_inverse(pb):
    delta, dinv, in_i0 = _ORIG_TABLES(pb)
    return delta, delta, in_i0


def _no_mask(pb):
    delta, dinv, in_i0 = _ORIG_TABLES(pb)
    return delta, dinv, np.ones_like(in_i0)


def _reversed_axes(shape, a_slice=None):
    return _ORIG_AXES(shape, a_slice)[::-1]


@pytest.mark.parametrize("target,attr,fake", [
    (green, "truncated", _no_nyquist),
    (green, "filter_weights", _swapped_weights),
    (green, "gamma0", _neg_gamma0),
    (green, "gamma0", _unsym_gamma0),
    (op, "phase_tables", _direct_instead_of_inverse),
    (op, "phase_tables", _no_mask),
    (green, "_axis_indices", _reversed_axes),
])
def test_planted_mistake_is_caught(monkeypatch, target, attr, fake):
    monkeypatch.setattr(target, attr, fake)
    try:
        assert _battery() != []
    finally:
        op._TABLE_CACHE.clear()
