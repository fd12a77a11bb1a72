"""Pins of the oracle's sliced Green-table route.

The full tables of ``oracle.green`` are pinned by closed values and identities
(test_oracle_green.py).  Two other routes evaluate the same definitions on part
of the grid and feed large cases: ``table(..., a_slice=s)`` (planes of the
slowest array axis; the slab route of ``oracle.operator.gamma_apply``) and
``at(shape, ..., kidx)`` (single wave-vectors; the expected values of the
full-size operator tests).  Both must reproduce the pinned full table entry by
entry for every operator: truncated (eqs. 14/15 with the Nyquist rule of
Section 3.2.1), filtered (Section 3.2.2), consistent (eq. 11) and
finite-difference (Section 3.2.3), scalar 2D/3D and elastic, at k = 0, on the
Nyquist planes and at mixed Nyquist indices.  A planted off-by-one slice must
be caught.
"""
import numpy as np
import pytest

from oracle import green
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

CASES = [
    # (physics, shape (array order), A0)
    ("scalar", (6, 8), np.array([[2.0, 0.3], [0.3, 1.5]])),
    ("scalar", (4, 6, 8), np.array([[2.0, 0.3, 0.1], [0.3, 1.5, -0.2], [0.1, -0.2, 1.2]])),
    ("elastic", (4, 6, 8), I.elastic_isotropic_mandel(0.7, 0.4)),
]


def _variants(physics):
    return ["truncated", "filtered", "consistent"] + (["fd"] if physics == "scalar" else [])


def _slices(n0):
    h = n0 // 2
    return [slice(0, 1), slice(h, h + 1), slice(n0 - 1, n0), slice(1, n0 - 1), slice(0, n0), slice(h - 1, n0, 2)]


def _kidx(shape):
    """Physical-axis index rows (kx, ky[, kz]): k = 0, the Nyquist index on
    each axis alone, all Nyquist, mixed Nyquist and generic indices."""
    d = len(shape)
    n = [shape[d - 1 - a] for a in range(d)]
    rows = [[0] * d]
    for a in range(d):
        r = [1] * d
        r[a] = n[a] // 2
        rows.append(r)
    rows.append([m // 2 for m in n])
    rows.append([n[0] // 2] + [m - 1 for m in n[1:]])
    rows.append([m - 1 for m in n])
    rows.append([1 + a for a in range(d)])
    return np.array(rows)


def _mismatches(nmax=2):
    """Every (case, variant, route) whose entries differ from the full table."""
    bad = []
    for physics, shape, A0 in CASES:
        for v in _variants(physics):
            full = green.table(shape, physics, A0, v, nmax=nmax)
            scale = np.max(np.abs(full))
            for s in _slices(shape[0]):
                part = green.table(shape, physics, A0, v, a_slice=s, nmax=nmax)
                if part.shape != full[s].shape or np.max(np.abs(part - full[s])) > 1e-14 * scale:
                    bad.append((physics, shape, v, "slice", s))
            kidx = _kidx(shape)
            got = green.at(shape, physics, A0, v, kidx, nmax=nmax)
            d = len(shape)
            for row, g in zip(kidx, got):
                ref = full[tuple(int(row[d - 1 - ax]) for ax in range(d))]
                if np.max(np.abs(g - ref)) > 1e-14 * scale:
                    bad.append((physics, shape, v, "at", tuple(row)))
    return bad


def test_sliced_and_pointwise_tables_equal_full_table():
    assert _mismatches() == []


def test_at_hits_the_nyquist_rule_and_zero():
    # the routes reach the special entries: truncated A0^{-1} at a Nyquist index,
    # 0 at k = 0 (every operator), on a single-point slice
    for physics, shape, A0 in CASES:
        d = len(shape)
        S = green.reference_compliance(A0)
        for v in _variants(physics):
            # exactly 0, except the consistent series' sin^2(pi n) tails (~1e-33)
            np.testing.assert_allclose(green.at(shape, physics, A0, v, [[0] * d], nmax=2)[0], 0.0, rtol=0, atol=1e-30)
        k = [shape[d - 1] // 2] + [1] * (d - 1)   # kx = N/2
        np.testing.assert_allclose(green.at(shape, physics, A0, "truncated", [k])[0], S, atol=1e-15)


def test_slab_route_of_the_operator_equals_the_cached_table(monkeypatch):
    # gamma_apply with the cache disabled takes the slab route (tables above the
    # cache limit); it must equal the route through the full table
    rng = np.random.default_rng(3)
    for physics, shape, A0 in CASES:
        ph = I.random_phases(shape, 2, seed=4)
        c = A0.shape[0]
        mod = np.stack([A0 + np.eye(c), 3.0 * A0])
        for v in ("truncated", "filtered"):
            pb = op.Problem(ph, mod, A0, physics, v)
            tau = rng.standard_normal((c,) + shape)
            op._TABLE_CACHE.clear()
            ref = op.gamma_apply(pb, tau, slab=2)
            op._TABLE_CACHE.clear()
            monkeypatch.setattr(op, "_CACHE_LIMIT", 0.0)
            got = op.gamma_apply(pb, tau, slab=2)
            monkeypatch.setattr(op, "_CACHE_LIMIT", 2.0e8)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))
    op._TABLE_CACHE.clear()


def test_planted_off_by_one_slice_is_caught(monkeypatch):
    real = green._axis_indices

    def shifted(shape, a_slice=None):
        out = real(shape, None)
        if a_slice is None:
            return out
        d = len(shape)
        ax = 0
        a = d - 1 - ax                      # physical axis held by array axis 0
        k = np.arange(shape[ax])[a_slice]
        k = (k + 1) % shape[ax]             # planted: one plane too far
        view = [1] * d
        view[ax] = k.size
        out[a] = k.reshape(view)
        return out

    monkeypatch.setattr(green, "_axis_indices", shifted)
    bad = _mismatches()
    routes = {b[3] for b in bad}
    assert "slice" in routes and "at" in routes, bad
