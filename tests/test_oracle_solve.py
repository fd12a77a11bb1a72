"""Pins of the oracle's operator and solvers.

* The FFT route of eq. (13) against the real-space assembly of eq. (12)
  (direct DFT sums, LAPACK solve) on grids of at most a few hundred voxels.
* Symmetry of the bilinear form (eq. 5) and definiteness when A0 is softer
  than every phase (Section 5).
* Closed forms: homogeneous media, empty I0, laminates (harmonic and
  arithmetic means; the exact elastic laminate), the 2D checkerboard limit
  sqrt(a1 a2), Hashin--Shtrikman and Voigt/Reuss bounds.
* Table 1: the truncated scheme does not depend on A0, the filtered one does.
"""
import math

import numpy as np
import pytest

from oracle import dense, effective, green
from oracle import operator as op
from oracle import solvers
from paper_1411_0330_amd import inputs as I

from . import closed_forms as cf


def _elastic_pb(shape, green_variant, seed=0, nphase=2):
    ph = I.random_phases(shape, nphase, seed)
    C = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2),
                  I.elastic_from_young(3.0, 0.25)][:nphase])
    mu0 = 0.5 * I.lame_from_young(1.0, 0.3)[1]
    lam0 = 2 * mu0 * 0.3 / 0.4
    return op.Problem(ph, C, I.elastic_isotropic_mandel(lam0, mu0), "elastic", green_variant)


def _scalar_pb(shape, green_variant, a0=0.5, seed=0, aniso=False):
    d = len(shape)
    ph = I.random_phases(shape, 2, seed)
    mod = [I.scalar_isotropic(1.0, d), I.scalar_isotropic(10.0, d)]
    if aniso:
        rng = np.random.default_rng(seed + 7)
        M = rng.standard_normal((d, d))
        mod[1] = mod[1] + 0.3 * (M @ M.T)
    return op.Problem(ph, np.stack(mod), a0 * np.eye(d), "scalar", green_variant)


CASES = [
    ("scalar", (6, 8), "truncated"),
    ("scalar", (7, 5), "filtered"),
    ("scalar", (4, 4, 6), "truncated"),
    ("scalar", (4, 5, 4), "filtered"),
    ("elastic", (4, 4, 4), "filtered"),
    ("elastic", (4, 2, 4), "truncated"),
]


def _pb(kind, shape, variant, seed=0):
    return _scalar_pb(shape, variant, seed=seed, aniso=True) if kind == "scalar" else _elastic_pb(shape, variant, seed)


@pytest.mark.parametrize("kind,shape,variant", CASES)
def test_fft_operator_matches_real_space_assembly(kind, shape, variant):
    pb = _pb(kind, shape, variant)
    M, i0 = dense.assemble(pb)
    tau = I.random_field(shape, pb.c, 1, seed=3)[0]
    q = op.apply(pb, tau)
    x = tau.reshape(pb.c, -1)[:, i0].T.ravel()
    ref = (M @ x).reshape(-1, pb.c).T
    np.testing.assert_allclose(q.reshape(pb.c, -1)[:, i0], ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("kind,shape,variant", CASES)
def test_cg_and_basic_match_dense_solve(kind, shape, variant):
    pb = _pb(kind, shape, variant)
    for j in range(pb.c):
        p = np.eye(pb.c)[j]
        exact = dense.solve(pb, p)
        r = solvers.cg(pb, p, tol=1e-13, maxit=2000)
        np.testing.assert_allclose(r["tau"], exact, atol=1e-10 * np.abs(exact).max())
    if kind == "scalar":
        # the basic scheme needs |a - a0| < a0: a0 above half the stiffest phase
        amax = max(np.linalg.eigvalsh(m).max() for m in pb.moduli)
        pb2 = op.Problem(pb.phase, pb.moduli, 0.6 * amax * np.eye(pb.d), "scalar", variant)
        p = np.eye(pb.c)[0]
        exact = dense.solve(pb2, p)
        r = solvers.basic(pb2, p, tol=1e-13, maxit=5000)
        np.testing.assert_allclose(r["tau"], exact, atol=1e-10 * np.abs(exact).max())


@pytest.mark.parametrize("kind,shape,variant", CASES)
def test_operator_symmetric_and_positive(kind, shape, variant):
    pb = _pb(kind, shape, variant)
    s, t = I.random_field(shape, pb.c, 2, seed=5)
    lhs = op.dot(s, op.apply(pb, t))
    rhs = op.dot(op.apply(pb, s), t)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    # A0 softer than every phase: positive definite
    assert op.dot(t, op.apply(pb, t)) > 0


def test_gamma_kills_constants_and_local_inverse():
    pb = _elastic_pb((4, 4, 4), "filtered")
    const = np.ones((6, 4, 4, 4)) * np.arange(1, 7).reshape(6, 1, 1, 1)
    np.testing.assert_allclose(op.gamma_apply(pb, const), 0, atol=1e-13)
    t = I.random_field((4, 4, 4), 6, 1, seed=1)[0]
    back = op.local_apply(pb, op.local_apply(pb, t, "direct"), "inverse")
    np.testing.assert_allclose(back, t, atol=1e-12)


@pytest.mark.parametrize("variant", ["truncated", "filtered"])
def test_homogeneous_medium(variant):
    # A = a everywhere (a != a0): tau = (a - a0) p, A* = a, CG in one iteration
    shape = (8, 8, 8)
    a, a0 = 3.0, 1.25
    pb = op.Problem(np.zeros(shape, np.uint8), np.stack([a * np.eye(3)]), a0 * np.eye(3), "scalar", variant)
    p = np.array([0.3, -1.0, 2.0])
    r = solvers.cg(pb, p, tol=1e-14)
    assert r["iters"] == 1
    np.testing.assert_allclose(r["tau"], (a - a0) * p.reshape(3, 1, 1, 1) * np.ones(shape), atol=1e-14)
    np.testing.assert_allclose(effective.mean_stress(pb.A0, p, r["tau"]), a * p, atol=1e-13)
    # elastic
    C = I.elastic_from_young(2.0, 0.3)
    C0 = I.elastic_from_young(0.7, 0.3)
    pbe = op.Problem(np.zeros((4, 4, 4), np.uint8), np.stack([C]), C0, "elastic", variant)
    pe = np.arange(1.0, 7.0)
    r = solvers.cg(pbe, pe, tol=1e-14)
    # L acts on constants as the 6x6 (C - C0)^{-1}, which has two distinct
    # eigenvalues (bulk and shear) for isotropic C and C0
    assert r["iters"] == 2
    np.testing.assert_allclose(r["tau"], ((C - C0) @ pe).reshape(6, 1, 1, 1) * np.ones((4, 4, 4)), atol=1e-12)
    np.testing.assert_allclose(effective.mean_stress(C0, pe, r["tau"]), C @ pe, atol=1e-12)


def test_zero_correction_and_partial_mask():
    # every voxel equals A0: I0 is empty, tau = 0, A* = A0
    shape = (6, 6)
    A0 = 2.0 * np.eye(2)
    pb = op.Problem(np.zeros(shape, np.uint8), np.stack([A0]), A0, "scalar", "filtered")
    r = solvers.cg(pb, np.array([1.0, 0.0]))
    assert r["iters"] == 0 and np.all(r["tau"] == 0)
    np.testing.assert_array_equal(effective.mean_stress(A0, [1.0, 0.0], r["tau"]), [2.0, 0.0])
    # phase 0 equals A0: tau vanishes there, the dense solve agrees
    ph = I.random_phases((6, 6), 2, seed=4)
    pb = op.Problem(ph, np.stack([A0, 7.0 * np.eye(2)]), A0, "scalar", "truncated")
    r = solvers.cg(pb, np.array([1.0, 0.5]), tol=1e-13)
    assert np.all(r["tau"][:, ph == 0] == 0)
    np.testing.assert_allclose(r["tau"], dense.solve(pb, np.array([1.0, 0.5])), atol=1e-11)


@pytest.mark.parametrize("variant,a0", [("truncated", 0.5), ("truncated", 5.5), ("truncated", 20.0),
                                        ("filtered", 0.5), ("filtered", 20.0)])
def test_scalar_laminate(variant, a0):
    # layers normal to e1 with even thicknesses starting on even voxels
    n = 32
    ph = I.laminate((8, n), 0, [(1, 10), (0, 22)])
    a = [1.0, 10.0]
    pb = op.Problem(ph, np.stack([I.scalar_isotropic(x, 2) for x in a]), a0 * np.eye(2), "scalar", variant)
    A = effective.effective_matrix(pb.A0, np.eye(2), [solvers.cg(pb, p, tol=1e-13, maxit=500)["tau"] for p in np.eye(2)])
    harm, arith = cf.scalar_laminate([22 / 32, 10 / 32], a)
    np.testing.assert_allclose(A, [[harm, 0], [0, arith]], atol=1e-10)


def test_scalar_laminate_odd_layers_filtered_exact_truncated_not():
    # odd thickness: filtered stays exact, truncated loses the arithmetic mean (Nyquist rule)
    ph = I.laminate((4, 16), 0, [(1, 5), (0, 11)])
    mod = np.stack([I.scalar_isotropic(1.0, 2), I.scalar_isotropic(10.0, 2)])
    harm, arith = cf.scalar_laminate([11 / 16, 5 / 16], [1.0, 10.0])
    pf = op.Problem(ph, mod, 0.5 * np.eye(2), "scalar", "filtered")
    tau = solvers.cg(pf, [0.0, 1.0], tol=1e-13)["tau"]
    assert abs(effective.mean_stress(pf.A0, [0, 1], tau)[1] - arith) < 1e-10
    pt = op.Problem(ph, mod, 0.5 * np.eye(2), "scalar", "truncated")
    tau = solvers.cg(pt, [0.0, 1.0], tol=1e-13)["tau"]
    assert abs(effective.mean_stress(pt.A0, [0, 1], tau)[1] - arith) > 1e-4


@pytest.mark.parametrize("variant", ["truncated", "filtered"])
def test_elastic_laminate(variant):
    ph = I.laminate((2, 2, 16), 0, [(1, 6), (0, 10)])
    Cm, Ci = I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)
    mu0 = 0.5 * I.lame_from_young(1.0, 0.3)[1]
    C0 = I.elastic_isotropic_mandel(2 * mu0 * 0.3 / 0.4, mu0)
    pb = op.Problem(ph, np.stack([Cm, Ci]), C0, "elastic", variant)
    taus = [solvers.cg(pb, p, tol=1e-13, maxit=500)["tau"] for p in np.eye(6)]
    A = effective.effective_matrix(C0, np.eye(6), taus)
    np.testing.assert_allclose(A, cf.elastic_laminate([10 / 16, 6 / 16], [Cm, Ci]), atol=1e-10)


def test_truncated_independent_of_a0_filtered_not():
    w = I.disk_workload(16)
    res = {}
    for variant in ("truncated", "filtered"):
        vals = []
        for a0 in (5.5, 20.0):
            pb = op.Problem(w.phase, w.moduli, a0 * np.eye(2), "scalar", variant)
            tau = solvers.cg(pb, [1.0, 0.0], tol=1e-13, maxit=2000)["tau"]
            vals.append(effective.mean_stress(pb.A0, [1.0, 0.0], tau)[0])
        res[variant] = vals
    assert abs(res["truncated"][0] - res["truncated"][1]) < 1e-10
    assert abs(res["filtered"][0] - res["filtered"][1]) > 1e-3


def test_disk_symmetry_bounds_and_basic_equals_cg():
    w = I.disk_workload(32)
    pb = op.Problem(w.phase, w.moduli, w.A0, "scalar", "truncated")
    taus = [solvers.cg(pb, p, tol=1e-12, maxit=2000)["tau"] for p in np.eye(2)]
    A = effective.effective_matrix(w.A0, np.eye(2), taus)
    assert abs(A[0, 0] - A[1, 1]) < 1e-10 and abs(A[0, 1]) < 1e-10 and abs(A[1, 0]) < 1e-10
    f = w.phase.mean()
    harm, arith = cf.scalar_laminate([1 - f, f], [1.0, 10.0])
    assert harm <= A[0, 0] <= arith
    # a0 = 5.5 is between the phases: basic scheme converges (|a - a0| < a0)
    tb = solvers.basic(pb, [1.0, 0.0], tol=1e-12)["tau"]
    assert abs(effective.mean_stress(w.A0, [1, 0], tb)[0] - A[0, 0]) < 1e-10


def test_effective_symmetric_and_voigt_reuss():
    pb = _scalar_pb((6, 6, 6), "filtered", a0=0.5, seed=2)
    taus = [solvers.cg(pb, p, tol=1e-13, maxit=500)["tau"] for p in np.eye(3)]
    A = effective.effective_matrix(pb.A0, np.eye(3), taus)
    np.testing.assert_allclose(A, A.T, atol=1e-10)
    f = pb.phase.mean()
    harm, arith = cf.scalar_laminate([1 - f, f], [1.0, 10.0])
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() >= harm - 1e-10 and ev.max() <= arith + 1e-10
    pe = _elastic_pb((4, 4, 4), "filtered", seed=3)
    taus = [solvers.cg(pe, p, tol=1e-13, maxit=500)["tau"] for p in np.eye(6)]
    C = effective.effective_matrix(pe.A0, np.eye(6), taus)
    np.testing.assert_allclose(C, C.T, atol=1e-9)


def test_cg_diagonal_increases_monotonically():
    # A0 softer than every phase: <b, e_k> = ||e_k||_L^2 decreases, so A*_pp increases
    pb = _scalar_pb((8, 8, 8), "filtered", a0=0.5, seed=4)
    p = np.array([1.0, 0.0, 0.0])
    b = op.rhs(pb, p)
    x = np.zeros_like(b)
    r = b.copy()
    d = r.copy()
    rr = op.dot(r, r)
    vals = []
    for _ in range(12):
        q = op.apply(pb, d)
        al = rr / op.dot(d, q)
        x += al * d
        r -= al * q
        vals.append(effective.mean_stress(pb.A0, p, x)[0])
        rn = op.dot(r, r)
        d = r + rn / rr * d
        rr = rn
    assert all(b2 >= b1 - 1e-14 for b1, b2 in zip(vals, vals[1:]))


def test_checkerboard_approaches_keller_dykhne():
    target = cf.keller_dykhne(1.0, 10.0)
    for variant in ("filtered", "truncated"):
        errs = []
        for n in (8, 16, 32, 64):
            ph = I.checkerboard_2d(n)
            pb = op.Problem(ph, np.stack([np.eye(2), 10 * np.eye(2)]), 0.5 * np.eye(2), "scalar", variant)
            tau = solvers.cg(pb, [1.0, 0.0], tol=1e-11, maxit=3000)["tau"]
            errs.append(abs(effective.mean_stress(pb.A0, [1, 0], tau)[0] - target))
        assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), (variant, errs)
        assert errs[-1] < 0.1 * target


def test_disk_within_hashin_shtrikman():
    w = I.disk_workload(64)
    pb = op.Problem(w.phase, w.moduli, w.A0, "scalar", "truncated")
    tau = solvers.cg(pb, [1.0, 0.0], tol=1e-10)["tau"]
    a = effective.mean_stress(w.A0, [1, 0], tau)[0]
    lo, hi = cf.hashin_shtrikman_scalar(w.phase.mean(), 10.0, 1.0, 2)
    assert lo <= a <= hi


def test_fd_and_consistent_operators_solve_and_fd_is_a0_independent():
    # Table 1: the finite-difference scheme does not depend on A0
    w = I.disk_workload(16)
    vals = []
    for a0 in (0.4, 5.5, 20.0):
        pb = op.Problem(w.phase, w.moduli, a0 * np.eye(2), "scalar", "fd")
        tau = solvers.cg(pb, [1.0, 0.0], tol=1e-13, maxit=3000)["tau"]
        vals.append(effective.mean_stress(pb.A0, [1.0, 0.0], tau)[0])
    assert max(vals) - min(vals) < 1e-10
    # both operators: FFT route = dense eq. (12) route, laminate exact
    ph = I.laminate((4, 16), 0, [(1, 6), (0, 10)])
    mod = np.stack([I.scalar_isotropic(1.0, 2), I.scalar_isotropic(10.0, 2)])
    harm, arith = cf.scalar_laminate([10 / 16, 6 / 16], [1.0, 10.0])
    pb = op.Problem(ph, mod, 0.5 * np.eye(2), "scalar", "fd")
    A = effective.effective_matrix(pb.A0, np.eye(2), [solvers.cg(pb, p, tol=1e-13)["tau"] for p in np.eye(2)])
    np.testing.assert_allclose(A, [[harm, 0], [0, arith]], atol=1e-9)
    # the cut consistent series converges slowly to the exact laminate (eq. 11)
    errs = []
    for nmax in (1, 4, 16):
        pb = op.Problem(ph, mod, 0.5 * np.eye(2), "scalar", "consistent", series=nmax)
        A = effective.effective_matrix(pb.A0, np.eye(2), [solvers.cg(pb, p, tol=1e-13)["tau"] for p in np.eye(2)])
        errs.append(np.abs(A - [[harm, 0], [0, arith]]).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.02
    for variant in ("fd", "consistent"):
        pbr = op.Problem(I.random_phases((6, 4), 2, seed=1), mod, 0.5 * np.eye(2), "scalar", variant, series=3)
        p = np.array([1.0, 0.3])
        np.testing.assert_allclose(solvers.cg(pbr, p, tol=1e-13)["tau"], dense.solve(pbr, p), atol=1e-10)
