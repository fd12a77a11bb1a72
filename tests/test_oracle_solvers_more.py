"""Pins of the oracle's MINRES, SYMMLQ and Eyre--Milton solvers.

* Both reach the exact solution of eq. (12) (dense LAPACK solve) on small
  grids: scalar 2D with A0 between the phases (symmetric indefinite system)
  and softer than both, anisotropic phases and reference, elasticity with an
  indefinite reference, truncated and filtered operators.
* MINRES: the residual norm phi_k never increases, and equals the true
  residual at the end.
* Eyre--Milton: for A0 = a0 Id the error contracts at every step by at most
  rho = max |(a - a0)/(a + a0)| (Euclidean norm), the bound that follows from
  0 <= a0 Gamma <= Id; at a0 = sqrt(a_min a_max) it needs fewer iterations than
  the basic scheme at its own best a0.
* SYMMLQ: reaches the dense solution; each iterate x^L_k is the orthogonal
  projection of the exact solution onto L K_k(L, b) (least error), and each
  CG point x^C_k is the Galerkin solution over K_k(L, b) -- both computed by
  brute force from explicitly orthonormalised Krylov bases -- with the
  residual the recurrence reports; on a definite system the CG points are
  the CG iterates.
* Planted mistakes in any of the solvers break one of these pins.
"""
import math

import numpy as np
import pytest

from oracle import dense, solvers
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

MODS2 = np.stack([I.scalar_isotropic(1.0, 2), I.scalar_isotropic(10.0, 2)])


def _aniso():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((2, 2))
    return np.stack([np.eye(2) + 0.2 * M @ M.T, 8.0 * np.eye(2) + np.array([[0.5, 1.0], [1.0, -0.3]])])


def _elastic_indefinite():
    ph = I.random_phases((4, 4, 4), 2, seed=3)
    mods = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)])
    lam0, mu0 = I.lame_from_young(4.0, 0.25)
    return op.Problem(ph, mods, I.elastic_isotropic_mandel(lam0, mu0), "elastic", "filtered")


def _cases():
    disk = I.disk_2d(12)
    out = []
    for a0 in (5.5, 0.5):
        for g in ("truncated", "filtered"):
            out.append((f"disk-a0={a0}-{g}", op.Problem(disk, MODS2, a0 * np.eye(2), "scalar", g), [1.0, 0.3]))
    A0 = np.array([[4.0, 0.4], [0.4, 3.5]])      # between the phases: indefinite
    out.append(("aniso-filtered", op.Problem(I.random_phases((6, 8), 2, seed=1), _aniso(), A0, "scalar",
                                             "filtered"), [0.2, 1.0]))
    out.append(("elastic-indefinite", _elastic_indefinite(), np.eye(6)[0] + 0.5 * np.eye(6)[5]))
    return out


CASES = _cases()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("name,pb,p", CASES, ids=[c[0] for c in CASES])
def test_minres_reaches_the_dense_solution_with_monotone_residuals(name, pb, p):
    exact = dense.solve(pb, p)
    hist = []
    r = solvers.minres(pb, p, tol=1e-13, maxit=2000, history=hist)
    assert _rel(r["tau"], exact) <= 1e-9
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    assert r["rel_res"] <= 1e-11 and abs(r["rel_res"] - hist[-1]) <= 1e-10


@pytest.mark.parametrize("name,pb,p", CASES, ids=[c[0] for c in CASES])
def test_eyre_milton_reaches_the_dense_solution(name, pb, p):
    exact = dense.solve(pb, p)
    r = solvers.eyre_milton(pb, p, tol=1e-13, maxit=5000)
    assert _rel(r["tau"], exact) <= 1e-10


@pytest.mark.parametrize("green", ["truncated", "filtered"])
@pytest.mark.parametrize("a0", [0.5, 3.0, 20.0])
def test_eyre_milton_contraction_bound(green, a0):
    pb = op.Problem(I.disk_2d(12), MODS2, a0 * np.eye(2), "scalar", green)
    p = [1.0, 0.0]
    exact = dense.solve(pb, p)
    rho = max(abs(a - a0) / (a + a0) for a in (1.0, 10.0))
    errs = []
    for k in range(1, 25):
        tau = solvers.eyre_milton(pb, p, tol=0.0, maxit=k)["tau"]
        errs.append(np.linalg.norm(tau - exact))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= rho * e0 * (1 + 1e-9) + 1e-13


def test_eyre_milton_at_the_geometric_mean_beats_the_basic_scheme():
    disk = I.disk_2d(16)
    em = solvers.eyre_milton(op.Problem(disk, MODS2, math.sqrt(10.0) * np.eye(2), "scalar", "filtered"),
                             [1.0, 0.0], tol=1e-10)
    bs = solvers.basic(op.Problem(disk, MODS2, 5.5 * np.eye(2), "scalar", "filtered"), [1.0, 0.0], tol=1e-10)
    assert em["iters"] < 0.7 * bs["iters"]


# planted mistakes --------------------------------------------------------
def _em_variant(pb, p, two=2.0, swap=False, tol=1e-13, maxit=5000):
    """The oracle's Eyre--Milton loop with one planted change."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    m = op.mask(pb)
    tau = np.zeros_like(b)
    delta, _, in_i0 = op.voxel_tables(pb)
    A0 = np.asarray(pb.A0)
    M = np.zeros_like(delta)
    inv = np.linalg.inv(delta[in_i0] + 2.0 * A0)
    M[in_i0] = inv @ delta[in_i0] if swap else delta[in_i0] @ inv
    pcol = np.asarray(p, dtype=np.float64).reshape((-1,) + (1,) * pb.d)
    for _ in range(maxit):
        u = pcol - op.gamma_apply(pb, tau)
        res = m * (u - op.local_apply(pb, tau))
        if math.sqrt(op.dot(res, res)) <= tol * bnorm:
            break
        y = (tau + two * np.einsum("ij,j...->i...", A0, u)).reshape(pb.c, -1)
        tau = m * np.einsum("vij,jv->iv", M, y).reshape(tau.shape)
    return {"tau": tau}


@pytest.mark.parametrize("variant", [dict(two=1.0), dict(swap=True)])
def test_planted_eyre_milton_mistake_is_caught(variant):
    bad = 0
    for name, pb, p in CASES:
        tau = _em_variant(pb, p, maxit=3000, **variant)["tau"]
        if not np.all(np.isfinite(tau)) or _rel(tau, dense.solve(pb, p)) > 1e-6:
            bad += 1
    assert bad >= 1


def _minres_variant(pb, p, drop_eps=False, delta_sign=1.0, tol=1e-13, maxit=2000):
    """The oracle's MINRES loop with one planted change."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    x = np.zeros_like(b)
    v_prev, v = np.zeros_like(b), b / bnorm
    w1, w2 = np.zeros_like(b), np.zeros_like(b)
    beta, c_prev, s_prev, delta1, eps, phi = 0.0, -1.0, 0.0, 0.0, 0.0, bnorm
    for _ in range(maxit):
        q = op.apply(pb, v)
        alpha = op.dot(v, q)
        q = q - alpha * v - beta * v_prev
        bn = math.sqrt(op.dot(q, q))
        delta2 = c_prev * delta1 + delta_sign * s_prev * alpha
        gamma1 = s_prev * delta1 - c_prev * alpha
        eps_n, delta1_n = s_prev * bn, -c_prev * bn
        g2 = math.hypot(gamma1, bn)
        c, s = gamma1 / g2, bn / g2
        t, phi = c * phi, s * phi
        w = (v - delta2 * w1 - (0.0 if drop_eps else eps) * w2) / g2
        x += t * w
        if abs(phi) <= tol * bnorm or bn == 0.0:
            break
        v_prev, v = v, q / bn
        w2, w1 = w1, w
        beta, delta1, eps, c_prev, s_prev = bn, delta1_n, eps_n, c, s
    return x


@pytest.mark.parametrize("variant", [dict(drop_eps=True), dict(delta_sign=-1.0)])
def test_planted_minres_mistake_is_caught(variant):
    name, pb, p = CASES[0]
    assert _rel(_minres_variant(pb, p), dense.solve(pb, p)) <= 1e-9       # the unplanted copy agrees
    assert _rel(_minres_variant(pb, p, **variant), dense.solve(pb, p)) > 1e-6


# SYMMLQ ------------------------------------------------------------------
@pytest.mark.parametrize("name,pb,p", CASES, ids=[c[0] for c in CASES])
def test_symmlq_reaches_the_dense_solution(name, pb, p):
    exact = dense.solve(pb, p)
    hist = []
    r = solvers.symmlq(pb, p, tol=1e-13, maxit=2000, history=hist)
    assert _rel(r["tau"], exact) <= 1e-9
    assert r["rel_res"] <= 1e-11 and abs(r["rel_res"] - hist[-1]) <= 1e-10


def _krylov_basis(pb, b, k):
    """Orthonormal basis of K_k(L, b) by Arnoldi with full re-orthogonalisation
    (columns flattened), and L applied to each basis vector."""
    shape = b.shape
    Q = [b.ravel() / np.linalg.norm(b)]
    LQ = []
    for j in range(k):
        y = op.apply(pb, Q[j].reshape(shape)).ravel()
        LQ.append(y)
        if j + 1 < k:
            for _ in range(2):
                for q in Q:
                    y = y - (q @ y) * q
            Q.append(y / np.linalg.norm(y))
    return np.stack(Q, axis=1), np.stack(LQ, axis=1)


SMALL = [
    ("disk8-indefinite", op.Problem(I.disk_2d(8), MODS2, 5.5 * np.eye(2), "scalar", "filtered"), [1.0, 0.3]),
    ("aniso-indefinite", op.Problem(I.random_phases((4, 6), 2, seed=1), _aniso(), np.array([[4.0, 0.4], [0.4, 3.5]]),
                                    "scalar", "truncated"), [0.2, 1.0]),
    ("elastic-indefinite", _elastic_indefinite(), np.eye(6)[0] + 0.5 * np.eye(6)[5]),
]


@pytest.mark.parametrize("name,pb,p", SMALL, ids=[c[0] for c in SMALL])
def test_symmlq_iterates_by_brute_force(name, pb, p):
    K = 7
    exact = dense.solve(pb, p).ravel()
    b = op.rhs(pb, p)
    its, hist = [], []
    solvers.symmlq(pb, p, tol=0.0, maxit=K + 1, history=hist, iterates=its)
    assert len(its) == K
    for k in range(1, K + 1):
        Q, LQ = _krylov_basis(pb, b, k)
        U, _ = np.linalg.qr(LQ)
        xl_ref = U @ (U.T @ exact)                                   # least error over L K_k
        xc_ref = Q @ np.linalg.solve(Q.T @ LQ, Q.T @ b.ravel())      # Galerkin over K_k
        xl, xc = its[k - 1]
        assert np.linalg.norm(xl.ravel() - xl_ref) <= 1e-8 * np.linalg.norm(xl_ref)
        assert xc is not None
        assert np.linalg.norm(xc.ravel() - xc_ref) <= 1e-8 * np.linalg.norm(xc_ref)
        rc = np.linalg.norm(b - op.apply(pb, xc)) / np.linalg.norm(b)
        assert abs(rc - hist[k - 1]) <= 1e-9 * max(1.0, rc)


def test_symmlq_cg_points_are_the_cg_iterates_on_a_definite_system():
    pb = op.Problem(I.disk_2d(10), MODS2, 0.5 * np.eye(2), "scalar", "filtered")
    p = [1.0, 0.0]
    its = []
    solvers.symmlq(pb, p, tol=0.0, maxit=12, iterates=its)
    for k in (1, 4, 11):
        x_cg = solvers.cg(pb, p, tol=0.0, maxit=k)["tau"]
        assert _rel(its[k - 1][1], x_cg) <= 1e-10


def _symmlq_variant(pb, p, wbar_sign=1.0, drop_eps=False, tol=1e-13, maxit=2000):
    """The oracle's SYMMLQ loop with one planted change."""
    b = op.rhs(pb, p)
    bnorm = math.sqrt(op.dot(b, b))
    x = np.zeros_like(b)
    v_prev, v = np.zeros_like(b), b / bnorm
    wbar = v.copy()
    beta, c_prev, s_prev, dbar, eps, z1, z2, first = 0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0, bnorm
    xc = x
    for _ in range(maxit):
        q = op.apply(pb, v)
        alpha = op.dot(v, q)
        q = q - alpha * v - beta * v_prev
        bn = math.sqrt(op.dot(q, q))
        delta = c_prev * dbar + s_prev * alpha
        gbar = s_prev * dbar - c_prev * alpha
        num = first - delta * z1 - (0.0 if drop_eps else eps) * z2
        zbar = num / gbar
        xc = x + zbar * wbar
        if bn * abs(s_prev * z1 - c_prev * zbar) <= tol * bnorm:
            break
        gamma = math.hypot(gbar, bn)
        c, s = gbar / gamma, bn / gamma
        vn = q / bn
        w = c * wbar + s * vn
        wbar = wbar_sign * s * wbar - c * vn
        x = x + (num / gamma) * w
        eps, dbar = s_prev * bn, -c_prev * bn
        v_prev, v, beta, c_prev, s_prev, z2, z1, first = v, vn, bn, c, s, z1, num / gamma, 0.0
    return xc


@pytest.mark.parametrize("variant", [dict(wbar_sign=-1.0), dict(drop_eps=True)])
def test_planted_symmlq_mistake_is_caught(variant):
    name, pb, p = SMALL[0]
    exact = dense.solve(pb, p)
    assert _rel(_symmlq_variant(pb, p), exact) <= 1e-9       # the unplanted copy agrees
    assert _rel(_symmlq_variant(pb, p, maxit=400, **variant), exact) > 1e-6
