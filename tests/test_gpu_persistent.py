"""GPU parity of the persistent CG launch (one workgroup per load runs the
whole loop) for small grids.

* Against the multi-kernel loop on the same context: A* within rounding and
  iteration counts within one, for every persistent grid (squares 8..64,
  cubes of 8, scalar cubes of 16), scalar and elastic, FP64 and mixed, phase
  maps and per-voxel moduli, truncated/filtered/consistent operators.
* Against the oracle (64^2 disk) and the stored disk A*.
* Loads that converge at different steps, a zero load, maxit, and an
  indefinite system (A0 between the phases).
"""
import json
import os

import numpy as np
import pytest

from oracle import effective, solvers
from paper_1411_0330_amd import inputs as I

from .gpu_util import context, problem, rel_max_err
from .test_gpu_transform_operator import C0, ELAS, _op_setup

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pair(lsh, ph, moduli, A0, physics, green, precision, loads, tol, maxit=3000, series=None):
    out = []
    for persistent in (True, False):
        ctx = context(lsh, ph, moduli, A0, physics, green, precision=precision, max_loads=len(loads))
        if series is not None:
            ctx.set_green(green, series=series)
        ctx.set_persistent(persistent)
        rep = ctx.solve(loads, "cg", tol=tol, maxit=maxit)
        out.append((ctx.effective().copy(), rep))
    return out


@pytest.mark.parametrize("physics,shape", [("scalar", (8, 8)), ("scalar", (16, 16)), ("scalar", (32, 32)),
                                           ("scalar", (64, 64)), ("scalar", (8, 8, 8)), ("scalar", (16, 16, 16)),
                                           ("elastic", (8, 8, 8)),
                                           # beyond the persistent grids: the multi-kernel loop runs either way
                                           ("scalar", (32, 32, 32)), ("elastic", (16, 16, 16))])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_persistent_matches_multi_kernel_loop(lsh, physics, shape, precision):
    ph, moduli, A0 = _op_setup(physics, shape, "filtered", "masked")
    c = 6 if physics == "elastic" else len(shape)
    loads = np.eye(c)[:2] * np.array([[1.0], [1e-2]])
    tol = 1e-11 if precision == "fp64" else 1e-8
    (Ap, rp), (Am, rm) = _pair(lsh, ph, moduli, A0, physics, "filtered", precision, loads, tol)
    assert rp["status"] == lsh.OK and rm["status"] == lsh.OK
    assert max(rp["rel_residual"]) <= tol
    assert rel_max_err(Ap, Am) <= (1e-10 if precision == "fp64" else 1e-7)
    assert all(abs(a - b) <= 1 for a, b in zip(rp["iterations"], rm["iterations"]))


@pytest.mark.parametrize("green,series", [("truncated", None), ("consistent", 2)])
def test_persistent_other_operators_and_voxel_moduli(lsh, green, series):
    ph, moduli, A0 = _op_setup("elastic", (8, 8, 8), green, "")
    loads = np.eye(6)[[0, 5]]
    (Ap, rp), (Am, rm) = _pair(lsh, ph, moduli, A0, "elastic", green, "fp64", loads, 1e-11, series=series)
    assert rel_max_err(Ap, Am) <= 1e-10
    # per-voxel scalar moduli
    rng = np.random.default_rng(3)
    coef = rng.uniform(1.0, 10.0, size=(1, 32, 32))
    res = []
    for persistent in (True, False):
        ctx = lsh.Context((32, 32), "scalar", "fp64", max_loads=2)
        ctx.set_reference(0.5 * np.eye(2))
        ctx.set_voxel_moduli(coef)
        ctx.set_green("filtered")
        ctx.set_persistent(persistent)
        ctx.solve(np.eye(2), "cg", tol=1e-12)
        res.append(ctx.effective())
    assert rel_max_err(res[0], res[1]) <= 1e-10


def test_persistent_disk_against_golden_and_oracle(lsh):
    gold = json.load(open(os.path.join(GOLDEN, "disk2d_n64_truncated.json")))
    w = I.disk_workload(64, "truncated")
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=2)
    rep = ctx.solve(w.loads, "cg", tol=1e-12)
    assert rep["status"] == lsh.OK
    assert rel_max_err(ctx.effective().T, gold["A_star"]) <= 1e-10
    rep10 = ctx.solve(w.loads, "cg", tol=1e-10)
    assert abs(rep10["iterations"][0] - gold["cg_iterations_tol1e-10"]) <= 1
    # elastic 8^3 against the oracle
    ph = I.random_phases((8, 8, 8), 2, seed=6)
    mods = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)])
    pb = problem(ph, mods, C0, "elastic", "filtered")
    loads = np.eye(6)[[0, 3]]
    taus = [solvers.cg(pb, p, tol=1e-12, maxit=2000)["tau"] for p in loads]
    ctx = context(lsh, ph, mods, C0, "elastic", "filtered", max_loads=2)
    ctx.solve(loads, "cg", tol=1e-12)
    assert rel_max_err(ctx.effective().T, effective.effective_matrix(C0, loads, taus)) <= 1e-10


def test_persistent_edge_cases(lsh):
    w = I.disk_workload(32, "truncated")
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=3)
    rep = ctx.solve(np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 1.0]]), "cg", tol=1e-12, maxit=7)
    assert rep["status"] == lsh.MAXIT
    assert rep["load_status"] == [lsh.MAXIT, lsh.OK, lsh.MAXIT]
    assert rep["iterations"] == [7, 0, 7]
    assert np.all(ctx.effective()[1] == 0.0)
    # the MAXIT iterate equals the multi-kernel loop's
    ctx2 = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=3)
    ctx2.set_persistent(False)
    ctx2.solve(np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 1.0]]), "cg", tol=1e-12, maxit=7)
    assert rel_max_err(ctx.effective(), ctx2.effective()) <= 1e-12
