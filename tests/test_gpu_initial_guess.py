"""GPU tests of warm starts (lsh_set_initial_guess).

* From the converged solution every solver stops at once: CG (FP64), MINRES
  and SYMMLQ take no iteration, mixed-precision CG no FP32 application, the
  fixed-point schemes one step; A* is unchanged.
* From a perturbed oracle solution every solver reaches the oracle's A* with
  fewer iterations than from zero.
* Values outside I0 are ignored (a guess that vanishes on I0 is the zero
  start); a guess applies to one solve; None clears it; an FP32 device guess
  and an FP64 host guess reach the same A*; bad slots are refused and the
  fields of the previous solve are gone once a guess overwrites them.
"""
import numpy as np
import pytest

from oracle import effective, solvers
from paper_1411_0330_amd import inputs as I

from .gpu_util import context, problem, rel_max_err

pytestmark = pytest.mark.gpu
LOADS = np.array([[1.0, 0.0], [0.3, 1.0]])
CASES = [("cg", "fp64"), ("cg", "mixed"), ("minres", "fp64"), ("symmlq", "fp64"), ("basic", "fp64"),
         ("eyre_milton", "fp64")]


def _disk():
    w = I.disk_workload(32, "filtered")
    return w.phase, w.moduli, 5.5 * np.eye(2)      # A0 between the phases: indefinite, basic scheme contracts


@pytest.mark.parametrize("solver,precision", CASES)
def test_converged_guess_stops_at_once(lsh, solver, precision):
    ph, mods, A0 = _disk()
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", precision=precision, max_loads=2)
    ctx.solve(LOADS, solver, tol=1e-11, maxit=5000)
    A1 = ctx.effective().copy()
    taus = [ctx.field(l, "tau", device=False) for l in range(2)]
    for l in range(2):
        ctx.set_initial_guess(l, taus[l])
    rep = ctx.solve(LOADS, solver, tol=1e-8, maxit=5000)
    assert rep["status"] == lsh.OK
    if solver in ("basic", "eyre_milton"):
        assert max(rep["iterations"]) <= 1
    elif precision == "mixed":
        assert rep["applications_fp32"] == 0
    else:
        assert rep["iterations"] == [0, 0]
    assert max(rep["rel_residual"]) <= 1e-8
    assert rel_max_err(ctx.effective(), A1) <= 1e-9


@pytest.mark.parametrize("solver,precision", CASES)
def test_perturbed_guess_reaches_the_oracle(lsh, solver, precision):
    ph, mods, A0 = _disk()
    pb = problem(ph, mods, A0, "scalar", "filtered")
    exact = [solvers.cg(pb, p, tol=1e-13, maxit=5000)["tau"] for p in LOADS]
    A_ref = effective.effective_matrix(A0, LOADS, exact)
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", precision=precision, max_loads=2)
    cold = ctx.solve(LOADS, solver, tol=1e-10, maxit=5000)
    rng = np.random.default_rng(7)
    for l in range(2):
        ctx.set_initial_guess(l, exact[l] * (1.0 + 1e-3 * rng.standard_normal(exact[l].shape)))
    warm = ctx.solve(LOADS, solver, tol=1e-10, maxit=5000)
    assert warm["status"] == lsh.OK and max(warm["rel_residual"]) <= 1e-10
    assert rel_max_err(ctx.effective().T, A_ref) <= 1e-8
    assert all(w < c for w, c in zip(warm["iterations"], cold["iterations"]))


def test_values_outside_I0_are_ignored(lsh):
    # phase 0 equals A0: those voxels lie outside I0
    ph = I.disk_workload(32, "filtered").phase
    mods = np.stack([np.eye(2), 10.0 * np.eye(2)])
    A0 = np.eye(2)
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", max_loads=2)
    cold = ctx.solve(LOADS, "cg", tol=1e-10, maxit=2000)
    A_cold = ctx.effective().copy()
    junk = np.random.default_rng(3).standard_normal((2,) + ph.shape) * 100.0
    junk[:, ph == 1] = 0.0                           # zero on I0, junk elsewhere
    for l in range(2):
        ctx.set_initial_guess(l, junk)
    warm = ctx.solve(LOADS, "cg", tol=1e-10, maxit=2000)
    assert warm["iterations"] == cold["iterations"]
    assert rel_max_err(ctx.effective(), A_cold) <= 1e-13


def test_guess_applies_once_and_clears(lsh):
    ph, mods, A0 = _disk()
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", max_loads=2)
    fresh = ctx.solve(LOADS, "cg", tol=1e-10, maxit=2000)["iterations"]
    taus = [ctx.field(l, "tau", device=False) for l in range(2)]
    ctx.set_initial_guess(0, taus[0])
    ctx.set_initial_guess(1, taus[1])
    assert ctx.solve(LOADS, "cg", tol=1e-8, maxit=2000)["iterations"] == [0, 0]
    assert ctx.solve(LOADS, "cg", tol=1e-10, maxit=2000)["iterations"] == fresh      # consumed
    ctx.set_initial_guess(0, taus[0])
    ctx.set_initial_guess(0, None)                                                   # cleared
    assert ctx.solve(LOADS, "cg", tol=1e-10, maxit=2000)["iterations"] == fresh


def test_fp32_device_and_fp64_host_guesses(lsh):
    import torch
    ph, mods, A0 = _disk()
    pb = problem(ph, mods, A0, "scalar", "filtered")
    exact = [solvers.cg(pb, p, tol=1e-13, maxit=5000)["tau"] for p in LOADS]
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", precision="mixed", max_loads=2)
    ctx.set_initial_guess(0, torch.tensor(0.9 * exact[0], dtype=torch.float32, device="cuda:0"))
    ctx.set_initial_guess(1, 0.9 * exact[1])
    rep = ctx.solve(LOADS, "cg", tol=1e-10, maxit=5000)
    assert rep["status"] == lsh.OK
    assert rel_max_err(ctx.effective().T, effective.effective_matrix(A0, LOADS, exact)) <= 1e-8


def test_guess_errors(lsh):
    ph, mods, A0 = _disk()
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", max_loads=2)
    ctx.solve(LOADS, "cg", tol=1e-8, maxit=2000)
    tau = ctx.field(0, "tau", device=False)
    with pytest.raises(lsh.LshError) as e:
        ctx.set_initial_guess(2, tau)
    assert e.value.status == lsh.EINVAL
    with pytest.raises(ValueError):
        ctx.set_initial_guess(0, tau[:1])
    ctx.set_initial_guess(0, tau)
    with pytest.raises(lsh.LshError) as e:
        ctx.field(0, "tau", device=False)
    assert e.value.status == lsh.ESTATE


@pytest.mark.parametrize("solver,precision", [("cg", "fp64"), ("cg", "mixed"), ("symmlq", "fp64")])
def test_resume_after_the_iteration_limit(lsh, solver, precision):
    # checkpoint / resume: stop at maxit, read tau, restart from it
    ph, mods, A0 = _disk()
    pb = problem(ph, mods, A0, "scalar", "filtered")
    exact = [solvers.cg(pb, p, tol=1e-13, maxit=5000)["tau"] for p in LOADS]
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", precision=precision, max_loads=2)
    first = ctx.solve(LOADS, solver, tol=1e-10, maxit=12)
    assert first["status"] == lsh.MAXIT
    taus = [ctx.field(l, "tau", device=False) for l in range(2)]
    for l in range(2):
        ctx.set_initial_guess(l, taus[l])
    rest = ctx.solve(LOADS, solver, tol=1e-10, maxit=5000)
    assert rest["status"] == lsh.OK and max(rest["rel_residual"]) <= 1e-10
    assert rel_max_err(ctx.effective().T, effective.effective_matrix(A0, LOADS, exact)) <= 1e-8


@pytest.mark.parametrize("solver", ["cg", "symmlq", "basic"])
def test_zero_load_ignores_its_guess(lsh, solver):
    # the solution of a zero load is zero whatever the guess
    ph, mods, A0 = _disk()
    ctx = context(lsh, ph, mods, A0, "scalar", "filtered", max_loads=2)
    ctx.solve(LOADS, solver, tol=1e-10, maxit=5000)
    tau = ctx.field(1, "tau", device=False)
    ctx.set_initial_guess(1, tau)
    rep = ctx.solve(np.array([[1.0, 0.0], [0.0, 0.0]]), solver, tol=1e-10, maxit=5000)
    assert rep["load_status"][1] == lsh.OK and rep["iterations"][1] == 0
    assert np.all(ctx.field(1, "tau", device=False) == 0.0)
    assert np.all(ctx.effective()[1] == 0.0)
