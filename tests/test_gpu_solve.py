"""GPU parity of the solvers (conjugate gradients, basic scheme, mixed
precision refinement) against the oracle and closed forms.

Bars: FP64 A* within 1e-10 of the FP64 oracle (relative to max|A*|), mixed
precision A* within 1e-6; fields within the same relative bars.
"""
import functools
import json
import os

import numpy as np
import pytest

from oracle import effective, solvers
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

from . import closed_forms as cf
from .gpu_util import context, problem, rel_max_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _oracle_effective(pb, loads, tol=1e-12, maxit=5000):
    taus = [solvers.cg(pb, p, tol=tol, maxit=maxit)["tau"] for p in loads]
    return effective.effective_matrix(pb.A0, loads, taus), taus


def _gpu_effective(ctx, loads, solver="cg", tol=1e-12, maxit=5000):
    rep = ctx.solve(loads, solver=solver, tol=tol, maxit=maxit)
    return ctx.effective().T, rep


def test_disk2d_cg_and_basic_fp64_against_golden_and_oracle(lsh):
    w = I.disk_workload(64, "truncated")
    gold = json.load(open(os.path.join(GOLDEN, "disk2d_n64_truncated.json")))
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=2)
    A_cg, rep = _gpu_effective(ctx, w.loads, "cg", tol=1e-12)
    assert rep["status"] == lsh.OK and max(rep["rel_residual"]) <= 1e-12
    assert rel_max_err(A_cg, gold["A_star"]) <= 1e-10
    A_b, repb = _gpu_effective(ctx, w.loads, "basic", tol=1e-12, maxit=2000)
    assert repb["status"] == lsh.OK
    assert rel_max_err(A_b, gold["A_star"]) <= 1e-10
    # the paper's setting (tol 1e-10): iteration counts match the oracle's
    rep10 = ctx.solve(w.loads, "cg", tol=1e-10)
    assert abs(rep10["iterations"][0] - gold["cg_iterations_tol1e-10"]) <= 1
    # D4 symmetry of the centred disk
    assert abs(A_cg[0, 0] - A_cg[1, 1]) < 1e-12 and abs(A_cg[0, 1]) < 1e-12


@functools.lru_cache(maxsize=None)
def _small_elastic(n=16, seed=1):
    ph, _ = I.rsa_spheres(n, 3.0, 6.0, 0.2, seed)
    return ph


@pytest.mark.parametrize("variant", ["filtered", "truncated"])
def test_elastic_small_fp64_and_mixed(lsh, variant):
    ph = _small_elastic()
    moduli = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)])
    mu0 = 0.5 * I.lame_from_young(1.0, 0.3)[1]
    C0 = I.elastic_isotropic_mandel(2 * mu0 * 0.3 / 0.4, mu0)
    loads = np.eye(6)
    pb = problem(ph, moduli, C0, "elastic", variant)
    A_ref, taus = _oracle_effective(pb, loads)
    ctx = context(lsh, ph, moduli, C0, "elastic", variant, max_loads=6)
    A, rep = _gpu_effective(ctx, loads, tol=1e-12)
    assert rep["status"] == lsh.OK
    assert rel_max_err(A, A_ref) <= 1e-10
    np.testing.assert_allclose(A, A.T, atol=1e-9 * np.abs(A).max())
    # fields
    t5 = ctx.field(5, "tau").cpu().numpy()
    assert rel_max_err(t5, taus[5]) <= 1e-9
    eps = ctx.field(5, "strain", dtype="f32", device=False)
    assert rel_max_err(eps, op.strain(pb, loads[5], taus[5])) <= 1e-6
    # mixed precision: FP32 fields, FP64 refinement to 1e-10
    ctxm = context(lsh, ph, moduli, C0, "elastic", variant, precision="mixed", max_loads=6)
    Am, repm = _gpu_effective(ctxm, loads, tol=1e-10)
    assert repm["status"] == lsh.OK and max(repm["rel_residual"]) <= 1e-10
    assert repm["outer_iterations"] >= 2 and repm["applications_fp32"] > 0
    assert rel_max_err(Am, A_ref) <= 1e-6


def test_scalar3d_boolean_fp64_mixed_batched(lsh):
    w = I.boolean_workload(32, seed=2)
    pb = problem(w.phase, w.moduli, w.A0, "scalar", "filtered")
    A_ref, _ = _oracle_effective(pb, w.loads)
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "filtered", max_loads=3)
    A, rep = _gpu_effective(ctx, w.loads, tol=1e-12)
    assert rel_max_err(A, A_ref) <= 1e-10
    # a load solved alone gives bitwise the same answer as in the batch
    A1, _ = _gpu_effective(ctx, w.loads[1:2], tol=1e-12)
    assert np.array_equal(A1[:, 0], A[:, 1])
    # determinism: same solve twice, bitwise equal
    A2, _ = _gpu_effective(ctx, w.loads, tol=1e-12)
    assert np.array_equal(A2, A)
    ctxm = context(lsh, w.phase, w.moduli, w.A0, "scalar", "filtered", precision="mixed", max_loads=3)
    Am, repm = _gpu_effective(ctxm, w.loads, tol=1e-9)
    assert max(repm["rel_residual"]) <= 1e-9
    assert rel_max_err(Am, A_ref) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_homogeneous_and_zero_correction(lsh, precision):
    shape = (8, 8, 16)
    a, a0 = 3.0, 1.25
    ctx = context(lsh, np.zeros(shape, np.uint8), np.stack([a * np.eye(3)]), a0 * np.eye(3), "scalar", "filtered",
                  precision=precision, max_loads=3)
    A, rep = _gpu_effective(ctx, np.eye(3), tol=1e-12)
    np.testing.assert_allclose(A, a * np.eye(3), atol=1e-12)
    if precision == "fp64":
        assert rep["iterations"] == [1, 1, 1]
    # every voxel equals A0: I0 empty, tau = 0, A* = A0, no iteration
    ctx = context(lsh, np.zeros(shape, np.uint8), np.stack([a0 * np.eye(3)]), a0 * np.eye(3), "scalar", "truncated",
                  precision=precision, max_loads=3)
    A, rep = _gpu_effective(ctx, np.eye(3), tol=1e-12)
    assert rep["status"] == lsh.OK
    np.testing.assert_array_equal(A, a0 * np.eye(3))
    assert np.all(ctx.field(0).cpu().numpy() == 0)


@pytest.mark.parametrize("variant", ["truncated", "filtered"])
def test_laminates_match_closed_forms(lsh, variant):
    ph = I.laminate((4, 8, 32), 0, [(1, 10), (0, 22)])
    mod = np.stack([I.scalar_isotropic(1.0, 3), I.scalar_isotropic(10.0, 3)])
    ctx = context(lsh, ph, mod, 0.5 * np.eye(3), "scalar", variant, max_loads=3)
    A, _ = _gpu_effective(ctx, np.eye(3), tol=1e-13)
    harm, arith = cf.scalar_laminate([22 / 32, 10 / 32], [1.0, 10.0])
    np.testing.assert_allclose(A, np.diag([harm, arith, arith]), atol=1e-10)
    phe = I.laminate((2, 2, 16), 0, [(1, 6), (0, 10)])
    Cm, Ci = I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)
    C0 = I.elastic_isotropic_mandel(0.2, 0.15)
    ctx = context(lsh, phe, np.stack([Cm, Ci]), C0, "elastic", variant, precision="mixed", max_loads=6)
    A, _ = _gpu_effective(ctx, np.eye(6), tol=1e-10)
    np.testing.assert_allclose(A, cf.elastic_laminate([10 / 16, 6 / 16], [Cm, Ci]), atol=1e-7)


def test_maxit_reports_unconverged(lsh):
    w = I.disk_workload(32, "truncated")
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=2)
    rep = ctx.solve(w.loads, "cg", tol=1e-12, maxit=3)
    assert rep["status"] == lsh.MAXIT
    assert rep["iterations"] == [3, 3]
    assert all(r > 1e-12 for r in rep["rel_residual"])
    # the unconverged iterate matches the oracle's after the same 3 iterations
    pb = problem(w.phase, w.moduli, w.A0, "scalar", "truncated")
    ref = solvers.cg(pb, w.loads[0], tol=1e-12, maxit=3)
    assert rel_max_err(ctx.field(0).cpu().numpy(), ref["tau"]) <= 1e-10


@pytest.mark.parametrize("graphs", [True, False])
def test_multikernel_cg_iterates_match_oracle_at_every_stop(lsh, graphs):
    # the fused step of the multi-kernel loop applies the solution updates of
    # its steps in pairs; stopping after an odd or an even number of steps must
    # give the oracle's k-th CG iterate (both loads, pending steps flushed)
    w = I.disk_workload(32, "truncated")
    pb = problem(w.phase, w.moduli, w.A0, "scalar", "truncated")
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "truncated", max_loads=2)
    ctx.set_persistent(False)
    ctx.set_graphs(graphs)
    for k in (1, 2, 3, 4, 5, 8):
        rep = ctx.solve(w.loads, "cg", tol=1e-14, maxit=k)
        assert rep["iterations"] == [k, k]
        for l in range(2):
            ref = solvers.cg(pb, w.loads[l], tol=1e-14, maxit=k)
            assert rel_max_err(ctx.field(l).cpu().numpy(), ref["tau"]) <= 1e-10, (k, l)


def test_boolean_128_fp64_and_mixed_against_golden(lsh):
    gold = json.load(open(os.path.join(GOLDEN, "boolean3d_n128_filtered.json")))
    w = I.boolean_workload(128)
    ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "filtered", max_loads=3)
    A, rep = _gpu_effective(ctx, w.loads, tol=1e-11)
    assert rep["status"] == lsh.OK
    assert rel_max_err(A, gold["A_star"]) <= 1e-10
    ctxm = context(lsh, w.phase, w.moduli, w.A0, "scalar", "filtered", precision="mixed", max_loads=3)
    Am, repm = _gpu_effective(ctxm, w.loads, tol=1e-8)
    assert max(repm["rel_residual"]) <= 1e-8
    assert rel_max_err(Am, gold["A_star"]) <= 1e-6


def test_elastic_rsa_64_fp64_and_mixed_against_golden(lsh):
    gold = json.load(open(os.path.join(GOLDEN, "elastic_rsa_n64_filtered.json")))
    w = I.elastic_rsa_workload(64, tol=1e-10)
    ctx = context(lsh, w.phase, w.moduli, w.A0, "elastic", "filtered", max_loads=6)
    A, rep = _gpu_effective(ctx, w.loads, tol=1e-11)
    assert rep["status"] == lsh.OK
    assert rel_max_err(A, gold["A_star"]) <= 1e-10
    ctxm = context(lsh, w.phase, w.moduli, w.A0, "elastic", "filtered", precision="mixed", max_loads=6)
    Am, repm = _gpu_effective(ctxm, w.loads, tol=1e-8)
    assert max(repm["rel_residual"]) <= 1e-8
    assert rel_max_err(Am, gold["A_star"]) <= 1e-6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager(lsh, precision):
    # the captured iteration replays across solves, with eager work in between,
    # and gives bitwise the results of the eager launches
    w = I.boolean_workload(32, seed=3)
    def run(graphs):
        ctx = context(lsh, w.phase, w.moduli, w.A0, "scalar", "filtered", precision=precision, max_loads=3)
        ctx.set_persistent(False)      # the multi-kernel loop is what graphs capture
        ctx.set_graphs(graphs)
        outs = []
        for rep in range(3):
            r = ctx.solve(w.loads, "cg", tol=1e-10 if precision == "fp64" else 1e-8)
            outs.append((ctx.effective().copy(), ctx.field(1).cpu().numpy(), r["iterations"]))
            ctx.apply(ctx.field(0).reshape((1,) + ctx.field(0).shape).contiguous())   # eager work between replays
        return outs
    eager, graph = run(False), run(True)
    for (a1, f1, i1), (a2, f2, i2) in zip(eager, graph):
        assert np.array_equal(a1, a2) and np.array_equal(f1, f2) and i1 == i2
    assert np.array_equal(graph[0][0], graph[2][0])
    # basic scheme too
    w2 = I.disk_workload(32, "truncated")
    res = []
    for graphs in (False, True):
        ctx = context(lsh, w2.phase, w2.moduli, w2.A0, "scalar", "truncated", precision=precision, max_loads=2)
        ctx.set_persistent(False)
        ctx.set_graphs(graphs)
        ctx.solve(w2.loads, "basic", tol=1e-10, maxit=3000)
        res.append(ctx.effective())
    assert np.array_equal(res[0], res[1])


def test_fd_and_consistent_solves_match_oracle(lsh):
    w = I.disk_workload(32, "truncated")
    for variant, a0s in (("fd", (0.5, 5.5)), ("consistent", (5.5,))):
        vals = []
        for a0 in a0s:
            pb = problem(w.phase, w.moduli, a0 * np.eye(2), "scalar", variant)
            pb.series = 6
            A_ref, _ = _oracle_effective(pb, w.loads)
            ctx = lsh.Context(w.phase.shape, "scalar", "fp64", max_loads=2)
            ctx.set_reference(a0 * np.eye(2))
            ctx.set_phases(w.phase, w.moduli)
            ctx.set_green(variant, series=6)
            A, rep = _gpu_effective(ctx, w.loads, tol=1e-12)
            assert rel_max_err(A, A_ref) <= 1e-10
            vals.append(A[0, 0])
        if variant == "fd":   # Table 1: independent of A0
            assert abs(vals[0] - vals[1]) < 1e-10


def test_full_size_elastic_rsa_256_mixed_against_fp64_and_bounds(lsh, tmp_path):
    # the benchmark's workload and launch configuration: 256^3, six loads, filtered, mixed CG to 1e-6,
    # kernel shapes from the committed autotuner cache (a copy, so that nothing writes the package file).
    # The oracle cannot solve 256^3 in a test; the reference is the GPU's FP64 path solved to 1e-10, whose
    # kernels are oracle-pinned at 64^3 and 128^3 (A* within 1e-10) and at this size by the plane-wave
    # operator test (1e-11).  Target: the mixed A* within 1e-6 of it (max|dC*| / max|C*|, Theorem 4).
    w = I.elastic_rsa_workload(256, tol=1e-6)
    import shutil
    import torch
    cache = tmp_path / "tune_cache.txt"
    shutil.copy(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1411_0330_amd",
                             "tune_cache.txt"), cache)
    phase_dev = torch.from_numpy(w.phase).to("cuda:0")
    res = {}
    for precision, tol in (("mixed", 1e-6), ("fp64", 1e-10)):
        ctx = lsh.Context(w.phase.shape, "elastic", precision, max_loads=6)
        ctx.set_reference(w.A0)
        ctx.set_phases(phase_dev, w.moduli)
        ctx.set_green("filtered")
        if precision == "mixed":
            _, hit = ctx.autotune(6, cache)
            assert hit
        rep = ctx.solve(w.loads, "cg", tol=tol, maxit=3000)
        assert rep["status"] == lsh.OK and max(rep["rel_residual"]) <= tol
        res[precision] = ctx.effective().T.copy()
        del ctx
        torch.cuda.empty_cache()
    C, C64 = res["mixed"], res["fp64"]
    assert rel_max_err(C, C64) <= 1e-6
    assert np.abs(C64 - C64.T).max() <= 1e-7 * np.abs(C64).max()
    # Voigt and Reuss bounds of the discrete problem (A0 softer than both phases)
    f = float(w.phase.mean())
    Cv = (1 - f) * w.moduli[0] + f * w.moduli[1]
    Cr = np.linalg.inv((1 - f) * np.linalg.inv(w.moduli[0]) + f * np.linalg.inv(w.moduli[1]))
    for i in range(6):
        assert Cr[i, i] * (1 - 1e-9) <= C64[i, i] <= Cv[i, i] * (1 + 1e-9)
    # Hashin-Shtrikman band for the bulk and shear estimates of the isotropic part
    K = (C64[:3, :3].sum()) / 9.0
    mu = (np.trace(C64) - C64[:3, :3].sum() / 3.0) / 10.0
    assert 1.243 <= K <= 1.767 and 0.650 <= mu <= 1.102, (K, mu)


@pytest.mark.parametrize("green", ["filtered", "truncated"])
def test_checkerboard_converges_to_keller_dykhne_on_large_grids(lsh, green):
    # the 2D checkerboard's effective conductivity is sqrt(a1 a2) (Keller-Dykhne); the
    # discrete A*_h approaches it as the grid is refined (O(h) trend, Section 5)
    target = cf.keller_dykhne(1.0, 10.0)
    errs = []
    for n in (64, 128, 256, 512):
        ph = I.checkerboard_2d(n)
        ctx = context(lsh, ph, np.stack([np.eye(2), 10.0 * np.eye(2)]), 0.5 * np.eye(2), "scalar", green)
        rep = ctx.solve(np.array([[1.0, 0.0]]), "cg", tol=1e-10, maxit=20000)
        assert rep["status"] == lsh.OK
        errs.append(abs(ctx.effective()[0][0] - target))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.5 * errs[0], errs
