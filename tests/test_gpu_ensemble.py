"""GPU tests of the ensemble scheduler (lsh_solve_many) and the autotuner.

* A small ensemble (16^3, 32^3, 48^3 members with per-voxel lognormal
  conductivities) against the oracle's CG, FP64 and mixed.
* Concurrent solves equal the same contexts solved one after another,
  bitwise (A*, iteration counts).
* The full ensemble (48 cubes of 64/96/128/160, Gaussian fields of
  correlation length 4, a = exp(g), mixed to 1e-6, 3 loads each): every member
  converges, its A* lies between the harmonic and arithmetic means of its
  conductivity (the Wiener bounds of the discrete problem with A0 <= A), and
  A* and the iteration counts equal those of each member solved alone.
* The autotuner: chosen shapes are valid, the cache file is written and hit,
  a foreign cache line is ignored, and results with the tuned shapes equal
  the default shapes' within FP64 rounding.
"""
import functools

import numpy as np
import pytest
import torch

from oracle import effective, gradient, solvers
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

from .gpu_util import rel_max_err

pytestmark = pytest.mark.gpu


def _member_ctx(lsh, m, precision, green="filtered", stream=True):
    ctx = lsh.Context((m.n,) * 3, "scalar", precision, max_loads=3,
                      stream=torch.cuda.Stream() if stream else None)
    ctx.set_reference(m.a0 * np.eye(3))
    ctx.set_voxel_moduli(m.a[None])
    ctx.set_green(green)
    return ctx


@functools.lru_cache(maxsize=None)
def _small_ensemble():
    members = [I.EnsembleMember(n, np.exp(I.gaussian_random_field((n,) * 3, 2.0, seed=40 + n)), 0.0)
               for n in (16, 32, 48)]
    for m in members:
        m.a0 = 0.5 * float(m.a.min())
    refs = []
    for m in members:
        vox = gradient.isotropic_moduli("scalar", m.a[None], 3)
        pb = op.Problem(np.zeros((m.n,) * 3, np.uint8), np.zeros((1, 3, 3)), m.a0 * np.eye(3), "scalar",
                        "filtered", voxel=vox)
        taus = [solvers.cg(pb, p, tol=1e-12, maxit=3000)["tau"] for p in np.eye(3)]
        refs.append(effective.effective_matrix(pb.A0, np.eye(3), taus))
    return members, refs


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_ensemble_matches_oracle(lsh, precision):
    members, refs = _small_ensemble()
    ctxs = [_member_ctx(lsh, m, precision) for m in members]
    tol = 1e-11 if precision == "fp64" else 1e-8
    reps = lsh.solve_many(ctxs, [np.eye(3)] * len(ctxs), "cg", tol=tol, maxit=3000, threads=3)
    for ctx, rep, ref in zip(ctxs, reps, refs):
        assert rep["status"] == lsh.OK and max(rep["rel_residual"]) <= tol
        assert rel_max_err(ctx.effective().T, ref) <= (1e-10 if precision == "fp64" else 1e-7)


def test_concurrent_equals_sequential(lsh):
    members = I.ensemble_workload(members=6, sizes=(64, 96), seed=5)
    ctxs = [_member_ctx(lsh, m, "mixed") for m in members]
    seq = []
    for ctx in ctxs:
        rep = ctx.solve(np.eye(3), "cg", tol=1e-6, maxit=2000)
        seq.append((ctx.effective().copy(), rep["iterations"]))
    reps = lsh.solve_many(ctxs, [np.eye(3)] * len(ctxs), "cg", tol=1e-6, maxit=2000, threads=4)
    for ctx, rep, (A, its) in zip(ctxs, reps, seq):
        assert np.array_equal(ctx.effective(), A)
        assert rep["iterations"] == its


def test_full_ensemble_converges_within_wiener_bounds(lsh):
    # the full 48-member ensemble with four members in flight: every member
    # converges within the Wiener bounds, and gives bitwise the A* and the
    # iteration counts of the same member solved alone afterwards
    members = I.ensemble_workload()
    ctxs = [_member_ctx(lsh, m, "mixed") for m in members]
    reps = lsh.solve_many(ctxs, [np.eye(3)] * len(ctxs), "cg", tol=1e-6, maxit=3000, threads=4)
    got = []
    for m, ctx, rep in zip(members, ctxs, reps):
        assert rep["status"] == lsh.OK and max(rep["rel_residual"]) <= 1e-6
        A = ctx.effective()
        harm = 1.0 / np.mean(1.0 / m.a)
        arit = float(np.mean(m.a))
        d = np.diag(A)
        assert np.all(d >= harm * (1 - 1e-5)) and np.all(d <= arit * (1 + 1e-5)), (m.n, d, harm, arit)
        assert np.abs(A - A.T).max() <= 1e-4 * np.abs(A).max()
        got.append((A.copy(), rep["iterations"]))
    for m, ctx, (A, its) in zip(members, ctxs, got):
        rep = ctx.solve(np.eye(3), "cg", tol=1e-6, maxit=3000)
        assert np.array_equal(ctx.effective(), A), m.n
        assert rep["iterations"] == its, m.n


def test_autotune_cache_and_results(lsh, tmp_path):
    m = I.ensemble_workload(members=1, sizes=(128,), seed=7)[0]
    ctx = _member_ctx(lsh, m, "mixed", stream=False)
    rep0 = ctx.solve(np.eye(3), "cg", tol=1e-8, maxit=2000)
    A0 = ctx.effective().copy()
    cache = tmp_path / "tune.txt"
    cache.write_text("some other key = 9 9 9 9 9 9 9 9\nbad line\n")
    v, hit = ctx.autotune(3, cache)
    assert not hit
    assert all(0 <= x < 4 for x in v["fp32"] + v["fp64"])
    assert ctx.variants() == v
    text = cache.read_text()
    assert "128x128x128" in text and "some other key" not in text.split("128x128x128")[0][-5:]
    ctx2 = _member_ctx(lsh, m, "mixed", stream=False)
    v2, hit2 = ctx2.autotune(3, cache)
    assert hit2 and v2 == v
    rep1 = ctx2.solve(np.eye(3), "cg", tol=1e-8, maxit=2000)
    assert rel_max_err(ctx2.effective(), A0) <= 1e-7
    assert abs(rep1["iterations"][0] - rep0["iterations"][0]) <= 2
