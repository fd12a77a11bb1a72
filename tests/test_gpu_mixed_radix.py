"""GPU parity at axis lengths with the odd factors 3 and 5 (48, 96, 192, 80,
160): the mixed-radix pencil FFTs against numpy.fft.rfftn, the operator of
eq. (13) against the oracle, and a CG solve against the oracle's CG.

These are the ensemble sizes 96 and 160 and the 192^3 grid of the gradient
workload, plus ragged combinations of them with powers of two.
"""
import functools

import numpy as np
import pytest

from oracle import effective, solvers
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

from .gpu_util import context, problem, rel_max_err, to_dev
from .test_gpu_transform_operator import C0, ELAS, SCAL2, SCAL3, _op_setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,physics,nload,dtype", [
    ((96, 48), "scalar", 2, "f64"),
    ((80, 160), "scalar", 1, "f32"),
    ((192, 96), "scalar", 1, "f64"),
    ((2, 160, 80), "scalar", 1, "f64"),
    ((48, 8, 96), "scalar", 2, "f32"),
    ((160, 96, 48), "scalar", 1, "f64"),
    ((192, 4, 192), "scalar", 1, "f32"),
    ((8, 80, 16), "elastic", 1, "f64"),
    ((96, 48, 80), "elastic", 1, "f32"),
    ((48, 48, 160), "elastic", 1, "f64"),
    ((192, 16, 64), "elastic", 2, "f32"),
])
def test_mixed_radix_forward_dft_matches_numpy(lsh, shape, physics, nload, dtype):
    d = len(shape)
    c = 6 if physics == "elastic" else d
    moduli = ELAS if physics == "elastic" else (SCAL2 if d == 2 else SCAL3)
    A0 = C0 if physics == "elastic" else 0.5 * np.eye(d)
    ctx = context(lsh, np.zeros(shape, np.uint8), moduli, A0, physics, "filtered",
                  precision="mixed" if dtype == "f32" else "fp64", max_loads=nload)
    f = I.random_field(shape, c, nload, seed=13)
    main, nyq = ctx.forward_dft(to_dev(f, dtype))
    ref = np.fft.rfftn(f, axes=tuple(range(2, 2 + d)))
    mx = shape[-1] // 2
    tol = 1e-12 if dtype == "f64" else 5e-6
    scale = np.abs(ref).max()
    assert np.abs(main.cpu().numpy() - ref[..., :mx]).max() <= tol * scale
    assert np.abs(nyq.cpu().numpy() - ref[..., mx]).max() <= tol * scale


@pytest.mark.parametrize("physics,shape,variant,nload,extra", [
    ("scalar", (96, 80), "truncated", 2, "aniso"),
    ("scalar", (48, 160), "filtered", 1, ""),
    ("scalar", (80, 48, 96), "filtered", 3, "aniso-A0"),
    ("scalar", (8, 96, 48), "truncated", 1, "masked"),
    ("scalar", (48, 80, 48), "consistent", 1, ""),
    ("scalar", (160, 48), "fd", 2, ""),
    ("elastic", (48, 48, 48), "filtered", 2, ""),
    ("elastic", (16, 80, 96), "truncated", 1, "masked"),
])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_mixed_radix_operator_matches_oracle(lsh, physics, shape, variant, nload, extra, dtype):
    ph, moduli, A0 = _op_setup(physics, shape, variant, extra)
    pb = problem(ph, moduli, A0, physics, variant)
    ctx = context(lsh, ph, moduli, A0, physics, variant, precision="mixed" if dtype == "f32" else "fp64",
                  max_loads=nload)
    m = op.mask(pb)
    tau = I.random_field(shape, pb.c, nload, seed=17) * m
    out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(nload)])
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_max_err(out, ref) <= tol
    if extra == "masked":
        assert np.all(out[:, :, ~m] == 0)


@functools.lru_cache(maxsize=None)
def _boolean_box():
    # overlapping spheres in a 48 x 48 x 80 cell, contrast 100, softer reference (SPD)
    shape = (48, 48, 80)
    phase, _ = I.boolean_spheres(shape, radius=4.0, fraction=0.25, seed=4)
    A0 = 0.5 * np.eye(3)
    loads = np.eye(3)[[0, 2]]
    pb = problem(phase, SCAL3, A0, "scalar", "filtered")
    taus = [solvers.cg(pb, p, tol=1e-12, maxit=4000)["tau"] for p in loads]
    return phase, A0, loads, effective.effective_matrix(A0, loads, taus)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mixed_radix_boolean_solve_matches_oracle(lsh, precision):
    phase, A0, loads, Aref = _boolean_box()
    ctx = context(lsh, phase, SCAL3, A0, "scalar", "filtered", precision=precision, max_loads=2)
    tol = 1e-10 if precision == "fp64" else 1e-8
    rep = ctx.solve(loads, "cg", tol=tol, maxit=2000)
    assert rep["status"] == lsh.OK and max(rep["rel_residual"]) <= tol
    assert rel_max_err(ctx.effective().T, Aref) <= (1e-9 if precision == "fp64" else 1e-7)
