"""The allocation-free operator lsh_apply_noalloc against lsh_apply.

Both run the same kernels on the same inputs (the operator of eq. (13)); the
allocation-free entry point keeps the main spectrum in the caller's output
and the Nyquist plane in the library's per-GPU scratch array, so the results
must agree bit for bit.  Two calls in a row, the second on a smaller input,
check that the shared scratch carries nothing from one call to the next.
"""
import ctypes as C

import numpy as np
import pytest

from paper_1411_0330_amd import inputs as I

pytestmark = pytest.mark.gpu


def _ctx(lsh, shape, physics, precision, max_loads, green="filtered"):
    d = len(shape)
    c = 6 if physics == "elastic" else d
    if physics == "elastic":
        mod = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)])
        A0 = I.elastic_isotropic_mandel(0.2, 0.2)
    else:
        mod = np.stack([np.eye(d), 10.0 * np.eye(d)])
        A0 = 0.5 * np.eye(d)
    ctx = lsh.Context(shape, physics, precision, max_loads=max_loads)
    ctx.set_reference(A0)
    ctx.set_phases(I.random_phases(shape, 2, seed=11), mod)
    ctx.set_green(green)
    return ctx, c


def _noalloc(lsh, ctx, tau, out):
    code = lsh.F64 if str(tau.dtype) == "torch.float64" else lsh.F32
    return ctx.lib.lsh_apply_noalloc(ctx.h, tau.shape[0], C.c_void_p(tau.data_ptr()), C.c_void_p(out.data_ptr()),
                                     code)


def _random_tau(shape, nload, c, dtype, seed):
    import torch
    rng = np.random.default_rng(seed)
    t = rng.standard_normal((nload, c) + shape)
    return torch.tensor(t, dtype=dtype, device="cuda:0")


@pytest.mark.parametrize("physics,shape,precision", [
    ("scalar", (32, 48, 64), "fp64"),
    ("scalar", (32, 48, 64), "mixed"),
    ("elastic", (16, 32, 32), "fp64"),
    ("elastic", (16, 32, 32), "mixed"),
    ("scalar", (64, 128), "fp64"),
])
def test_noalloc_apply_equals_apply_twice(lsh, physics, shape, precision):
    import torch
    ctx, c = _ctx(lsh, shape, physics, precision, max_loads=3)
    dtypes = [torch.float64] + ([torch.float32] if precision == "mixed" else [])
    for dt in dtypes:
        # first call: three loads; second: one load (smaller input)
        for nload, seed in ((3, 1), (1, 2)):
            tau = _random_tau(shape, nload, c, dt, seed)
            ref = ctx.apply(tau)
            out = torch.full_like(tau, float("nan"))
            assert _noalloc(lsh, ctx, tau, out) == lsh.OK
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (physics, shape, precision, dt, nload)


def test_noalloc_second_context_smaller_grid(lsh):
    # a larger grid, then a smaller one on another context: the scratch is shared by both
    import torch
    big, c = _ctx(lsh, (64, 64, 64), "elastic", "fp64", max_loads=2)
    small, _ = _ctx(lsh, (8, 16, 16), "elastic", "fp64", max_loads=1)
    for ctx, shape, nload in ((big, (64, 64, 64), 2), (small, (8, 16, 16), 1)):
        tau = _random_tau(shape, nload, c, torch.float64, 7)
        ref = ctx.apply(tau)
        out = torch.empty_like(tau)
        assert _noalloc(lsh, ctx, tau, out) == lsh.OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


def test_noalloc_keeps_the_solution_and_refuses_oversize(lsh):
    import torch
    ctx, c = _ctx(lsh, (16, 32, 32), "scalar", "fp64", max_loads=1)
    ctx.solve(np.eye(3)[:1], "cg", tol=1e-10, maxit=500)
    A = ctx.effective().copy()
    tau_sol = ctx.field(0, "tau")
    tau = _random_tau((16, 32, 32), 1, c, torch.float64, 3)
    out = torch.empty_like(tau)
    assert _noalloc(lsh, ctx, tau, out) == lsh.OK
    np.testing.assert_array_equal(ctx.effective(), A)
    assert torch.equal(ctx.field(0, "tau"), tau_sol)
    # 512^3 elastic, three loads: a 75 MB Nyquist plane, refused before any GPU work
    huge = lsh.Context((512, 512, 512), "elastic", "fp64", max_loads=3, bind=False)
    st = huge.lib.lsh_apply_noalloc(huge.h, 3, C.c_void_p(tau.data_ptr()), C.c_void_p(out.data_ptr()), lsh.F64)
    assert st == lsh.ENOMEM
    assert b"scratch" in huge.lib.lsh_last_error(huge.h)
    # misaligned output
    st = ctx.lib.lsh_apply_noalloc(ctx.h, 1, C.c_void_p(tau.data_ptr()), C.c_void_p(out.data_ptr() + 8), lsh.F64)
    assert st == lsh.EINVAL
