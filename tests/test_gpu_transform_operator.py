"""GPU parity of the transform passes and of the operator of eq. (13).

* The packed half spectrum of the forward passes against numpy.fft.rfftn
  (the unnormalised DFT of Section 3.1), in FP64 and FP32, over axis lengths
  2..1024 and ragged (non-cubic) grids.
* L tau from the HIP kernels against the oracle's L tau (full complex FFTs,
  generic Green tables and per-voxel inverses) on seeded random fields:
  scalar 2D/3D with anisotropic phases, elasticity, truncated and filtered,
  a phase equal to A0 (outside I0), several loads.
* Full size: at the 256^3 elastic shape of the benchmark (6 loads, FP32 and
  FP64), plane-wave polarisations tau = a cos(2 pi k.x) whose exact image is
  1_{I0}((A - A0)^{-1} tau + Gamma_hat_k a cos(2 pi k.x)), with Gamma_hat_k
  evaluated by the oracle at those wave-vectors only.
"""
import math
import os

import numpy as np
import pytest

from oracle import green
from oracle import operator as op
from paper_1411_0330_amd import inputs as I

from .gpu_util import context, problem, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

SCAL2 = np.stack([I.scalar_isotropic(1.0, 2), I.scalar_isotropic(10.0, 2)])
SCAL3 = np.stack([I.scalar_isotropic(1.0, 3), I.scalar_isotropic(100.0, 3)])
ELAS = np.stack([I.elastic_from_young(1.0, 0.3), I.elastic_from_young(10.0, 0.2)])
MU0 = 0.5 * I.lame_from_young(1.0, 0.3)[1]
C0 = I.elastic_isotropic_mandel(2 * MU0 * 0.3 / 0.4, MU0)


@pytest.mark.parametrize("shape,physics,nload,dtype", [
    ((4, 8), "scalar", 1, "f64"),
    ((16, 4), "scalar", 2, "f64"),
    ((64, 64), "scalar", 2, "f32"),
    ((1024, 8), "scalar", 1, "f64"),
    ((8, 1024), "scalar", 1, "f32"),
    ((2, 2, 4), "scalar", 1, "f64"),
    ((8, 4, 16), "scalar", 3, "f64"),
    ((8, 4, 16), "scalar", 3, "f32"),
    ((32, 16, 64), "scalar", 1, "f32"),
    ((4, 8, 8), "elastic", 2, "f64"),
    ((16, 128, 256), "scalar", 1, "f64"),
    ((1024, 2, 4), "scalar", 1, "f64"),
    ((2, 1024, 4), "elastic", 1, "f32"),
    ((4, 4, 1024), "scalar", 1, "f32"),
    ((64, 64, 64), "elastic", 1, "f32"),
])
def test_forward_dft_matches_numpy(lsh, shape, physics, nload, dtype):
    d = len(shape)
    c = 6 if physics == "elastic" else d
    moduli = ELAS if physics == "elastic" else (SCAL2 if d == 2 else SCAL3)
    A0 = C0 if physics == "elastic" else 0.5 * np.eye(d)
    ctx = context(lsh, np.zeros(shape, np.uint8), moduli, A0, physics, "filtered",
                  precision="mixed" if dtype == "f32" else "fp64", max_loads=nload)
    f = I.random_field(shape, c, nload, seed=11)
    main, nyq = ctx.forward_dft(to_dev(f, dtype))
    ref = np.fft.rfftn(f, axes=tuple(range(2, 2 + d)))
    mx = shape[-1] // 2
    tol = 1e-12 if dtype == "f64" else 5e-6
    scale = np.abs(ref).max()
    assert np.abs(main.cpu().numpy() - ref[..., :mx]).max() <= tol * scale
    assert np.abs(nyq.cpu().numpy() - ref[..., mx]).max() <= tol * scale


def _aniso_scalar(d, seed):
    rng = np.random.default_rng(seed)
    mods = []
    for a in (1.0, 10.0, 3.0):
        M = rng.standard_normal((d, d))
        mods.append(a * np.eye(d) + 0.2 * a * (M @ M.T) / d)
    return np.stack(mods)


OP_CASES = [
    # physics, shape, green, nload, extra
    ("scalar", (16, 32), "truncated", 2, "aniso"),
    ("scalar", (8, 64), "filtered", 1, "aniso"),
    ("scalar", (8, 16, 4), "truncated", 3, "masked"),
    ("scalar", (4, 8, 16), "filtered", 2, "aniso-A0"),
    ("scalar", (32, 32, 32), "filtered", 3, ""),
    ("elastic", (8, 8, 8), "truncated", 2, "masked"),
    ("elastic", (4, 16, 8), "filtered", 6, ""),
    ("elastic", (16, 16, 16), "filtered", 1, ""),
    ("elastic", (2, 4, 32), "truncated", 1, ""),
]


def _op_setup(physics, shape, variant, extra, seed=0):
    d = len(shape)
    ph = I.random_phases(shape, 3, seed=seed)
    if physics == "elastic":
        moduli = np.stack([ELAS[0], ELAS[1], I.elastic_from_young(4.0, 0.25)])
        A0 = C0
        if extra == "masked":
            moduli[2] = C0
    else:
        moduli = _aniso_scalar(d, seed + 1)
        A0 = 0.5 * np.eye(d)
        if extra == "aniso-A0":
            A0 = np.diag(np.linspace(0.3, 0.5, d)) + 0.05 * (np.ones((d, d)) - np.eye(d))
        if extra == "masked":
            moduli[2] = A0
    return ph, moduli, A0


@pytest.mark.parametrize("physics,shape,variant,nload,extra", OP_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_matches_oracle(lsh, physics, shape, variant, nload, extra, dtype):
    ph, moduli, A0 = _op_setup(physics, shape, variant, extra)
    pb = problem(ph, moduli, A0, physics, variant)
    ctx = context(lsh, ph, moduli, A0, physics, variant, precision="mixed" if dtype == "f32" else "fp64",
                  max_loads=nload)
    m = op.mask(pb)
    tau = I.random_field(shape, pb.c, nload, seed=7) * m
    out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(nload)])
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_max_err(out, ref) <= tol
    if extra == "masked":
        assert np.all(out[:, :, ~m] == 0)


def _plane_wave_case(shape, physics, variant, nload, seed):
    """Per load: tau = sum over two wave-vectors of a_m cos(2 pi k_m.x/N), and
    the exact Gamma tau from Gamma_hat at those wave-vectors."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    c = 6 if physics == "elastic" else d
    A0 = C0 if physics == "elastic" else 0.5 * np.eye(d)
    nphys = shape[::-1]
    coords = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")   # array axes
    tau = np.zeros((nload, c) + shape)
    gam = np.zeros_like(tau)
    special = [np.zeros(d, int), np.array([n // 2 for n in nphys]), np.array([nphys[0] // 2] + [1] * (d - 1))]
    for l in range(nload):
        for mnum in range(2):
            if l < len(special) and mnum == 0:
                k = special[l]
            else:
                k = np.array([rng.integers(0, n) for n in nphys])
            amp = rng.standard_normal(c)
            phase = 2 * math.pi * sum(k[a] * coords[d - 1 - a] / nphys[a] for a in range(d))
            cosw = np.cos(phase)
            G = green.at(shape, physics, A0, variant, k[None, :])[0]
            tau[l] += amp.reshape(c, *([1] * d)) * cosw
            gam[l] += (G @ amp).reshape(c, *([1] * d)) * cosw
    return tau, gam, A0


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_full_size_plane_waves(lsh, dtype, tmp_path):
    # the benchmark's shape and batch: 256^3 elasticity, 6 loads, filtered; FP32 with the
    # benchmark's kernel shapes (the committed autotuner cache, read from a copy)
    import shutil
    shape, nload, variant = (256, 256, 256), 6, "filtered"
    w = I.elastic_rsa_workload(256)
    tau, gam, A0 = _plane_wave_case(shape, "elastic", variant, nload, seed=3)
    ctx = context(lsh, w.phase, w.moduli, A0, "elastic", variant, precision="mixed" if dtype == "f32" else "fp64",
                  max_loads=nload)
    if dtype == "f32":
        cache = tmp_path / "tune_cache.txt"
        shutil.copy(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1411_0330_amd",
                                 "tune_cache.txt"), cache)
        _, hit = ctx.autotune(nload, cache)
        assert hit
    out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
    pb = problem(w.phase, w.moduli, A0, "elastic", variant)
    _, dinv, in_i0 = op.phase_tables(pb)
    tol = 1e-11 if dtype == "f64" else 2e-5
    for l in range(nload):
        loc = np.einsum("...ij,j...->i...", dinv[w.phase], tau[l])
        ref = in_i0[w.phase] * (loc + gam[l])
        assert rel_max_err(out[l], ref) <= tol, l


@pytest.mark.timeout(600)
def test_operator_full_size_scalar_128_plane_waves(lsh):
    shape, nload, variant = (128, 128, 128), 3, "filtered"
    w = I.boolean_workload(128)
    tau, gam, A0 = _plane_wave_case(shape, "scalar", variant, nload, seed=5)
    for dtype in ("f64", "f32"):
        ctx = context(lsh, w.phase, w.moduli, A0, "scalar", variant,
                      precision="mixed" if dtype == "f32" else "fp64", max_loads=nload)
        out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
        pb = problem(w.phase, w.moduli, A0, "scalar", variant)
        _, dinv, in_i0 = op.phase_tables(pb)
        for l in range(nload):
            ref = in_i0[w.phase] * (np.einsum("...ij,j...->i...", dinv[w.phase], tau[l]) + gam[l])
            assert rel_max_err(out[l], ref) <= (1e-11 if dtype == "f64" else 2e-5)


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("physics,shape", [("scalar", (128, 8, 128)), ("scalar", (4, 128, 256)),
                                           ("elastic", (256, 4, 128)), ("elastic", (8, 256, 256))])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_kernel_shape_variants(lsh, monkeypatch, physics, shape, variant, dtype):
    # every compiled kernel shape of the 128/256-point passes gives the oracle's L tau
    bits = "64" if dtype == "f64" else "32"
    monkeypatch.setenv("LSH_TUNE", ",".join(f"{p}{bits}={variant}" for p in ("xfwd", "y", "zg", "xinv")))
    ph, moduli, A0 = _op_setup(physics, shape, "filtered", "")
    pb = problem(ph, moduli, A0, physics, "filtered")
    ctx = context(lsh, ph, moduli, A0, physics, "filtered", precision="mixed" if dtype == "f32" else "fp64",
                  max_loads=2)
    tau = I.random_field(shape, pb.c, 2, seed=9)
    out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(2)])
    assert rel_max_err(out, ref) <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("physics,shape,variant,series", [
    ("scalar", (16, 32), "fd", 8),
    ("scalar", (8, 16, 4), "fd", 8),
    ("scalar", (16, 16), "consistent", 6),
    ("scalar", (8, 8, 8), "consistent", 3),
    ("elastic", (4, 8, 8), "consistent", 2),
])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fd_and_consistent_operators_match_oracle(lsh, physics, shape, variant, series, dtype):
    ph, moduli, A0 = _op_setup(physics, shape, variant, "aniso-A0" if physics == "scalar" else "")
    pb = problem(ph, moduli, A0, physics, variant)
    pb.series = series
    ctx = lsh.Context(shape, physics, "mixed" if dtype == "f32" else "fp64", max_loads=2)
    ctx.set_reference(A0)
    ctx.set_phases(ph, moduli)
    ctx.set_green(variant, series=series)
    tau = I.random_field(shape, pb.c, 2, seed=13)
    out = ctx.apply(to_dev(tau, dtype)).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(2)])
    assert rel_max_err(out, ref) <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("green", ["truncated", "filtered", "consistent"])
@pytest.mark.parametrize("physics,shape,nload", [("scalar", (128, 8, 16), 3), ("elastic", (256, 4, 8), 4),
                                                 ("elastic", (128, 16, 32), 1)])
def test_multi_load_z_pass_matches_oracle(lsh, monkeypatch, physics, shape, nload, green):
    # z pass shape 4: every load of a tile in one workgroup, operator matrices formed once
    monkeypatch.setenv("LSH_TUNE", "zg32=4")
    ph, moduli, A0 = _op_setup(physics, shape, green, "masked")
    pb = problem(ph, moduli, A0, physics, green)
    ctx = context(lsh, ph, moduli, A0, physics, green, precision="mixed", max_loads=nload)
    if green == "consistent":
        ctx.set_green(green, series=2)
        pb.series = 2
    assert ctx.variants()["fp32"][2] == 4
    m = op.mask(pb)
    tau = I.random_field(shape, pb.c, nload, seed=21) * m
    out = ctx.apply(to_dev(tau, "f32")).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(nload)])
    assert rel_max_err(out, ref) <= 1e-5


@pytest.mark.parametrize("physics", ["elastic", "scalar"])
def test_multi_load_z_pass_in_a_batched_solve(lsh, monkeypatch, physics):
    # loads converging at different steps: frozen loads are skipped inside the
    # workgroup loop, and the fused CG step takes its p.Gamma p partials from it
    ph = I.random_phases((128, 16, 16), 2, seed=5)
    if physics == "elastic":
        moduli, A0, c = np.stack([ELAS[0], ELAS[1]]), C0, 6
    else:
        moduli, A0, c = np.stack([np.eye(3), 10.0 * np.eye(3)]), 0.5 * np.eye(3), 3
    loads = np.eye(c)[[0, c // 2, c - 1]] * np.array([[1.0], [1e-3], [5.0]])
    res = {}
    for tune in ("", "zg32=4"):
        monkeypatch.setenv("LSH_TUNE", tune)
        ctx = context(lsh, ph, moduli, A0, physics, "filtered", precision="mixed", max_loads=3)
        rep = ctx.solve(loads, "cg", tol=1e-8, maxit=2000)
        assert rep["status"] == lsh.OK
        res[tune] = (ctx.effective().copy(), rep["iterations"])
    A0_, it0 = res[""]
    A4, it4 = res["zg32=4"]
    assert rel_max_err(A4, A0_) <= 1e-7
    assert all(abs(a - b) <= 3 for a, b in zip(it0, it4))


@pytest.mark.parametrize("shape,nload,ytune", [((128, 128, 16), 2, "0"), ((128, 128, 48), 3, "3"),
                                               ((128, 256, 8), 1, "3"), ((256, 256, 16), 2, "1")])
def test_paired_z_pass_matches_oracle(lsh, monkeypatch, shape, nload, ytune):
    # z pass shape 5: the y forward pass writes the component-paired layout
    # (16 or 32 wave-vectors of two components per tile), the z pass reads and
    # writes it in 8-pencil tiles, the y inverse pass writes the plain layout
    # back; ragged tiles (mx = 24 of 32 wave-vectors in a y tile of shape 3,
    # mx = 4 of 8 pencils in a z tile), a masked phase, and y shape 1 (too
    # narrow for paired rows) falling back to shape 0
    monkeypatch.setenv("LSH_TUNE", f"zg32=5,y32={ytune}")
    ph, moduli, A0 = _op_setup("elastic", shape, "filtered", "masked")
    pb = problem(ph, moduli, A0, "elastic", "filtered")
    ctx = context(lsh, ph, moduli, A0, "elastic", "filtered", precision="mixed", max_loads=nload)
    assert ctx.variants()["fp32"][2] == 5
    m = op.mask(pb)
    tau = I.random_field(shape, pb.c, nload, seed=23) * m
    out = ctx.apply(to_dev(tau, "f32")).cpu().numpy()
    ref = np.stack([op.apply(pb, tau[l]) for l in range(nload)])
    assert rel_max_err(out, ref) <= 1e-5


@pytest.mark.parametrize("shape,fused", [((128, 128, 16), "1"), ((128, 256, 48), "1"), ((256, 128, 8), "1"),
                                         ((128, 128, 16), "0")])
def test_paired_z_pass_in_a_batched_solve(lsh, monkeypatch, shape, fused):
    # CG on the paired layout, loads converging at different steps (frozen
    # loads skipped), against the plain layout's solve: the fused step with
    # every pass in place on the paired layout (ragged x tiles: mx = 24 of 32
    # pair entries per y tile row segment, mx = 4 of 8 z pencils), and the
    # unfused step, whose y passes convert the layout
    monkeypatch.setenv("LSH_CG_FUSED", fused)
    ph = I.random_phases(shape, 2, seed=5)
    moduli, A0 = np.stack([ELAS[0], ELAS[1]]), C0
    loads = np.eye(6)[[0, 3, 5]] * np.array([[1.0], [1e-3], [5.0]])
    res = {}
    for tune in ("zg32=0", "zg32=5"):
        monkeypatch.setenv("LSH_TUNE", tune)
        ctx = context(lsh, ph, moduli, A0, "elastic", "filtered", precision="mixed", max_loads=3)
        rep = ctx.solve(loads, "cg", tol=1e-8, maxit=2000)
        assert rep["status"] == lsh.OK
        res[tune] = (ctx.effective().copy(), rep["iterations"])
    A0_, it0 = res["zg32=0"]
    A5, it5 = res["zg32=5"]
    assert rel_max_err(A5, A0_) <= 1e-7
    assert all(abs(a - b) <= 3 for a, b in zip(it0, it5))
