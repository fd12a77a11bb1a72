"""Seeded synthetic inputs: microstructures, phase moduli and macroscopic loads.

This module builds the *inputs* of the corrector problem (Section 2.1) and
nothing else: voxel phase maps, per-phase moduli matrices and the macroscopic
gradients/strains p. It holds none of the solver's arithmetic (no Green
operator, no transform, no local inverse, no effective-tensor formula), so both
the HIP product path and the CPU oracle may consume what it produces.

Conventions shared by every producer here:

* Grids are NumPy arrays in C order with the x axis fastest: shape
  ``(NY, NX)`` in 2D and ``(NZ, NY, NX)`` in 3D.  Physical axis 1 is x,
  axis 2 is y, axis 3 is z.
* Voxel ``beta`` is the cell ``h*(beta + [0,1)^d)`` of the unit cell; it is
  given the phase of its centre ``(beta + 1/2) h`` (the binary rule the paper
  uses for its reference microstructure in Section 5).  Distances are
  periodic (minimum image).
* Scalar conduction has ``c = d`` components per voxel.  Elasticity has
  ``c = 6`` components in Mandel notation
  ``(e11, e22, e33, sqrt2 e23, sqrt2 e13, sqrt2 e12)``, in which the Euclidean
  dot product of two vectors equals the double contraction of the tensors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------------------
# moduli (inputs)
# --------------------------------------------------------------------------
def scalar_isotropic(a: float, d: int) -> np.ndarray:
    """Isotropic conductivity ``a * Id`` as a d x d matrix."""
    return float(a) * np.eye(d)


def lame_from_young(E: float, nu: float) -> tuple[float, float]:
    """Lame constants (lambda, mu) of an isotropic solid from (E, nu)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elastic_isotropic_mandel(lam: float, mu: float) -> np.ndarray:
    """6x6 Mandel matrix of the isotropic stiffness ``lam I(x)I + 2 mu Id``."""
    C = 2.0 * mu * np.eye(6)
    C[:3, :3] += lam
    return C


def elastic_from_young(E: float, nu: float) -> np.ndarray:
    return elastic_isotropic_mandel(*lame_from_young(E, nu))


def unit_loads(c: int) -> np.ndarray:
    """The c unit macroscopic loads (rows).  In Mandel notation row 5 is a
    pure shear with e12 = e21 = 1/sqrt2; ``sqrt2 * row5`` is the paper's
    p_shear of Section 5."""
    return np.eye(c)


# --------------------------------------------------------------------------
# geometry helpers
# --------------------------------------------------------------------------
def _centres(shape):
    """Voxel-centre coordinates (in voxel units) along each array axis."""
    return [np.arange(n, dtype=np.float64) + 0.5 for n in shape]


def _periodic_delta(a, b, n):
    d = np.abs(a - b) % n
    return np.minimum(d, n - d)


def disk_2d(n: int, fraction: float = 0.3, centre=(0.5, 0.5)) -> np.ndarray:
    """Centred disk of area ``fraction`` in a periodic n x n grid (phase 1 inside).

    Radius ``sqrt(fraction/pi)`` in unit-cell units; voxel-centre rule."""
    r = math.sqrt(fraction / math.pi) * n
    cy, cx = centre[1] * n, centre[0] * n
    yc, xc = _centres((n, n))
    dy = _periodic_delta(yc[:, None], cy, n)
    dx = _periodic_delta(xc[None, :], cx, n)
    return (dx * dx + dy * dy <= r * r).astype(np.uint8)


def _paint_sphere(phase, centre_zyx, radius, value=1):
    """Set voxels whose centre lies within ``radius`` (voxel units, periodic)."""
    shape = phase.shape
    idx = []
    for ax in range(3):
        c = centre_zyx[ax]
        lo = int(math.floor(c - radius - 0.5))
        hi = int(math.ceil(c + radius + 0.5))
        i = np.arange(lo, hi + 1)
        idx.append(i)
    iz, iy, ix = idx
    dz = (iz + 0.5 - centre_zyx[0])[:, None, None]
    dy = (iy + 0.5 - centre_zyx[1])[None, :, None]
    dx = (ix + 0.5 - centre_zyx[2])[None, None, :]
    inside = dz * dz + dy * dy + dx * dx <= radius * radius
    zz = np.broadcast_to((iz % shape[0])[:, None, None], inside.shape)[inside]
    yy = np.broadcast_to((iy % shape[1])[None, :, None], inside.shape)[inside]
    xx = np.broadcast_to((ix % shape[2])[None, None, :], inside.shape)[inside]
    newly = int(np.count_nonzero(phase[zz, yy, xx] != value))
    phase[zz, yy, xx] = value
    return newly


def boolean_spheres(n, radius: float, fraction: float, seed: int = 0):
    """Boolean model: overlapping spheres of ``radius`` voxels with continuous
    uniform centres in the periodic box (an ``n``^3 cube, or ``n`` = (nz, ny,
    nx)).  The sphere count is fixed so that the expected volume fraction is
    ``fraction``: ``round(-ln(1-f) * V / (4/3 pi r^3))``.

    Returns ``(phase, centres)``."""
    shape = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    rng = np.random.default_rng(seed)
    vol = 4.0 / 3.0 * math.pi * radius ** 3
    count = int(round(-math.log(1.0 - fraction) * float(np.prod(shape)) / vol))
    centres = rng.uniform(0.0, 1.0, size=(count, 3)) * np.array(shape, dtype=np.float64)  # (z, y, x)
    phase = np.zeros(shape, dtype=np.uint8)
    for c in centres:
        _paint_sphere(phase, c, radius)
    return phase, centres


def rsa_spheres(n: int, radius: float, min_distance: float, fraction: float,
                seed: int = 0, max_attempts: int = 2_000_000):
    """Periodic random sequential addition of non-overlapping spheres.

    Candidate centres are continuous uniform in [0, n)^3; a candidate is kept
    when its periodic distance to every kept centre is at least
    ``min_distance``.  Addition stops once the voxel volume fraction reaches
    ``fraction``.  Returns ``(phase, centres)``."""
    rng = np.random.default_rng(seed)
    phase = np.zeros((n, n, n), dtype=np.uint8)
    kept = np.empty((0, 3))
    target = fraction * n ** 3
    filled = 0
    attempts = 0
    md2 = min_distance * min_distance
    while filled < target:
        batch = rng.uniform(0.0, n, size=(256, 3))
        for cand in batch:
            attempts += 1
            if attempts > max_attempts:
                raise RuntimeError("RSA did not reach the requested fraction")
            if kept.shape[0]:
                dd = np.abs(kept - cand) % n
                dd = np.minimum(dd, n - dd)
                if np.min(np.einsum("ij,ij->i", dd, dd)) < md2:
                    continue
            kept = np.vstack([kept, cand])
            filled += _paint_sphere(phase, cand, radius)
            if filled >= target:
                break
    return phase, kept


def laminate(shape, axis: int, layers) -> np.ndarray:
    """Layered microstructure: ``layers`` is a list of (phase, thickness in
    voxels) repeated along physical ``axis`` (0 = x, 1 = y, 2 = z)."""
    d = len(shape)
    arr_axis = d - 1 - axis
    n = shape[arr_axis]
    prof = np.concatenate([np.full(t, p, dtype=np.uint8) for p, t in layers])
    if prof.size != n:
        raise ValueError("layer thicknesses must sum to the grid size")
    view = [1] * d
    view[arr_axis] = n
    return np.broadcast_to(prof.reshape(view), shape).copy()


def checkerboard_2d(n: int) -> np.ndarray:
    """2D checkerboard of four n/2 x n/2 squares (phases 0/1)."""
    h = n // 2
    y = (np.arange(n) >= h).astype(np.uint8)
    return (y[:, None] ^ y[None, :]).astype(np.uint8)


def random_phases(shape, nphase: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, nphase, size=shape, dtype=np.uint8)


def random_field(shape, c: int, nload: int = 1, seed: int = 0) -> np.ndarray:
    """Standard normal test fields of shape ``(nload, c, *shape)``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nload, c) + tuple(shape))


def gaussian_random_field(shape, corr_length: float, seed: int = 0) -> np.ndarray:
    """Periodic Gaussian random field: white N(0,1) noise smoothed by a
    periodic Gaussian kernel of standard deviation ``corr_length`` voxels,
    then re-standardised to mean 0 and variance 1."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    freqs = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    k2 = sum(f * f for f in freqs)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * np.exp(-2.0 * math.pi ** 2 * corr_length ** 2 * k2)))
    g -= g.mean()
    g /= g.std()
    return g


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    """A complete corrector-problem input: grid, phases, moduli, reference
    medium, Green variant and loads."""
    name: str
    physics: str            # "scalar" | "elastic"
    phase: np.ndarray       # uint8 grid (NY,NX) or (NZ,NY,NX)
    moduli: np.ndarray      # (nphase, c, c)
    A0: np.ndarray          # (c, c)
    green: str              # "truncated" | "filtered"
    loads: np.ndarray       # (nload, c)
    tol: float
    info: dict = field(default_factory=dict)

    @property
    def dim(self):
        return self.phase.ndim

    @property
    def c(self):
        return self.moduli.shape[1]


def disk_workload(n: int = 64, green: str = "truncated") -> Workload:
    """2D conduction: centred disk, f = 0.3, a = 10 in the disk, 1 outside,
    a0 = (amin + amax)/2, both unit gradients, tol 1e-10."""
    ph = disk_2d(n, 0.3)
    moduli = np.stack([scalar_isotropic(1.0, 2), scalar_isotropic(10.0, 2)])
    return Workload("disk2d", "scalar", ph, moduli, scalar_isotropic(5.5, 2), green,
                    unit_loads(2), 1e-10, {"fraction": float(ph.mean())})


def boolean_workload(n: int = 128, seed: int = 0, green: str = "filtered") -> Workload:
    """3D conduction: Boolean spheres of radius 6 voxels (scaled with n/128),
    expected fraction 0.25, contrast 100:1, a0 = half the softest phase."""
    r = 6.0 * n / 128.0
    ph, centres = boolean_spheres(n, r, 0.25, seed)
    moduli = np.stack([scalar_isotropic(1.0, 3), scalar_isotropic(100.0, 3)])
    return Workload("boolean3d", "scalar", ph, moduli, scalar_isotropic(0.5, 3), green,
                    unit_loads(3), 1e-10,
                    {"fraction": float(ph.mean()), "spheres": int(len(centres)), "seed": seed})


def elastic_rsa_workload(n: int = 256, seed: int = 0, green: str = "filtered",
                         tol: float = 1e-6) -> Workload:
    """3D isotropic elasticity: RSA spheres of radius 8 voxels (scaled with
    n/256), minimum centre distance one diameter, voxel fraction >= 0.30.
    Matrix E=1 nu=0.3, inclusions E=10 nu=0.2; reference mu0 = mu_m/2,
    nu0 = 0.3; the six Mandel unit strains."""
    r = 8.0 * n / 256.0
    ph, centres = rsa_spheres(n, r, 2.0 * r, 0.30, seed)
    Cm = elastic_from_young(1.0, 0.3)
    Ci = elastic_from_young(10.0, 0.2)
    mu_m = lame_from_young(1.0, 0.3)[1]
    mu0 = 0.5 * mu_m
    nu0 = 0.3
    lam0 = 2.0 * mu0 * nu0 / (1.0 - 2.0 * nu0)
    return Workload("elastic_rsa3d", "elastic", ph, np.stack([Cm, Ci]),
                    elastic_isotropic_mandel(lam0, mu0), green, unit_loads(6), tol,
                    {"fraction": float(ph.mean()), "spheres": int(len(centres)), "seed": seed})


@dataclass
class GradientWorkload:
    """Per-voxel elasticity for sensitivity studies: a smoothed Gaussian field
    theta sets Young's modulus E = 1 + 9 sigmoid(theta) at fixed Poisson's
    ratio; the reference medium (E0, nu0), the loads and the weights W of the
    scalar J = sum_lm W_lm p_l . C* p_m are part of the workload."""
    theta: np.ndarray       # (NZ, NY, NX)
    nu: float
    A0: np.ndarray          # (6, 6) Mandel
    green: str
    loads: np.ndarray       # (nload, 6)
    W: np.ndarray           # (nload, nload)
    tol: float


def gradient_workload(n: int = 192, corr_length: float = 2.0, seed: int = 0) -> GradientWorkload:
    """192^3 by default; theta with correlation length 2 voxels, nu = 0.3,
    reference E0 = 0.5, nu0 = 0.3, filtered operator, loads e_1 and the Mandel
    shear unit e_6 with W = diag(1, 1/2), so that J = C*_1111 + C*_1212, FP64
    tolerance 1e-10."""
    theta = gaussian_random_field((n, n, n), corr_length, seed)
    lam0, mu0 = lame_from_young(0.5, 0.3)
    loads = unit_loads(6)[[0, 5]]
    return GradientWorkload(theta, 0.3, elastic_isotropic_mandel(lam0, mu0), "filtered", loads,
                            np.diag([1.0, 0.5]), 1e-10)


@dataclass
class EnsembleMember:
    """One realisation of a stochastic-homogenisation ensemble: a cube of n^3
    voxels with per-voxel scalar conductivity a and its reference a0."""
    n: int
    a: np.ndarray           # (n, n, n)
    a0: float


def ensemble_workload(members: int = 48, sizes=(64, 96, 128, 160), corr_length: float = 4.0,
                      sigma_log: float = 1.0, seed: int = 0):
    """Members with sizes drawn uniformly from ``sizes``; a = exp(sigma_log g)
    with g a periodic Gaussian field of correlation length ``corr_length``
    voxels (one seed per member); reference a0 = min(a)/2, so that A - A0 is
    positive definite everywhere.  The loads are the three unit gradients."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(members):
        n = int(rng.choice(np.asarray(sizes)))
        g = gaussian_random_field((n, n, n), corr_length, seed=seed * 100003 + i + 1)
        a = np.exp(sigma_log * g)
        out.append(EnsembleMember(n, a, 0.5 * float(a.min())))
    return out
