"""Helpers shared by the GPU parity tests: build a library context and the
matching oracle problem from the same seeded inputs."""
import numpy as np

from oracle import operator as op


def context(lsh, phase, moduli, A0, physics, green, precision="fp64", max_loads=1):
    ctx = lsh.Context(phase.shape, physics, precision, max_loads=max_loads)
    ctx.set_reference(A0)
    ctx.set_phases(phase, moduli)
    ctx.set_green(green)
    return ctx


def problem(phase, moduli, A0, physics, green):
    return op.Problem(phase, np.asarray(moduli), np.asarray(A0), physics, green)


def rel_max_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def to_dev(a, dtype="f64"):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0")
