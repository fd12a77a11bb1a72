"""Writes the stored expected values of the GPU parity tests.

Every number here comes from the CPU oracle (``oracle/``) on the seeded
inputs of ``paper_1411_0330_amd.inputs``; nothing is read from the HIP path.

    python tests/golden/make_golden.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import effective, solvers  # noqa: E402
from oracle import operator as op  # noqa: E402
from paper_1411_0330_amd import inputs as I  # noqa: E402


def _solve_all(w, tol, maxit=20000):
    pb = op.Problem(w.phase, w.moduli, w.A0, w.physics, w.green)
    taus, iters, res = [], [], []
    for p in w.loads:
        r = solvers.cg(pb, p, tol=tol, maxit=maxit)
        taus.append(r["tau"])
        iters.append(r["iters"])
        res.append(r["rel_res"])
    return effective.effective_matrix(w.A0, w.loads, taus), iters, res, pb


def disk2d():
    w = I.disk_workload(64, "truncated")
    A, iters, res, pb = _solve_all(w, 1e-12)
    it10 = solvers.cg(pb, w.loads[0], tol=1e-10)["iters"]
    return {"workload": "2D disk f=0.3, 64x64, a=10/1, a0=5.5, truncated",
            "A_star": A.tolist(), "cg_iterations_tol1e-12": iters, "cg_iterations_tol1e-10": it10,
            "true_rel_residual": res, "voxel_fraction": w.info["fraction"], "oracle_tol": 1e-12}


def boolean128():
    w = I.boolean_workload(128)
    A, iters, res, _ = _solve_all(w, 1e-12)
    return {"workload": "3D Boolean spheres r=6, 128^3, a=100/1, a0=0.5, filtered, seed 0",
            "A_star": A.tolist(), "cg_iterations": iters, "true_rel_residual": res,
            "voxel_fraction": w.info["fraction"], "spheres": w.info["spheres"], "oracle_tol": 1e-12}


def elastic64():
    w = I.elastic_rsa_workload(64, tol=1e-10)
    A, iters, res, _ = _solve_all(w, 1e-11)
    return {"workload": "3D elastic RSA spheres r=2, 64^3, E=10/1, nu=0.2/0.3, mu0=mu_m/2, filtered, seed 0",
            "A_star": A.tolist(), "cg_iterations": iters, "true_rel_residual": res,
            "voxel_fraction": w.info["fraction"], "spheres": w.info["spheres"], "oracle_tol": 1e-11}


JOBS = {"disk2d_n64_truncated": disk2d, "boolean3d_n128_filtered": boolean128,
        "elastic_rsa_n64_filtered": elastic64}


def main(names):
    for name in names or JOBS:
        t = time.time()
        out = JOBS[name]()
        out["generator"] = "tests/golden/make_golden.py (oracle only)"
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {time.time() - t:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
