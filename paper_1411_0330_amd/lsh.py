"""ctypes binding of the C ABI in include/lsh.h (argument marshalling only).

Every step of the solver runs in the HIP library ``_lib/liblsh.so``; this
module loads it (and fails loudly when it is missing), converts arguments and
lets PyTorch own the device memory (the workspace and field buffers) and the
stream.  Array conventions follow the C ABI: fields are
``[load][component][z][y][x]`` with x fastest; grid shapes are given in array
order ``(NY, NX)`` or ``(NZ, NY, NX)``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LSH_LIB_PATH selects another build of the same library (the host-sanitizer
# build of build.build_host_sanitized)
LIB_PATH = os.environ.get("LSH_LIB_PATH") or os.path.join(HERE, "_lib", "liblsh.so")

OK, MAXIT, EINVAL, ENOMEM, EHIP, EHYP2, EBREAKDOWN, ENUMERIC, ESTATE = 0, 1, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "OK", 1: "MAXIT", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EHYP2",
                -5: "EBREAKDOWN", -6: "ENUMERIC", -7: "ESTATE"}
SCALAR, ELASTIC = 0, 1
FP64, MIXED = 0, 1
TRUNCATED, FILTERED, CONSISTENT, FD = 0, 1, 2, 3
BASIC, CG, MINRES, EYRE_MILTON, SYMMLQ = 0, 1, 2, 3, 4
HOST, DEVICE = 0, 1
F64, F32 = 0, 1
TAU, STRAIN = 0, 1

GREEN = {"truncated": TRUNCATED, "filtered": FILTERED, "consistent": CONSISTENT, "fd": FD}
SOLVERS = {"basic": BASIC, "cg": CG, "minres": MINRES, "eyre_milton": EYRE_MILTON, "symmlq": SYMMLQ}
PHYSICS = {"scalar": SCALAR, "elastic": ELASTIC}
PRECISION = {"fp64": FP64, "mixed": MIXED}


class LoadReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("status", C.c_int32), ("rel_residual", C.c_double)]


class SolveReport(C.Structure):
    _fields_ = [("applications_fp64", C.c_int64), ("applications_fp32", C.c_int64),
                ("outer_iterations", C.c_int32), ("pad", C.c_int32), ("seconds", C.c_double)]


_lib = None

_SIGS = {
    "lsh_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int64), C.c_int, C.c_int, C.c_int,
                             C.c_void_p]),
    "lsh_destroy": (C.c_int, [C.c_void_p]),
    "lsh_workspace_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lsh_bind_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lsh_set_reference": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lsh_set_phases": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double)]),
    "lsh_set_voxel_moduli": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "lsh_gradient": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.c_int]),
    "lsh_set_green": (C.c_int, [C.c_void_p, C.c_int]),
    "lsh_green_table_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lsh_bind_green_table": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lsh_set_green_series": (C.c_int, [C.c_void_p, C.c_int]),
    "lsh_solver_buffer_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "lsh_bind_solver_buffer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lsh_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double), C.c_double, C.c_int,
                            C.POINTER(LoadReport), C.POINTER(SolveReport)]),
    "lsh_get_field": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int]),
    "lsh_set_initial_guess": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int]),
    "lsh_get_effective": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "lsh_get_residual_history": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_double),
                                           C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "lsh_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "lsh_apply_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "lsh_forward_dft": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "lsh_spectrum_bytes": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_size_t)]),
    "lsh_set_variant": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "lsh_get_variants": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "lsh_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_int)]),
    "lsh_solve_many": (C.c_int, [C.c_int, C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int32),
                                 C.POINTER(C.POINTER(C.c_double)), C.c_double, C.c_int,
                                 C.POINTER(C.POINTER(LoadReport)), C.POINTER(SolveReport), C.POINTER(C.c_int32),
                                 C.c_int]),
    "lsh_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "lsh_set_graphs": (C.c_int, [C.c_void_p, C.c_int]),
    "lsh_set_persistent": (C.c_int, [C.c_void_p, C.c_int]),
    "lsh_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]),
    "lsh_last_error": (C.c_char_p, [C.c_void_p]),
    "lsh_version": (C.c_char_p, []),
}


def _hip_runtimes():
    """Distinct HIP runtime files mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def load():
    """Load the HIP library (raises when it has not been built).

    PyTorch is imported first so that the library binds to the HIP runtime
    PyTorch already uses (same soname): device pointers and streams from
    PyTorch are then valid in the library.  Two runtimes in one process are
    refused."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the process's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (build it with __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes loaded in one process: {rts}")
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LshError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _dptr(a, n=None):
    return C.cast(a.ctypes.data, C.POINTER(C.c_double))


class Context:
    """One solver context on one stream (thin wrapper over lsh_ctx)."""

    def __init__(self, shape, physics="scalar", precision="fp64", max_loads=1, device="cuda:0",
                 stream=None, bind=True):
        self.lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.physics = physics
        self.precision = precision
        self.max_loads = int(max_loads)
        self.c = 6 if physics == "elastic" else self.dim
        n = (C.c_int64 * 3)(*reversed(self.shape), *([1] * (3 - self.dim)))
        self._stream = stream
        sptr = None
        if stream is not None:
            sptr = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        h = C.c_void_p()
        self._check(self.lib.lsh_create(C.byref(h), self.dim, n, PHYSICS[physics], PRECISION[precision],
                                        self.max_loads, sptr), ctx=None)
        self.h = h
        self.device = device
        self.workspace = None
        if bind:
            self.bind()

    # -- plumbing ------------------------------------------------------
    def _check(self, status, ctx="self", allow=(OK,)):
        if status in allow:
            return status
        msg = ""
        if ctx == "self":
            msg = (self.lib.lsh_last_error(self.h) or b"").decode()
        raise LshError(status, msg)

    def workspace_bytes(self):
        b = C.c_size_t()
        self._check(self.lib.lsh_workspace_bytes(self.h, C.byref(b)))
        return int(b.value)

    def bind(self):
        import torch
        nbytes = self.workspace_bytes()
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.workspace.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        self._check(self.lib.lsh_bind_workspace(self.h, C.c_void_p(ptr), nbytes))

    def close(self):
        if getattr(self, "h", None):
            self.lib.lsh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- problem -------------------------------------------------------
    def set_reference(self, A0):
        A0 = np.ascontiguousarray(A0, dtype=np.float64)
        return self._check(self.lib.lsh_set_reference(self.h, _dptr(A0)))

    def set_phases(self, phase, moduli):
        moduli = np.ascontiguousarray(moduli, dtype=np.float64)
        nphase = moduli.shape[0]
        if hasattr(phase, "data_ptr"):
            assert phase.dtype.__str__() == "torch.uint8" and phase.is_contiguous()
            self._phase_ref = phase
            return self._check(self.lib.lsh_set_phases(self.h, C.c_void_p(phase.data_ptr()), DEVICE, nphase,
                                                       _dptr(moduli)))
        ph = np.ascontiguousarray(phase, dtype=np.uint8)
        return self._check(self.lib.lsh_set_phases(self.h, C.c_void_p(ph.ctypes.data), HOST, nphase,
                                                   _dptr(moduli)))

    def set_voxel_moduli(self, coef):
        """Per-voxel isotropic coefficients (ncoef, *shape): a (scalar) or
        (K, mu) (elasticity); a torch tensor on the device or a host array,
        float64 or float32."""
        ncoef = 2 if self.physics == "elastic" else 1
        if hasattr(coef, "data_ptr"):
            import torch
            assert coef.dtype in (torch.float64, torch.float32)
            coef = coef.contiguous()
            code = F64 if coef.dtype == torch.float64 else F32
            mem = DEVICE if coef.is_cuda else HOST
            ptr = coef.data_ptr()
            keep = coef
        else:
            keep = np.ascontiguousarray(coef)
            if keep.dtype not in (np.float64, np.float32):
                keep = keep.astype(np.float64)
            code = F64 if keep.dtype == np.float64 else F32
            mem, ptr = HOST, keep.ctypes.data
        if tuple(keep.shape) != (ncoef,) + self.shape:
            raise ValueError(f"expected coefficients of shape {(ncoef,) + self.shape}, got {tuple(keep.shape)}")
        st = self._check(self.lib.lsh_set_voxel_moduli(self.h, C.c_void_p(ptr), code, mem, ncoef))
        self.solves = getattr(self, "solves", 0) + 1
        return st

    def gradient(self, W, dtype="f64"):
        """dJ/d(coefficients) for J = sum_lm W_lm p_l . A* p_m over the loads of
        the last solve: a device tensor (ncoef, *shape)."""
        import torch
        W = np.ascontiguousarray(np.atleast_2d(W), dtype=np.float64)
        if W.shape != (self.nload, self.nload):
            raise ValueError(f"W must be {self.nload} x {self.nload}")
        ncoef = 2 if self.physics == "elastic" else 1
        out = torch.empty((ncoef,) + self.shape, dtype=torch.float64 if dtype == "f64" else torch.float32,
                          device=self.device)
        self._check(self.lib.lsh_gradient(self.h, _dptr(W), C.c_void_p(out.data_ptr()), F64 if dtype == "f64" else F32))
        return out

    def set_green(self, variant, series=None):
        """Select the Green operator; the consistent one gets a table buffer
        (owned by this object) and optionally its series cut nmax."""
        code = GREEN[variant] if isinstance(variant, str) else variant
        if code == CONSISTENT and getattr(self, "green_table", None) is None:
            import torch
            b = C.c_size_t()
            self._check(self.lib.lsh_green_table_bytes(self.h, C.byref(b)))
            self.green_table = torch.empty(b.value + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.green_table.data_ptr() + 255) // 256 * 256
            self._check(self.lib.lsh_bind_green_table(self.h, C.c_void_p(ptr), b.value))
        if series is not None:
            self._check(self.lib.lsh_set_green_series(self.h, int(series)))
        return self._check(self.lib.lsh_set_green(self.h, code))

    # -- solve ---------------------------------------------------------
    def _solver_buffer(self, code):
        b = C.c_size_t()
        self._check(self.lib.lsh_solver_buffer_bytes(self.h, code, C.byref(b)))
        if b.value and getattr(self, "solver_buffer", None) is None:
            import torch
            self.solver_buffer = torch.empty(b.value + 256, dtype=torch.uint8, device=self.device)
            ptr = (self.solver_buffer.data_ptr() + 255) // 256 * 256
            self._check(self.lib.lsh_bind_solver_buffer(self.h, C.c_void_p(ptr), b.value))

    def solve(self, loads, solver="cg", tol=1e-10, maxit=1000, allow=(OK, MAXIT)):
        loads = np.ascontiguousarray(np.atleast_2d(loads), dtype=np.float64)
        self._solver_buffer(SOLVERS[solver])
        nload = loads.shape[0]
        reps = (LoadReport * nload)()
        summ = SolveReport()
        st = self.lib.lsh_solve(self.h, SOLVERS[solver], nload, _dptr(loads), float(tol), int(maxit), reps,
                                C.byref(summ))
        self._check(st, allow=allow)
        self.nload = nload
        self.solves = getattr(self, "solves", 0) + 1
        return {
            "status": st,
            "iterations": [r.iterations for r in reps],
            "load_status": [r.status for r in reps],
            "rel_residual": [r.rel_residual for r in reps],
            "applications_fp64": summ.applications_fp64,
            "applications_fp32": summ.applications_fp32,
            "outer_iterations": summ.outer_iterations,
            "seconds": summ.seconds,
        }

    def set_initial_guess(self, load, tau):
        """Warm start of the next solve for load slot `load`
        (lsh_set_initial_guess): tau of shape (c, *shape), a torch tensor on
        the device or a host array, float64 or float32; None clears it."""
        if tau is None:
            return self._check(self.lib.lsh_set_initial_guess(self.h, int(load), None, F64, HOST))
        if hasattr(tau, "data_ptr"):
            import torch
            assert tau.dtype in (torch.float64, torch.float32)
            keep = tau.contiguous()
            code = F64 if keep.dtype == torch.float64 else F32
            mem = DEVICE if keep.is_cuda else HOST
            ptr = keep.data_ptr()
        else:
            keep = np.ascontiguousarray(tau)
            assert keep.dtype in (np.float64, np.float32)
            code = F64 if keep.dtype == np.float64 else F32
            mem = HOST
            ptr = keep.ctypes.data
        if tuple(keep.shape) != (self.c,) + self.shape:
            raise ValueError(f"expected a guess of shape {(self.c,) + self.shape}, got {tuple(keep.shape)}")
        return self._check(self.lib.lsh_set_initial_guess(self.h, int(load), C.c_void_p(ptr), code, mem))

    def effective(self):
        """(nload, c) array: row l is A0 p_l + <tau_l>."""
        out = np.zeros((self.nload, self.c))
        self._check(self.lib.lsh_get_effective(self.h, _dptr(out)))
        return out

    def residual_history(self, load=0, cap=4096):
        """Relative residual after every iteration of the last solve of `load`
        (the last `cap` entries, at most 4096): dict with "rel" (float64),
        "level" (int32: 0 FP64, 1 FP32 inner CG of a mixed solve) and "total"."""
        rel = np.zeros(cap)
        lev = np.zeros(cap, dtype=np.int32)
        tot = C.c_int64(0)
        self._check(self.lib.lsh_get_residual_history(self.h, int(load), int(cap), _dptr(rel),
                                                      lev.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(tot)))
        n = min(cap, tot.value, 4096)
        return {"rel": rel[:n].copy(), "level": lev[:n].copy(), "total": int(tot.value)}

    def field(self, load=0, which="tau", dtype="f64", device=True):
        import torch
        tdt = torch.float64 if dtype == "f64" else torch.float32
        code = F64 if dtype == "f64" else F32
        w = TAU if which == "tau" else STRAIN
        if device:
            out = torch.empty((self.c,) + self.shape, dtype=tdt, device=self.device)
            self._check(self.lib.lsh_get_field(self.h, load, w, C.c_void_p(out.data_ptr()), code, DEVICE))
            return out
        out = np.empty((self.c,) + self.shape, dtype=np.float64 if dtype == "f64" else np.float32)
        self._check(self.lib.lsh_get_field(self.h, load, w, C.c_void_p(out.ctypes.data), code, HOST))
        return out

    # -- operator and transform ----------------------------------------
    def apply(self, tau):
        """L tau for a device tensor (nload, c, *shape), float64 or float32."""
        import torch
        code = F64 if tau.dtype == torch.float64 else F32
        tau = tau.contiguous()
        out = torch.empty_like(tau)
        self._check(self.lib.lsh_apply(self.h, tau.shape[0], C.c_void_p(tau.data_ptr()),
                                       C.c_void_p(out.data_ptr()), code))
        return out

    def forward_dft(self, field):
        """Packed half spectrum of a device tensor (nload, c, *shape):
        returns (main [nload, c, nz?, ny, nx/2], nyquist [nload, c, nz?, ny]) complex tensors."""
        import torch
        code = F64 if field.dtype == torch.float64 else F32
        field = field.contiguous()
        nload = field.shape[0]
        b = C.c_size_t()
        self._check(self.lib.lsh_spectrum_bytes(self.h, code, C.byref(b)))
        rdt = torch.float64 if code == F64 else torch.float32
        spec = torch.empty(nload * b.value // (8 if code == F64 else 4), dtype=rdt, device=self.device)
        self._check(self.lib.lsh_forward_dft(self.h, nload, C.c_void_p(field.data_ptr()),
                                             C.c_void_p(spec.data_ptr()), code))
        mx = self.shape[-1] // 2
        lead = self.shape[:-1]
        nmain = nload * self.c * int(np.prod(lead)) * mx
        cs = torch.view_as_complex(spec.view(-1, 2))
        main = cs[:nmain].reshape((nload, self.c) + lead + (mx,))
        nyq = cs[nmain:].reshape((nload, self.c) + lead)
        return main, nyq

    # -- graphs and timing ---------------------------------------------
    def set_variant(self, pass_, fp64, variant):
        return self._check(self.lib.lsh_set_variant(self.h, int(pass_), int(bool(fp64)), int(variant)))

    def variants(self):
        """Current kernel shapes: {"fp32": [xfwd, y, zg, xinv], "fp64": [...]}."""
        v = (C.c_int32 * 8)()
        self._check(self.lib.lsh_get_variants(self.h, v))
        return {"fp32": list(v[:4]), "fp64": list(v[4:])}

    def autotune(self, nload=None, cache=None):
        """Pick the fastest kernel shape per pass (lsh_autotune); returns
        (variants, from_cache)."""
        v = (C.c_int32 * 8)()
        hit = C.c_int(0)
        path = None if cache is None else os.fspath(cache).encode()
        self._check(self.lib.lsh_autotune(self.h, int(nload or self.max_loads), path, v, C.byref(hit)))
        return {"fp32": list(v[:4]), "fp64": list(v[4:])}, bool(hit.value)

    def set_persistent(self, enable=True):
        return self._check(self.lib.lsh_set_persistent(self.h, int(bool(enable))))

    def set_graphs(self, enable=True):
        self._check(self.lib.lsh_set_graphs(self.h, 1 if enable else 0))

    def set_timing(self, enable=True):
        self._check(self.lib.lsh_set_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        """{class: (total ms, launches, algorithmic bytes)} since timing was enabled."""
        cap = 32
        names = (C.c_char_p * cap)()
        ms = (C.c_double * cap)()
        cnt = (C.c_int64 * cap)()
        by = (C.c_double * cap)()
        n = C.c_int()
        self._check(self.lib.lsh_kernel_times(self.h, names, ms, cnt, by, cap, C.byref(n)))
        return {names[i].decode(): (ms[i], int(cnt[i]), by[i]) for i in range(min(n.value, cap))}


def solve_many(ctxs, loads, solver="cg", tol=1e-10, maxit=1000, threads=4, allow=(OK, MAXIT)):
    """Solve several contexts concurrently (lsh_solve_many): ``loads[i]`` is
    the (nload_i, c) array of context i.  Returns one report dict per context,
    as Context.solve."""
    lib = load()
    n = len(ctxs)
    arrs = [np.ascontiguousarray(np.atleast_2d(l), dtype=np.float64) for l in loads]
    handles = (C.c_void_p * n)(*[c.h.value for c in ctxs])
    nl = (C.c_int32 * n)(*[a.shape[0] for a in arrs])
    lp = (C.POINTER(C.c_double) * n)(*[_dptr(a) for a in arrs])
    reps = [(LoadReport * a.shape[0])() for a in arrs]
    rp = (C.POINTER(LoadReport) * n)(*[C.cast(r, C.POINTER(LoadReport)) for r in reps])
    summ = (SolveReport * n)()
    sts = (C.c_int32 * n)()
    for c in ctxs:
        c._solver_buffer(SOLVERS[solver])
    st = lib.lsh_solve_many(n, handles, SOLVERS[solver], nl, lp, float(tol), int(maxit), rp, summ, sts, int(threads))
    out = []
    for i, c in enumerate(ctxs):
        c._check(sts[i], allow=allow)
        c.nload = arrs[i].shape[0]
        c.solves = getattr(c, "solves", 0) + 1
        out.append({"status": sts[i], "iterations": [r.iterations for r in reps[i]],
                    "load_status": [r.status for r in reps[i]],
                    "rel_residual": [r.rel_residual for r in reps[i]],
                    "applications_fp64": summ[i].applications_fp64, "applications_fp32": summ[i].applications_fp32,
                    "outer_iterations": summ[i].outer_iterations, "seconds": summ[i].seconds})
    if st not in allow and all(s in allow for s in sts):
        raise LshError(st, "ensemble solve failed")
    return out


def header_symbols(header_path=None):
    """Function names declared in include/lsh.h."""
    import re
    header_path = header_path or os.path.join(os.path.dirname(HERE), "include", "lsh.h")
    text = open(header_path).read()
    # declarations: a return type at the start of a line, then the name and "("
    return sorted(set(re.findall(r"^(?:const\s+)?\w+\s*\*?\s*(lsh_[a-z_]+)\s*\(", text, re.M)))
