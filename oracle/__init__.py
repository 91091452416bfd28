"""Python access to the oracle (``pcg_oracle.c``).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this package.  It shares no
code with the HIP path (``paper_1706_05988_amd``) and neither imports the
other; both consume the seeded inputs of the ``problems`` package.

The C library implements classic CG (Alg. 1), pipelined CG (Alg. 2) and
shifted pipelined CG (Alg. 3) in plain binary64 loops, step by step in the
paper's order.  ``build()`` compiles it with gcc (no FMA contraction, no
fast-math, OpenMP over elementwise loops and fixed-chunk dot products, which
gives the same bits at any thread count).

The a-posteriori shift analysis of Section 3.2 (the propagation matrices
P_i(sigma), their products and psi_i(sigma)) is in ``oracle.psi``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

METHODS = {"cg": 0, "pipe": 1, "pipe_shift": 2, "pipe_var": 3, "pipe_rr": 4}
STATUS = {0: "converged", 1: "max_iter", 2: "breakdown", 3: "nonfinite"}
KINDS = {"2d5": 0, "3d7": 1, "csr": 2}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (binary64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("n", C.c_int64),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("centre", C.c_double), ("off", C.c_double),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("max_iter", C.c_int32), ("sigma", C.c_double),
                ("rtol", C.c_double), ("jacobi", C.c_int32), ("fp32_storage", C.c_int32),
                ("record_true", C.c_int32), ("record_gaps", C.c_int32), ("threads", C.c_int32),
                ("replace_max", C.c_int32), ("ignore_breakdown", C.c_int32),
                ("sigma_sched", C.c_void_p), ("sigma_sched_len", C.c_int32),
                ("w0_perturb", C.c_void_p), ("rr_tau", C.c_double), ("rr_period", C.c_int32),
                ("rr_floor", C.c_double), ("snap_iter", C.c_int32)]


_HIST = ["h_res", "h_true", "h_alpha", "h_beta", "h_gamma", "h_delta", "h_f", "h_g", "h_h", "h_j"]
# the stored vectors of a solve, in the oracle's slot order (absent ones come back as None)
VECTORS = ["r", "u", "w", "z", "q", "s", "t", "p", "dinv"]


class _Res(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("replacements", C.c_int32),
                ("pad_", C.c_int32), ("bnorm", C.c_double), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double)] + [(h, C.c_void_p) for h in _HIST] + \
               [("snap", C.c_void_p), ("final_vecs", C.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        lib.orc_solve.argtypes = [C.POINTER(_Op), C.POINTER(_Opts), C.c_void_p, C.c_void_p, C.POINTER(_Res)]
        lib.orc_solve.restype = C.c_int
        lib.orc_apply_A.argtypes = [C.POINTER(_Op), C.c_void_p, C.c_void_p]
        lib.orc_apply_A.restype = C.c_int
        lib.orc_dot.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_int]
        lib.orc_dot.restype = C.c_double
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _make_op(op):
    keep = []
    o = _Op()
    o.kind = KINDS[op.kind]
    o.n = op.n
    o.nx, o.ny, o.nz = op.nx, op.ny, op.nz
    o.centre = float(op.diag) + float(op.shift)
    o.off = float(op.off)
    if op.kind == "csr":
        rp = np.ascontiguousarray(op.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(op.col, dtype=np.int32)
        val = np.ascontiguousarray(op.val, dtype=np.float64)
        keep += [rp, col, val]
        o.row_ptr, o.col, o.val = _ptr(rp), _ptr(col), _ptr(val)
    return o, keep


def apply_A(op, v: np.ndarray) -> np.ndarray:
    lib = _load()
    o, keep = _make_op(op)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(op.n)
    assert lib.orc_apply_A(C.byref(o), _ptr(v), _ptr(out)) == 0
    del keep
    return out


def dot(a: np.ndarray, b: np.ndarray, threads: int = 1) -> float:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return lib.orc_dot(a.size, _ptr(a), _ptr(b), threads)


def max_threads() -> int:
    return _load().orc_max_threads()


def solve(op, b: np.ndarray, x0: Optional[np.ndarray] = None, method: str = "pipe_shift",
          sigma: float = 0.0, rtol: float = 1e-10, max_iter: int = 1000, jacobi: bool = False,
          fp32_storage: bool = False, record: bool = True, record_true: bool = False,
          record_gaps: bool = False, threads: int = 1, replace_max: int = 0,
          ignore_breakdown: bool = False, sigma_schedule=None, w0_perturb=None,
          rr_tau: Optional[float] = None, rr_period: int = 8, rr_floor: float = 100.0,
          snap_iter: Optional[int] = None, return_vectors: bool = False) -> dict:
    """Run the oracle.  Returns a dict with x, status, iterations, norms and
    (if ``record``) histories indexed by iteration (NaN where not reached).
    ``return_vectors``: also the stored vectors when the solve returns
    (``final``: name -> array, None for a vector the method does not keep);
    ``snap_iter``: the stored vectors as the body of that iteration finds
    them, after any restart or replacement at its top (``snap``, None if the
    solve never ran that body)."""
    lib = _load()
    o, keep = _make_op(op)
    opts = _Opts(METHODS[method], int(max_iter), float(sigma), float(rtol), int(bool(jacobi)),
                 int(bool(fp32_storage)), int(bool(record_true)), int(bool(record_gaps)),
                 int(threads), int(replace_max), int(bool(ignore_breakdown)))
    sched = None
    if method == "pipe_var":
        if sigma_schedule is None or len(sigma_schedule) < 1:
            raise ValueError("pipe_var needs sigma_schedule = [sigma_-1, sigma_0, sigma_1, ...]")
        sched = np.ascontiguousarray(sigma_schedule, dtype=np.float64)
        opts.sigma_sched = _ptr(sched)
        opts.sigma_sched_len = len(sched)
    # p-CG-rr: tau defaults to the cube root of the storage unit roundoff
    opts.rr_tau = float(rr_tau) if rr_tau is not None else (2.0 ** -8 if fp32_storage else 2.0 ** (-53 / 3))
    opts.rr_period = int(rr_period)
    opts.rr_floor = float(rr_floor)
    pert = None
    if w0_perturb is not None:
        pert = np.ascontiguousarray(w0_perturb, dtype=np.float64)
        assert pert.shape == (op.n,)
        opts.w0_perturb = _ptr(pert)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(op.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    res = _Res()
    hist = {}
    L = int(max_iter) + 2
    for h in _HIST:
        if not record or (h == "h_true" and not record_true):
            continue
        if h in ("h_f", "h_g", "h_h", "h_j") and not record_gaps:
            continue
        hist[h] = np.full(L, np.nan)
        setattr(res, h, _ptr(hist[h]))
    nv = len(VECTORS)
    opts.snap_iter = -1 if snap_iter is None else int(snap_iter)
    snap = np.full(nv * op.n, np.inf) if snap_iter is not None else None
    fin = np.empty(nv * op.n) if return_vectors else None
    res.snap, res.final_vecs = _ptr(snap), _ptr(fin)
    rc = lib.orc_solve(C.byref(o), C.byref(opts), _ptr(b), _ptr(x), C.byref(res))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    del keep
    out = dict(x=x, status=STATUS[res.status], iterations=res.iterations,
               replacements=res.replacements, bnorm=res.bnorm,
               rel_res_recursive=res.rel_res_recursive, rel_res_true=res.rel_res_true)
    for h, arr in hist.items():
        out[h[2:]] = arr[: res.iterations + 1]

    def unpack(buf):
        vs = buf.reshape(nv, op.n)
        return {name: (None if np.isnan(v).all() else v.copy()) for name, v in zip(VECTORS, vs)}

    if fin is not None:
        out["final"] = unpack(fin)
    if snap is not None:
        out["snap"] = None if np.isinf(snap).all() else unpack(snap)
    return out


def solve_problem(p, method: str = "pipe_shift", **kw) -> dict:
    """Convenience: run the oracle on a ``problems.Problem``."""
    args = dict(sigma=p.sigma if method == "pipe_shift" else 0.0, rtol=p.rtol,
                max_iter=p.max_iter, jacobi=p.jacobi)
    args.update(kw)
    return solve(p.op, p.b, p.x0, method=method, **args)
