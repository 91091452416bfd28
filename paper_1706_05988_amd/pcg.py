"""ctypes binding of libpcg (``include/pcg.h``): argument marshalling only.

Every function named ``pcg_*`` here calls the C entry point of the same name;
all solver work runs in the library's HIP kernels.  PyTorch supplies device
memory (workspace, operator arrays) and the HIP stream.  Importing this
module does not need a GPU; loading the library fails loudly when it has not
been built (``python -m paper_1706_05988_amd.build``) -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pcg.h")

PCG_OK, PCG_PENDING = 0, 1
PCG_ERR_INVALID, PCG_ERR_NONFINITE, PCG_ERR_HIP, PCG_ERR_BUDGET, PCG_ERR_STATE = -1, -2, -3, -4, -5
PCG_CONVERGED, PCG_MAX_ITER, PCG_BREAKDOWN, PCG_NONFINITE = 0, 1, 2, 3
PCG_CG, PCG_PIPE, PCG_PIPE_SHIFT, PCG_PIPE_VAR_SHIFT, PCG_PIPE_RR = 0, 1, 2, 3, 4
PCG_OP_STENCIL2D5, PCG_OP_STENCIL3D7, PCG_OP_CSR = 0, 1, 2
PCG_PC_NONE, PCG_PC_JACOBI = 0, 1
PCG_FP64, PCG_FP32_STREAM = 0, 1
PCG_HISTORY_FIELDS = 5
PCG_VAR_SET, PCG_VAR_XCD_MAP, PCG_VAR_NT, PCG_VAR_EPT1, PCG_VAR_EPT4 = 0x01, 0x02, 0x04, 0x10, 0x20
PCG_VAR_CG_ZMARCH = 0x40
PCG_VAR_CSR_SELL = 0x80
PCG_VAR_CSR_SELL_SORTED = 0x100
PCG_FLAG_RUN_THROUGH_BREAKDOWN = 0x01

METHOD = {"cg": PCG_CG, "pipe": PCG_PIPE, "pipe_shift": PCG_PIPE_SHIFT, "pipe_var": PCG_PIPE_VAR_SHIFT, "pipe_rr": PCG_PIPE_RR}
OUTCOME = {PCG_CONVERGED: "converged", PCG_MAX_ITER: "max_iter", PCG_BREAKDOWN: "breakdown",
           PCG_NONFINITE: "nonfinite"}
OPKIND = {"2d5": PCG_OP_STENCIL2D5, "3d7": PCG_OP_STENCIL3D7, "csr": PCG_OP_CSR}


class pcg_operator(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("n", C.c_int64), ("diag", C.c_double), ("offdiag", C.c_double), ("shift", C.c_double),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p),
                ("nnz", C.c_int64)]


class pcg_options(C.Structure):
    _fields_ = [("method", C.c_int32), ("pc", C.c_int32), ("prec", C.c_int32), ("max_iter", C.c_int32),
                ("sigma", C.c_double), ("rtol", C.c_double), ("true_residual_check", C.c_int32),
                ("replace_max", C.c_int32), ("iters_per_launch", C.c_int32), ("history_cap", C.c_int32),
                ("history", C.c_void_p), ("block_size", C.c_int32), ("grid_blocks", C.c_int32),
                ("timing", C.c_int32), ("use_graph", C.c_int32), ("variant", C.c_int32),
                ("sigma_schedule_len", C.c_int32), ("rr_period", C.c_int32), ("flags", C.c_int32),
                ("sigma_schedule", C.c_void_p), ("rr_tau", C.c_double), ("rr_floor", C.c_double)]


class pcg_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("replacements", C.c_int32),
                ("launches", C.c_int32), ("rel_res_recursive", C.c_double), ("rel_res_true", C.c_double),
                ("seconds", C.c_double), ("iter_kernel_ms", C.c_double), ("iter_passes", C.c_int32),
                ("admitted_at", C.c_int32), ("sigma", C.c_double)]


class pcg_solver_shape(C.Structure):
    _fields_ = [("block", C.c_int32), ("ept", C.c_int32), ("grid", C.c_int32), ("ntiles", C.c_int32),
                ("iters_per_launch", C.c_int32), ("csr_form", C.c_int32), ("csr_col_bits", C.c_int32),
                ("csr_val_bits", C.c_int32), ("csr_entries", C.c_int64)]


class pcg_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int32), ("running", C.c_int32), ("max_running", C.c_int32),
                ("launches", C.c_int32), ("arena_bytes", C.c_size_t), ("arena_free", C.c_size_t),
                ("arena_largest_free", C.c_size_t)]


class PcgError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {pcg_status_str(status)} ({status}) {pcg_last_error()}")
        self.status = status


_lib = None

_SIGS = {
    "pcg_default_options": (C.c_int32, [C.POINTER(pcg_options)]),
    "pcg_workspace_size": (C.c_int32, [C.POINTER(pcg_operator), C.POINTER(pcg_options), C.POINTER(C.c_size_t)]),
    "pcg_create": (C.c_int32, [C.POINTER(C.c_void_p), C.POINTER(pcg_operator), C.POINTER(pcg_options),
                               C.c_void_p, C.c_size_t, C.c_void_p]),
    "pcg_solve": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(pcg_result)]),
    "pcg_true_residual": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "pcg_destroy": (C.c_int32, [C.c_void_p]),
    "pcg_solver_info": (C.c_int32, [C.c_void_p, C.POINTER(pcg_solver_shape)]),
    "pcg_solve_static": (C.c_int32, [C.POINTER(pcg_operator), C.POINTER(pcg_options), C.c_void_p, C.c_void_p,
                                     C.POINTER(pcg_result), C.c_void_p]),
    "pcg_batch_workspace_size": (C.c_int32, [C.c_int32, C.POINTER(pcg_operator), C.POINTER(pcg_options),
                                             C.POINTER(C.c_size_t)]),
    "pcg_batch_solve": (C.c_int32, [C.c_int32, C.POINTER(pcg_operator), C.POINTER(pcg_options),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(pcg_result),
                                    C.c_void_p, C.c_size_t, C.c_void_p]),
    "pcg_batch_tune": (C.c_int32, [C.c_int32, C.POINTER(pcg_operator), C.POINTER(pcg_options),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_double)]),
    "pcg_server_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p]),
    "pcg_submit": (C.c_int32, [C.c_void_p, C.POINTER(pcg_operator), C.POINTER(pcg_options), C.c_void_p,
                               C.c_void_p, C.POINTER(C.c_uint64)]),
    "pcg_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(pcg_result)]),
    "pcg_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(pcg_result)]),
    "pcg_server_destroy": (C.c_int32, [C.c_void_p]),
    "pcg_server_info": (C.c_int32, [C.c_void_p, C.POINTER(pcg_server_stats)]),
    "pcg_status_str": (C.c_char_p, [C.c_int32]),
    "pcg_tune_workspace_size": (C.c_int32, [C.POINTER(pcg_operator), C.POINTER(pcg_options), C.POINTER(C.c_size_t)]),
    "pcg_tune": (C.c_int32, [C.POINTER(pcg_operator), C.POINTER(pcg_options), C.c_void_p, C.c_size_t, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "pcg_psi": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "pcg_psi_variable": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                     C.POINTER(C.c_double)]),
    "pcg_select_shift": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                     C.c_void_p, C.POINTER(C.c_double)]),
    "pcg_last_error": (C.c_char_p, []),
    "pcg_stream_probe": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_void_p, C.c_size_t,
                                     C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
}


def lib() -> C.CDLL:
    """Load libpcg.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_1706_05988_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/pcg.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pcg_[a-z_0-9]+)\s*\(", txt)))


def _check(st: int, what: str):
    if st != PCG_OK:
        raise PcgError(st, what)


def pcg_status_str(st: int) -> str:
    return lib().pcg_status_str(st).decode()


def pcg_last_error() -> str:
    return lib().pcg_last_error().decode()


def pcg_default_options() -> pcg_options:
    o = pcg_options()
    _check(lib().pcg_default_options(C.byref(o)), "pcg_default_options")
    return o


def pcg_workspace_size(op: pcg_operator, opt: pcg_options) -> int:
    n = C.c_size_t()
    _check(lib().pcg_workspace_size(C.byref(op), C.byref(opt), C.byref(n)), "pcg_workspace_size")
    return n.value


def pcg_create(op: pcg_operator, opt: pcg_options, workspace: int, nbytes: int, stream: int) -> int:
    h = C.c_void_p()
    _check(lib().pcg_create(C.byref(h), C.byref(op), C.byref(opt), workspace, nbytes, stream), "pcg_create")
    return h.value


def pcg_solve(handle: int, b: int, x: int) -> pcg_result:
    r = pcg_result()
    _check(lib().pcg_solve(handle, b, x, C.byref(r)), "pcg_solve")
    return r


def pcg_true_residual(handle: int, b: int, x: int) -> float:
    v = C.c_double()
    _check(lib().pcg_true_residual(handle, b, x, C.byref(v)), "pcg_true_residual")
    return v.value


def pcg_destroy(handle: int) -> None:
    _check(lib().pcg_destroy(handle), "pcg_destroy")


CSR_FORMS = {0: "csr", 1: "sell", 2: "sell_sorted"}


def pcg_solver_info(handle: int) -> dict:
    sh = pcg_solver_shape()
    _check(lib().pcg_solver_info(handle, C.byref(sh)), "pcg_solver_info")
    d = {name: getattr(sh, name) for name, _ in pcg_solver_shape._fields_}
    d["csr_form_name"] = CSR_FORMS.get(d["csr_form"], "?")
    return d


PCG_STATIC_SCRATCH_BYTES = 64 << 20


def pcg_solve_static(op: pcg_operator, opt: pcg_options, b: int, x: int, stream: int) -> pcg_result:
    r = pcg_result()
    _check(lib().pcg_solve_static(C.byref(op), C.byref(opt), b, x, C.byref(r), stream), "pcg_solve_static")
    return r


def solve_static(op, options: pcg_options, b, x, device="cuda", stream: Optional[int] = None) -> dict:
    """One solve through pcg_solve_static (the library's static device
    scratch, no workspace): b, x device tensors (binary64)."""
    import numpy as np
    dev = _device_op(op, options.prec, device)
    hist = None
    if options.history_cap > 0:
        hist = np.full((options.history_cap, PCG_HISTORY_FIELDS), np.nan)
        options.history = hist.ctypes.data
    st = current_stream_handle() if stream is None else stream
    r = pcg_solve_static(dev.struct, options, b.data_ptr(), x.data_ptr(), st)
    return result_dict(r, hist)


def pcg_batch_workspace_size(ops: Sequence[pcg_operator], opts: Sequence[pcg_options]) -> int:
    k = len(ops)
    OA, PA = (pcg_operator * k)(*ops), (pcg_options * k)(*opts)
    n = C.c_size_t()
    _check(lib().pcg_batch_workspace_size(k, OA, PA, C.byref(n)), "pcg_batch_workspace_size")
    return n.value


def pcg_batch_solve(ops, opts, b_ptrs, x_ptrs, workspace: int, nbytes: int, stream: int) -> list:
    k = len(ops)
    OA, PA = (pcg_operator * k)(*ops), (pcg_options * k)(*opts)
    BA, XA = (C.c_void_p * k)(*b_ptrs), (C.c_void_p * k)(*x_ptrs)
    R = (pcg_result * k)()
    _check(lib().pcg_batch_solve(k, OA, PA, BA, XA, R, workspace, nbytes, stream), "pcg_batch_solve")
    return list(R)


def pcg_batch_tune(ops, opts, b_ptrs, x0_ptrs, x_ptrs, workspace: int, nbytes: int, stream: int) -> float:
    """Launch-shape autotuner of the batched pass: writes the fastest grid and
    graph length into opts[0] (grid_blocks, iters_per_launch); returns the
    winning solve time in ms.  x_ptrs are scratch, x0_ptrs the initial guesses."""
    k = len(ops)
    OA, PA = (pcg_operator * k)(*ops), (pcg_options * k)(*opts)
    BA, X0, XA = (C.c_void_p * k)(*b_ptrs), (C.c_void_p * k)(*x0_ptrs), (C.c_void_p * k)(*x_ptrs)
    best = C.c_double()
    _check(lib().pcg_batch_tune(k, OA, PA, BA, X0, XA, workspace, nbytes, stream, C.byref(best)), "pcg_batch_tune")
    opts[0].grid_blocks = PA[0].grid_blocks
    opts[0].iters_per_launch = PA[0].iters_per_launch
    return best.value


def pcg_server_create(arena: int, nbytes: int, max_slots: int, stream: int) -> int:
    h = C.c_void_p()
    _check(lib().pcg_server_create(C.byref(h), arena, nbytes, max_slots, stream), "pcg_server_create")
    return h.value


def pcg_submit(server: int, op: pcg_operator, opt: pcg_options, b: int, x: int) -> int:
    t = C.c_uint64()
    _check(lib().pcg_submit(server, C.byref(op), C.byref(opt), b, x, C.byref(t)), "pcg_submit")
    return t.value


def pcg_poll(server: int, ticket: int):
    r = pcg_result()
    st = lib().pcg_poll(server, ticket, C.byref(r))
    if st == PCG_PENDING:
        return None
    _check(st, "pcg_poll")
    return r


def pcg_wait(server: int, ticket: int) -> pcg_result:
    r = pcg_result()
    _check(lib().pcg_wait(server, ticket, C.byref(r)), "pcg_wait")
    return r


def pcg_server_info(server: int) -> dict:
    st = pcg_server_stats()
    _check(lib().pcg_server_info(server, C.byref(st)), "pcg_server_info")
    return {name: getattr(st, name) for name, _ in pcg_server_stats._fields_}


def pcg_server_destroy(server: int) -> None:
    _check(lib().pcg_server_destroy(server), "pcg_server_destroy")


# ------------------------------------------------------------------ helpers
# (marshalling: operator description -> device arrays, tensors -> pointers)

def _torch():
    import torch
    return torch


def current_stream_handle(device=None) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class DeviceOperator:
    """Device copies of an operator description (an object with ``kind``,
    ``n``, ``nx``, ``ny``, ``nz``, ``diag``, ``off``, ``shift`` and, for CSR,
    ``row_ptr``, ``col``, ``val``) and its ``pcg_operator`` struct."""

    def __init__(self, op, prec: int = PCG_FP64, device="cuda"):
        torch = _torch()
        self.keep = []
        self.prec = prec
        s = pcg_operator()
        s.kind = OPKIND[op.kind]
        s.n = int(op.n)
        if op.kind == "csr":
            vdt = torch.float64 if prec == PCG_FP64 else torch.float32
            rp = torch.as_tensor(op.row_ptr).to(torch.int32).to(device)
            ci = torch.as_tensor(op.col).to(torch.int32).to(device)
            va = torch.as_tensor(op.val).to(vdt).to(device)
            self.keep += [rp, ci, va]
            s.row_ptr, s.col_idx, s.vals = rp.data_ptr(), ci.data_ptr(), va.data_ptr()
            s.nnz = int(op.row_ptr[-1])
            s.nx, s.ny, s.nz = 0, 0, 1
        else:
            s.nx, s.ny = int(op.nx), int(op.ny)
            s.nz = int(op.nz) if op.kind == "3d7" else 1
            s.diag, s.offdiag, s.shift = float(op.diag), float(op.off), float(op.shift)
        self.struct = s


def _device_op(op, prec: int, device) -> "DeviceOperator":
    """`op` itself when it is already a DeviceOperator of precision `prec`
    (operators resident on the device, uploaded once), else a new upload."""
    if isinstance(op, DeviceOperator):
        if op.prec != prec:
            raise ValueError("the device operator was uploaded for another precision")
        return op
    return DeviceOperator(op, prec, device)


def pcg_tune_workspace_size(op: pcg_operator, opt: pcg_options) -> int:
    n = C.c_size_t()
    _check(lib().pcg_tune_workspace_size(C.byref(op), C.byref(opt), C.byref(n)), "pcg_tune_workspace_size")
    return n.value


def pcg_tune(op: pcg_operator, opt: pcg_options, workspace: int, nbytes: int, b: int, x: int,
             stream: Optional[int]) -> float:
    """Tune `opt` in place; returns microseconds per pass of the chosen shape."""
    us = C.c_double()
    _check(lib().pcg_tune(C.byref(op), C.byref(opt), workspace, nbytes, b, x, stream, C.byref(us)), "pcg_tune")
    return us.value


def tune(op, options: pcg_options, b=None, device="cuda", stream: Optional[int] = None):
    """Run the launch-shape autotuner (pcg_tune) for `op` and `options`;
    returns (tuned options, microseconds per pass).  b: a device right-hand
    side (default: a seeded uniform random vector)."""
    torch = _torch()
    dev = _device_op(op, options.prec, device)
    n = int(dev.struct.n)
    if b is None:
        g = torch.Generator(device=device)
        g.manual_seed(0)
        b = torch.rand(n, dtype=torch.float64, device=device, generator=g) * 2.0 - 1.0
    x = torch.zeros(n, dtype=torch.float64, device=device)
    nbytes = pcg_tune_workspace_size(dev.struct, options)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (ws.data_ptr() + 255) & ~255
    st = current_stream_handle() if stream is None else stream
    out = pcg_options.from_buffer_copy(options)
    for k in ("_sched_keep",):
        if hasattr(options, k):
            setattr(out, k, getattr(options, k))
    us = pcg_tune(dev.struct, out, ptr, nbytes, b.data_ptr(), x.data_ptr(), st)
    torch.cuda.synchronize()
    return out, us


PCG_PROBE_NT, PCG_PROBE_BLOCKED, PCG_PROBE_FP32, PCG_PROBE_WIDE = 1, 2, 4, 8


def PCG_PROBE_BLOCKS_PER_CU(k: int) -> int:
    return int(k) << 8


def pcg_stream_probe(nin: int, nout: int, flags: int, n: int, buffer: int, nbytes: int, reps: int,
                     stream: int) -> float:
    """Average microseconds of one streaming launch (nin read, nout written
    streams of n binary64 values)."""
    us = C.c_double()
    _check(lib().pcg_stream_probe(int(nin), int(nout), int(flags), int(n), buffer, int(nbytes), int(reps),
                                  stream, C.byref(us)), "pcg_stream_probe")
    return us.value


def stream_probe_bytes(nin: int, nout: int, n: int) -> int:
    return (nin + nout) * ((8 * n + 4095) // 4096 * 4096) + 65536


def _f64(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.float64)


def pcg_psi(alpha, beta, i: int, sigma: float) -> float:
    """psi_i(sigma) from a recorded alpha / beta history (host)."""
    a, b = _f64(alpha), _f64(beta)
    if len(a) <= i or len(b) <= i:
        raise ValueError("alpha and beta need i + 1 entries")
    out = C.c_double()
    _check(lib().pcg_psi(a.ctypes.data, b.ctypes.data, int(i), float(sigma), C.byref(out)), "pcg_psi")
    return out.value


def pcg_psi_variable(alpha, beta, i: int, sigma_schedule) -> float:
    a, b, s = _f64(alpha), _f64(beta), _f64(sigma_schedule)
    if len(a) <= i or len(b) <= i:
        raise ValueError("alpha and beta need i + 1 entries")
    out = C.c_double()
    _check(lib().pcg_psi_variable(a.ctypes.data, b.ctypes.data, int(i), s.ctypes.data, len(s), C.byref(out)),
           "pcg_psi_variable")
    return out.value


def pcg_select_shift(alpha, beta, i: int, grid, slack: float = 2.0):
    """(sigma*, psi values on the grid)."""
    import numpy as np
    a, b, g = _f64(alpha), _f64(beta), _f64(grid)
    if len(a) <= i or len(b) <= i:
        raise ValueError("alpha and beta need i + 1 entries")
    vals = np.empty(len(g))
    best = C.c_double()
    _check(lib().pcg_select_shift(a.ctypes.data, b.ctypes.data, int(i), g.ctypes.data, len(g), float(slack),
                                  vals.ctypes.data, C.byref(best)), "pcg_select_shift")
    return best.value, vals


def make_options(method: str = "pipe_shift", jacobi: bool = False, fp32: bool = False,
                 sigma: Optional[float] = None, rtol: float = 1e-10, max_iter: int = 1000,
                 true_residual_check: bool = True, replace_max: int = 4, iters_per_launch: int = 0,
                 history_cap: int = 0, block_size: int = 0, grid_blocks: int = 0, timing: bool = False,
                 use_graph: bool = True, variant: int = 0, sigma_schedule=None, rr_tau: float = 0.0,
                 rr_period: int = 0, rr_floor: float = 0.0, run_through_breakdown: bool = False) -> pcg_options:
    """Options for pcg_create.  ``sigma_schedule`` (method "pipe_var") lists
    sigma_{-1}, sigma_0, sigma_1, ...; the returned struct keeps the array
    alive until the solver copies it at creation."""
    o = pcg_default_options()
    o.method = METHOD[method]
    o.pc = PCG_PC_JACOBI if jacobi else PCG_PC_NONE
    o.prec = PCG_FP32_STREAM if fp32 else PCG_FP64
    o.sigma = math.nan if sigma is None else float(sigma)
    o.rtol = float(rtol)
    o.max_iter = int(max_iter)
    o.true_residual_check = int(bool(true_residual_check))
    o.replace_max = int(replace_max)
    o.iters_per_launch = int(iters_per_launch)
    o.history_cap = int(history_cap)
    o.block_size = int(block_size)
    o.grid_blocks = int(grid_blocks)
    o.timing = int(bool(timing))
    o.use_graph = int(bool(use_graph))
    o.variant = int(variant)
    o.rr_tau = float(rr_tau)
    o.rr_period = int(rr_period)
    o.rr_floor = float(rr_floor)
    o.flags = PCG_FLAG_RUN_THROUGH_BREAKDOWN if run_through_breakdown else 0
    if sigma_schedule is not None:
        import numpy as np
        sched = np.ascontiguousarray(sigma_schedule, dtype=np.float64)
        o._sched_keep = sched
        o.sigma_schedule = sched.ctypes.data
        o.sigma_schedule_len = len(sched)
    return o


class Solver:
    """One solver: device operator, torch-allocated workspace, C handle."""

    def __init__(self, op, options: pcg_options, device="cuda", stream: Optional[int] = None):
        import numpy as np
        torch = _torch()
        self.dev = _device_op(op, options.prec, device)
        self.opt = options
        self.hist = None
        if options.history_cap > 0:
            self.hist = np.full((options.history_cap, PCG_HISTORY_FIELDS), np.nan)
            self.opt.history = self.hist.ctypes.data
        self.nbytes = pcg_workspace_size(self.dev.struct, self.opt)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = current_stream_handle() if stream is None else stream
        self.handle = pcg_create(self.dev.struct, self.opt, self.ws_ptr, self.nbytes, self.stream)

    def solve(self, b, x) -> dict:
        r = pcg_solve(self.handle, b.data_ptr(), x.data_ptr())
        return result_dict(r, self.hist)

    def true_residual(self, b, x) -> float:
        return pcg_true_residual(self.handle, b.data_ptr(), x.data_ptr())

    def info(self) -> dict:
        return pcg_solver_info(self.handle)

    def close(self):
        if self.handle:
            pcg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def result_dict(r: pcg_result, hist=None) -> dict:
    d = dict(status=OUTCOME.get(r.status, str(r.status)), iterations=r.iterations,
             replacements=r.replacements, launches=r.launches, rel_res_recursive=r.rel_res_recursive,
             rel_res_true=r.rel_res_true, seconds=r.seconds, iter_kernel_ms=r.iter_kernel_ms,
             iter_passes=r.iter_passes, admitted_at=r.admitted_at, sigma=r.sigma)
    if hist is not None:
        k = r.iterations + 1
        d.update(res=hist[:k, 0].copy(), alpha=hist[:k, 1].copy(), beta=hist[:k, 2].copy(),
                 gamma=hist[:k, 3].copy(), delta=hist[:k, 4].copy())
    return d


class Batch:
    """A batch of independent systems solved by pcg_batch_solve: device
    operators, torch-allocated workspace, per-system options."""

    def __init__(self, ops, options, device="cuda"):
        import numpy as np
        torch = _torch()
        self.devs = [_device_op(op, o.prec, device) for op, o in zip(ops, options)]
        self.opts = list(options)
        self.hists = []
        for o in self.opts:
            if o.history_cap > 0:
                h = np.full((o.history_cap, PCG_HISTORY_FIELDS), np.nan)
                o.history = h.ctypes.data
                self.hists.append(h)
            else:
                self.hists.append(None)
        self.structs = [d.struct for d in self.devs]
        self.nbytes = pcg_batch_workspace_size(self.structs, self.opts)
        self.ws = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        self.ws_ptr = (self.ws.data_ptr() + 255) & ~255

    def solve(self, bs, xs, stream: Optional[int] = None) -> list:
        st = current_stream_handle() if stream is None else stream
        res = pcg_batch_solve(self.structs, self.opts, [b.data_ptr() for b in bs], [x.data_ptr() for x in xs],
                              self.ws_ptr, self.nbytes, st)
        return [result_dict(r, h) for r, h in zip(res, self.hists)]

    def tune(self, bs, x0s, xs, stream: Optional[int] = None) -> dict:
        """pcg_batch_tune on this batch; later solves use the chosen shape."""
        st = current_stream_handle() if stream is None else stream
        ms = pcg_batch_tune(self.structs, self.opts, [b.data_ptr() for b in bs], [x.data_ptr() for x in x0s],
                            [x.data_ptr() for x in xs], self.ws_ptr, self.nbytes, st)
        return {"grid_blocks": self.opts[0].grid_blocks, "iters_per_launch": self.opts[0].iters_per_launch,
                "solve_ms": ms}


class Server:
    """A continuously batching solve server over a torch-allocated HBM arena."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, device="cuda", stream: Optional[int] = None):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=device)
        self.arena_ptr = (self.arena.data_ptr() + 255) & ~255
        self.device = device
        st = current_stream_handle() if stream is None else stream
        self.handle = pcg_server_create(self.arena_ptr, int(arena_bytes), int(max_slots), st)
        self._keep = {}

    def submit(self, op, options: pcg_options, b, x) -> int:
        """Enqueue a solve; b, x are device tensors (binary64) kept alive by
        the server object until the ticket is collected."""
        import numpy as np
        dev = _device_op(op, options.prec, self.device)
        hist = None
        if options.history_cap > 0:
            hist = np.full((options.history_cap, PCG_HISTORY_FIELDS), np.nan)
            options.history = hist.ctypes.data
        t = pcg_submit(self.handle, dev.struct, options, b.data_ptr(), x.data_ptr())
        self._keep[t] = (dev, options, b, x, hist)
        return t

    def poll(self, ticket: int):
        r = pcg_poll(self.handle, ticket)
        if r is None:
            return None
        return result_dict(r, self._keep.pop(ticket)[4])

    def wait(self, ticket: int) -> dict:
        try:
            r = pcg_wait(self.handle, ticket)
        except PcgError:
            self._keep.pop(ticket, None)
            raise
        return result_dict(r, self._keep.pop(ticket)[4])

    def info(self) -> dict:
        return pcg_server_info(self.handle)

    def close(self):
        if self.handle:
            pcg_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
