"""The C ABI without a GPU: the library loads, exports every function
include/pcg.h declares, and rejects invalid arguments before any device
work (these paths make no HIP call)."""
import ctypes as C
import math

import pytest

from paper_1706_05988_amd import pcg as P


def test_library_exports_every_declared_function():
    lib = P.lib()
    declared = P.header_functions()
    assert len(declared) >= 15
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_names_match_header():
    for f in P.header_functions():
        assert hasattr(P, f), f


def test_status_strings():
    assert P.pcg_status_str(P.PCG_OK) == "ok"
    assert "invalid" in P.pcg_status_str(P.PCG_ERR_INVALID)
    assert P.pcg_status_str(12345) == "unknown status"


def stencil_op(kind=P.PCG_OP_STENCIL3D7, nx=16, ny=16, nz=16):
    op = P.pcg_operator()
    op.kind, op.nx, op.ny, op.nz = kind, nx, ny, nz
    op.n = nx * ny * nz
    op.diag, op.offdiag = 6.0, -1.0
    return op


def test_workspace_size_scales_with_vectors():
    op = stencil_op()
    o = P.make_options()
    base = P.pcg_workspace_size(op, o)
    o.pc = P.PCG_PC_JACOBI
    jac = P.pcg_workspace_size(op, o)
    o.prec = P.PCG_FP32_STREAM
    f32 = P.pcg_workspace_size(op, o)
    assert jac > base > 0 and f32 < jac
    # 10 blocked slots (x + 9 vectors) of binary64 per unknown, plus small tables
    assert jac >= op.n * 8 * 10


@pytest.mark.parametrize("field,value", [
    ("n", 0), ("nx", 0), ("kind", 7), ("n", 17),
])
def test_invalid_operator(field, value):
    op = stencil_op()
    setattr(op, field, value)
    with pytest.raises(P.PcgError) as ei:
        P.pcg_workspace_size(op, P.make_options())
    assert ei.value.status == P.PCG_ERR_INVALID


@pytest.mark.parametrize("field,value", [
    ("method", 5), ("pc", 3), ("prec", 2), ("max_iter", -1), ("rtol", 0.0), ("rtol", math.inf),
    ("sigma", -1.0), ("iters_per_launch", 3), ("block_size", 96), ("block_size", 512), ("history_cap", 4),
    ("replace_max", -2),
])
def test_invalid_options(field, value):
    o = P.make_options()
    setattr(o, field, value)
    with pytest.raises(P.PcgError) as ei:
        P.pcg_workspace_size(stencil_op(), o)
    assert ei.value.status == P.PCG_ERR_INVALID
    assert "invalid argument" in P.pcg_last_error()


def test_csr_needs_arrays():
    op = P.pcg_operator()
    op.kind, op.n, op.nnz = P.PCG_OP_CSR, 10, 10
    with pytest.raises(P.PcgError):
        P.pcg_workspace_size(op, P.make_options())


def test_create_rejects_before_device_work():
    op = stencil_op()
    o = P.make_options()
    need = P.pcg_workspace_size(op, o)
    lib = P.lib()
    h = C.c_void_p()
    # null workspace, misaligned workspace, too small workspace
    assert lib.pcg_create(C.byref(h), C.byref(op), C.byref(o), None, need, None) == P.PCG_ERR_INVALID
    assert lib.pcg_create(C.byref(h), C.byref(op), C.byref(o), 0x1008, need, None) == P.PCG_ERR_INVALID
    assert lib.pcg_create(C.byref(h), C.byref(op), C.byref(o), 0x100000, need - 256, None) == P.PCG_ERR_INVALID
    assert lib.pcg_solve(None, None, None, None) == P.PCG_ERR_STATE
    assert lib.pcg_destroy(None) == P.PCG_OK


def test_batch_rejects_cg_and_mixed_precision():
    op = stencil_op()
    a, b = P.make_options(), P.make_options(method="cg")
    with pytest.raises(P.PcgError):
        P.pcg_batch_workspace_size([op, op], [a, b])
    c = P.make_options(fp32=True)
    with pytest.raises(P.PcgError):
        P.pcg_batch_workspace_size([op, op], [a, c])
    n1 = P.pcg_batch_workspace_size([op], [a])
    n2 = P.pcg_batch_workspace_size([op, op], [a, a])
    assert n2 > n1


def test_option_flags_validated():
    op = stencil_op()
    o = P.make_options(run_through_breakdown=True)
    assert o.flags == P.PCG_FLAG_RUN_THROUGH_BREAKDOWN
    assert P.pcg_workspace_size(op, o) > 0
    bad = P.make_options()
    bad.flags = 0x40
    with pytest.raises(P.PcgError) as ei:
        P.pcg_workspace_size(op, bad)
    assert ei.value.status == P.PCG_ERR_INVALID
    # the batched pass (and the server) take no flags
    with pytest.raises(P.PcgError):
        P.pcg_batch_workspace_size([op], [o])


def test_batch_rejects_an_empty_batch():
    with pytest.raises(P.PcgError) as ei:
        P.pcg_batch_workspace_size([], [])
    assert ei.value.status == P.PCG_ERR_INVALID


def test_server_argument_checks():
    lib = P.lib()
    h = C.c_void_p()
    assert lib.pcg_server_create(C.byref(h), None, 1 << 20, 4, None) == P.PCG_ERR_INVALID
    assert lib.pcg_server_create(C.byref(h), 0x1000, 1 << 20, 0, None) == P.PCG_ERR_INVALID
    r = P.pcg_result()
    assert lib.pcg_poll(None, 1, C.byref(r)) == P.PCG_ERR_STATE
    assert lib.pcg_server_destroy(None) == P.PCG_OK


def test_variable_shift_schedule_validation():
    """PCG_PIPE_VAR_SHIFT needs a host schedule of 1 .. 2^24 finite, >= 0
    shifts; every violation is PCG_ERR_INVALID before any device work."""
    op = stencil_op()
    ok = P.make_options(method="pipe_var", sigma_schedule=[0.5, 1.0, 2.0])
    assert P.pcg_workspace_size(op, ok) > 0
    bad = [P.make_options(method="pipe_var"),                              # no schedule
           P.make_options(method="pipe_var", sigma_schedule=[1.0, -0.5]),   # negative shift
           P.make_options(method="pipe_var", sigma_schedule=[1.0, math.nan])]
    for o in bad:
        with pytest.raises(P.PcgError) as ei:
            P.pcg_workspace_size(op, o)
        assert ei.value.status == P.PCG_ERR_INVALID


def test_variable_shift_workspace_holds_the_schedule():
    op = stencil_op()
    a = P.pcg_workspace_size(op, P.make_options(method="pipe_var", sigma_schedule=[1.0]))
    b = P.pcg_workspace_size(op, P.make_options(method="pipe_var", sigma_schedule=[1.0] * 100_000))
    assert b - a >= 8 * 100_000 - 256  # the schedule region, 256-byte rounded


def test_pcg_rr_option_validation():
    op = stencil_op()
    assert P.pcg_workspace_size(op, P.make_options(method="pipe_rr", rr_period=16, rr_tau=1e-5)) > 0
    with pytest.raises(P.PcgError) as ei:
        P.pcg_workspace_size(op, P.make_options(method="pipe_rr", rr_period=-1))
    assert ei.value.status == P.PCG_ERR_INVALID


def test_option_struct_layout_matches_header():
    """The ctypes mirrors have the C structs' sizes and field offsets
    (compiled from include/pcg.h with the host C compiler)."""
    import ctypes as C
    import os
    import subprocess
    import tempfile
    fields = {"pcg_options": [f for f, _ in P.pcg_options._fields_],
              "pcg_operator": [f for f, _ in P.pcg_operator._fields_],
              "pcg_result": [f for f, _ in P.pcg_result._fields_],
              "pcg_server_stats": [f for f, _ in P.pcg_server_stats._fields_],
              "pcg_solver_shape": [f for f, _ in P.pcg_solver_shape._fields_]}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "pcg.h"', "int main(void) {"]
    for st, fs in fields.items():
        src.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            src.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    src.append("return 0; }")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        open(c, "w").write("\n".join(src))
        exe = os.path.join(d, "layout")
        subprocess.run(["gcc", "-std=c99", "-I", inc, c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split() for line in out if line)
    for st, fs in fields.items():
        cls = getattr(P, st)
        assert int(got[st]) == C.sizeof(cls), st
        for f in fs:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def test_tune_workspace_covers_every_candidate():
    import ctypes as C
    op = stencil_op()
    o = P.make_options(jacobi=True)
    n = C.c_size_t()
    assert P.lib().pcg_tune_workspace_size(C.byref(op), C.byref(o), C.byref(n)) == P.PCG_OK
    assert n.value >= P.pcg_workspace_size(op, o)
    # a CSR operator: the candidates on its sliced-ELL copy need more room
    csr = P.pcg_operator()
    csr.kind, csr.n, csr.nnz = P.PCG_OP_CSR, 4096, 5 * 4096
    csr.row_ptr, csr.col_idx, csr.vals = 0x100000, 0x200000, 0x300000
    o32 = P.make_options(jacobi=True, fp32=True)
    assert P.lib().pcg_tune_workspace_size(C.byref(csr), C.byref(o32), C.byref(n)) == P.PCG_OK
    sell = P.make_options(jacobi=True, fp32=True, variant=P.PCG_VAR_SET | P.PCG_VAR_CSR_SELL | P.PCG_VAR_EPT1,
                          block_size=128, grid_blocks=2048)
    plain = P.make_options(jacobi=True, fp32=True, variant=P.PCG_VAR_SET | P.PCG_VAR_EPT1, block_size=128,
                           grid_blocks=2048)
    assert P.pcg_workspace_size(csr, sell) > P.pcg_workspace_size(csr, plain)
    assert n.value >= P.pcg_workspace_size(csr, sell)
    # ... and the sorted copy also its per-slot (length, position) words and
    # per-tile column windows
    srt, sell4 = (P.make_options(jacobi=True, fp32=True, variant=P.PCG_VAR_SET | form | P.PCG_VAR_EPT4,
                                 block_size=128, grid_blocks=2048)
                  for form in (P.PCG_VAR_CSR_SELL_SORTED, P.PCG_VAR_CSR_SELL))
    # 4 bytes per slot, and 8 per tile (8 tiles of 512 rows) for the column
    # windows, in 256-byte units
    assert P.pcg_workspace_size(csr, srt) == P.pcg_workspace_size(csr, sell4) + 4 * 4096 + 256
    assert n.value >= P.pcg_workspace_size(csr, srt)
    # the built-in shape reserves both copies' offsets and one set of entries
    assert P.pcg_workspace_size(csr, o32) >= P.pcg_workspace_size(csr, srt)


def test_solver_info_rejects_null():
    import ctypes as C
    sh = P.pcg_solver_shape()
    assert P.lib().pcg_solver_info(None, C.byref(sh)) == P.PCG_ERR_INVALID
    assert P.lib().pcg_solver_info(C.c_void_p(4096), None) == P.PCG_ERR_INVALID


def test_tune_rejects_bad_arguments_before_device_work():
    """Aliased b / x and a too-small workspace are PCG_ERR_INVALID; no device
    pointer is touched (the ones passed here are not device memory)."""
    import ctypes as C
    op = stencil_op()
    o = P.make_options()
    us = C.c_double()
    fake = 4096
    assert P.lib().pcg_tune(C.byref(op), C.byref(o), fake, 1 << 40, fake, fake, None, C.byref(us)) == \
        P.PCG_ERR_INVALID
    assert P.lib().pcg_tune(C.byref(op), C.byref(o), fake, 16, fake, fake + 8, None, C.byref(us)) == \
        P.PCG_ERR_INVALID


def test_batch_tune_rejects_bad_arguments_before_device_work():
    """Null arrays, an x0 aliasing its x and a too-small workspace are
    PCG_ERR_INVALID, found before any device call (the pointers passed here
    are not device memory)."""
    import ctypes as C
    op = stencil_op()
    o = P.make_options(method="pipe_shift", fp32=True)
    OA, PA = (P.pcg_operator * 1)(op), (P.pcg_options * 1)(o)
    fake = 4096
    B, X0, X = (C.c_void_p * 1)(fake), (C.c_void_p * 1)(fake + 8), (C.c_void_p * 1)(fake + 16)
    ms = C.c_double()
    L = P.lib()
    assert L.pcg_batch_tune(0, OA, PA, B, X0, X, fake, 1 << 40, None, C.byref(ms)) == P.PCG_ERR_INVALID
    assert L.pcg_batch_tune(1, OA, PA, B, None, X, fake, 1 << 40, None, C.byref(ms)) == P.PCG_ERR_INVALID
    assert L.pcg_batch_tune(1, OA, PA, B, X, X, fake, 1 << 40, None, C.byref(ms)) == P.PCG_ERR_INVALID
    assert L.pcg_batch_tune(1, OA, PA, B, X0, X, fake, 16, None, C.byref(ms)) == P.PCG_ERR_INVALID
    assert PA[0].grid_blocks == 0 and PA[0].iters_per_launch == 0  # unchanged on error


def test_static_solve_rejects_before_device_work():
    """pcg_solve_static checks its arguments and the scratch limit before any
    HIP call: a solve whose workspace exceeds the static scratch is refused
    with a message that states both sizes."""
    lib = P.lib()
    r = P.pcg_result()
    o = P.make_options(jacobi=True)
    big = stencil_op(nx=256, ny=256, nz=256)
    need = P.pcg_workspace_size(big, o)
    assert need > P.PCG_STATIC_SCRATCH_BYTES
    st = lib.pcg_solve_static(C.byref(big), C.byref(o), 0x100000, 0x200000, C.byref(r), None)
    assert st == P.PCG_ERR_INVALID
    msg = P.pcg_last_error()
    assert str(need) in msg and str(P.PCG_STATIC_SCRATCH_BYTES) in msg
    small = stencil_op()
    assert lib.pcg_solve_static(C.byref(small), C.byref(o), 0x100000, 0x200000, None, None) == P.PCG_ERR_INVALID
    assert lib.pcg_solve_static(C.byref(small), C.byref(o), None, 0x200000, C.byref(r), None) == P.PCG_ERR_INVALID
    bad = P.make_options(rtol=-1.0)
    assert lib.pcg_solve_static(C.byref(small), C.byref(bad), 0x100000, 0x200000, C.byref(r), None) == P.PCG_ERR_INVALID


def test_static_scratch_size_matches_header():
    import re
    txt = open(P.HEADER).read()
    m = re.search(r"#define PCG_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", txt)
    assert m, "PCG_STATIC_SCRATCH_BYTES not found in pcg.h"
    assert int(m.group(1)) << int(m.group(2)) == P.PCG_STATIC_SCRATCH_BYTES


def test_stream_probe_rejects_before_device_work():
    lib = P.lib()
    us = C.c_double()
    n = 1 << 20
    need = P.stream_probe_bytes(9, 9, n)
    assert need == 18 * 8 * n + 65536
    assert P.stream_probe_bytes(1, 1, 513) == 2 * 8192 + 65536
    assert lib.pcg_stream_probe(9, 9, 16, n, 0x100000, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 8 | 2, n, 0x100000, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 8 | 4, 1023, 0x100000, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    # an unsupported mix, a short buffer, a misaligned buffer, bad sizes
    assert lib.pcg_stream_probe(3, 3, 1, n, 0x100000, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 1, n, 0x100000, need - 8, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 1, n, 0x100008, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 1, 0, 0x100000, need, 10, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 1, n, 0x100000, need, 0, None, C.byref(us)) == P.PCG_ERR_INVALID
    assert lib.pcg_stream_probe(9, 9, 1, n, 0x100000, need, 10, None, None) == P.PCG_ERR_INVALID
