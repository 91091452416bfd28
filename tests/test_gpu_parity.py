"""Parity of the HIP path (through the C ABI) with the oracle.

Tolerances (FP64 form): the recursive residual history sqrt(rho_i)/||b||
matches the oracle's to 1e-10 relative over the first 50 iterations, and the
final explicit residual ||b - A x||/||b|| matches to 1e-12 absolute (p-CG: a
10x band, its stagnation level being rounding-determined).  The GPU sums
dot products in a different order and contracts multiply-adds, so iterates
differ from the oracle's by rounding only.
"""
import math

import numpy as np
import pytest

import oracle
import problems

pytestmark = pytest.mark.gpu

METHODS = ["cg", "pipe", "pipe_shift"]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def gpu_solve(torch, p, method, jacobi=None, fp32=False, sigma=None, rtol=None, max_iter=None,
              hist=True, x0=None, **kw):
    from paper_1706_05988_amd import pcg as P
    jac = p.jacobi if jacobi is None else jacobi
    if sigma is None:
        sigma = p.sigma if method == "pipe_shift" else 0.0
    mi = p.max_iter if max_iter is None else max_iter
    opt = P.make_options(method=method, jacobi=jac, fp32=fp32, sigma=sigma,
                         rtol=p.rtol if rtol is None else rtol, max_iter=mi,
                         history_cap=(mi + 2) if hist else 0, **kw)
    s = P.Solver(p.op, opt)
    b = torch.from_numpy(p.b).cuda()
    x = torch.from_numpy(p.x0 if x0 is None else x0).clone().cuda()
    r = s.solve(b, x)
    torch.cuda.synchronize()
    r["x"] = x.cpu().numpy()
    r["info"] = s.info()
    s.close()
    return r


def oracle_solve(p, method, jacobi=None, fp32=False, sigma=None, rtol=None, max_iter=None, threads=8, **kw):
    return oracle.solve(p.op, p.b, p.x0, method=method,
                        sigma=(p.sigma if method == "pipe_shift" else 0.0) if sigma is None else sigma,
                        rtol=p.rtol if rtol is None else rtol,
                        max_iter=p.max_iter if max_iter is None else max_iter,
                        jacobi=p.jacobi if jacobi is None else jacobi, fp32_storage=fp32, threads=threads, **kw)


def check_history(g, o, upto=50, rtol=1e-10):
    """Compare the first `upto` iterations, stopping where the recursive
    residual has fallen to 1e-12 (beyond it the histories are rounding noise)."""
    k = min(upto, len(o["res"]) - 1, len(g["res"]) - 1)
    below = np.nonzero(o["res"][: k + 1] < 1e-12)[0]
    if below.size:
        k = max(1, int(below[0]) - 1)
    np.testing.assert_allclose(g["res"][: k + 1], o["res"][: k + 1], rtol=rtol)
    # alpha and beta of the same iterations
    np.testing.assert_allclose(g["alpha"][:k], o["alpha"][:k], rtol=rtol)
    np.testing.assert_allclose(g["beta"][1:k], o["beta"][1:k], rtol=rtol)


# ---------------------------------------------------------------- config 1

@pytest.mark.parametrize("method", METHODS)
def test_config1_poisson2d_history_and_final_residual(torch, method):
    p = problems.poisson2d_manufactured(100)
    g = gpu_solve(torch, p, method, true_residual_check=False)
    o = oracle_solve(p, method)
    assert g["status"] == o["status"] == "converged"
    assert abs(g["iterations"] - o["iterations"]) <= 1
    check_history(g, o)
    if method == "pipe":
        assert g["rel_res_true"] <= 10 * o["rel_res_true"]
    else:
        assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12
        assert g["rel_res_true"] <= 1e-12
    np.testing.assert_allclose(g["x"], p.x_true, rtol=1e-8)


@pytest.mark.parametrize("method", METHODS)
def test_lapl200_table1_on_gpu(torch, method):
    """500 iterations of lapl200 (Table 1) run through any breakdown, as the
    paper's accuracy runs do: CG and p-CG-sh reach ~6.8e-12; p-CG stagnates
    orders of magnitude higher.  Its level is set by rounding (the oracle's
    lands at ~4e-9), so it is held to the oracle's own pin: at least 100x
    CG's printed level and at most 10x its own printed 3.1e-7."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_lapl200.json")) as f:
        printed = json.load(f)["true_residual"][method]  # ||b|| = 1: absolute = relative
    p = problems.lapl200()
    g = gpu_solve(torch, p, method, true_residual_check=False, rtol=1e-30, max_iter=500,
                  run_through_breakdown=True)
    o = oracle_solve(p, method, rtol=1e-30, max_iter=500, ignore_breakdown=True)
    check_history(g, o)
    assert g["iterations"] == 500
    if method == "pipe":
        with open(os.path.join(os.path.dirname(__file__), "golden", "table1_lapl200.json")) as f:
            cg_printed = json.load(f)["true_residual"]["cg"]
        assert 100 * cg_printed <= g["rel_res_true"] <= 10 * printed
    else:
        assert g["rel_res_true"] <= 3 * printed
        assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-11


def test_breakdown_stops_without_the_flag(torch):
    """Without the run-through flag the library stops p-CG on lapl200 at the
    first non-positive alpha or delta, with status breakdown."""
    p = problems.lapl200()
    g = gpu_solve(torch, p, "pipe", true_residual_check=False, rtol=1e-30, max_iter=500)
    assert g["status"] == "breakdown" and g["iterations"] < 500


# ---------------------------------------------------------------- 3-D, Jacobi, ragged

@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("jacobi", [False, True])
def test_3d_ragged_grid(torch, method, jacobi):
    op = problems.stencil3d(37, 41, 43)  # 65,231 unknowns: many tiles and a ragged tail
    rng = np.random.default_rng(11)
    xt = rng.uniform(-1, 1, op.n)
    b = problems.to_scipy(op) @ xt
    p = problems.Problem("ragged3d", op, b, np.zeros(op.n), xt, jacobi=jacobi,
                         sigma=1.0 if jacobi else 6.0, rtol=1e-10, max_iter=2000)
    g = gpu_solve(torch, p, method, true_residual_check=False)
    o = oracle_solve(p, method)
    assert g["status"] == o["status"] == "converged"
    assert abs(g["iterations"] - o["iterations"]) <= 1
    check_history(g, o)
    assert abs(g["rel_res_true"] - o["rel_res_true"]) <= (1e-11 if method == "pipe" else 1e-12)


@pytest.mark.parametrize("dims,jacobi", [((37, 41, 43), True), ((24, 17, 30), False), ((5, 3, 11), True),
                                         ((64, 64, 40), True), ((16, 12, 9), True)])
def test_cg_zmarch_pass_matches_oracle(torch, dims, jacobi):
    """Classic CG with pass A marching along z through LDS (forced here on
    grids where the built-in rule would run the plain pass; 64x64x40 spans
    several row chunks and segments, 16x12x9 ends in a one-plane segment):
    the oracle's history to 1e-10 over 50
    iterations and its final explicit residual to 1e-12, and the plain
    pass's history to rounding."""
    from paper_1706_05988_amd import pcg as P
    op = problems.stencil3d(*dims)
    rng = np.random.default_rng(sum(dims))
    xt = rng.uniform(-1, 1, op.n)
    p = problems.Problem("zm3d", op, problems.to_scipy(op) @ xt, np.zeros(op.n), xt, jacobi=jacobi,
                         sigma=0.0, rtol=1e-10, max_iter=3000)
    zm = gpu_solve(torch, p, "cg", true_residual_check=False, variant=P.PCG_VAR_SET | P.PCG_VAR_CG_ZMARCH)
    plain = gpu_solve(torch, p, "cg", true_residual_check=False)
    o = oracle_solve(p, "cg")
    assert zm["status"] == o["status"] == "converged"
    assert abs(zm["iterations"] - o["iterations"]) <= 1
    check_history(zm, o)
    assert abs(zm["rel_res_true"] - o["rel_res_true"]) <= 1e-12
    np.testing.assert_allclose(zm["x"], xt, atol=1e-8)
    check_history(zm, plain, rtol=1e-12)


def test_cg_zmarch_fp32_stream_with_restarts(torch):
    """The z-marching pass A in the FP32-stream form (binary32 p and s in
    HBM, binary64 values in LDS) reaches 1e-10 through restarts from x."""
    from paper_1706_05988_amd import pcg as P
    p = problems.poisson3d(40, seed=4)
    g = gpu_solve(torch, p, "cg", fp32=True, rtol=1e-10, max_iter=4000, replace_max=10, hist=False,
                  variant=P.PCG_VAR_SET | P.PCG_VAR_CG_ZMARCH)
    assert g["status"] == "converged" and g["rel_res_true"] <= 1e-10
    assert g["replacements"] >= 1


# ---------------------------------------------------------------- CSR

@pytest.mark.parametrize("method", METHODS)
def test_csr_anisotropic_jacobi(torch, method):
    p = problems.anisotropic_csr(48, seed=5)
    p.rtol, p.max_iter = 1e-10, 5000
    g = gpu_solve(torch, p, method, true_residual_check=False)
    o = oracle_solve(p, method)
    assert g["status"] == o["status"]
    assert abs(g["iterations"] - o["iterations"]) <= 2
    check_history(g, o)
    assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12


@pytest.mark.parametrize("method", ["cg", "pipe_shift"])
def test_csr_banded(torch, method):
    p = problems.banded_csr(5003, seed=3)
    p.rtol = 1e-10
    g = gpu_solve(torch, p, method, true_residual_check=False)
    o = oracle_solve(p, method)
    assert g["status"] == o["status"] == "converged"
    check_history(g, o)
    assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12
    if method == "pipe_shift":
        # rows of 4 to 40 entries: the built-in choice is the sorted copy,
        # with its own shape of 4 unknowns per thread
        assert g["info"]["csr_form_name"] == "sell_sorted" and g["info"]["ept"] == 4


def test_csr_default_sigma_gershgorin(torch):
    """sigma = NaN picks the Gershgorin midpoint of spec(M^-1 A): 1 for a
    Jacobi-scaled row-diagonally-dominant matrix (discs centred at 1)."""
    p = problems.banded_csr(2000, seed=1)
    g = gpu_solve(torch, p, "pipe_shift", sigma=math.nan)
    A = problems.to_scipy(p.op)
    d = A.diagonal()
    R = np.asarray(abs(A).sum(axis=1)).ravel() - d
    lo, hi = max(0.0, ((d - R) / d).min()), ((d + R) / d).max()
    assert g["sigma"] == pytest.approx(0.5 * (lo + hi), rel=1e-12)
    assert g["status"] == "converged"


# ---------------------------------------------------------------- FP32-stream form

@pytest.mark.parametrize("method", ["cg", "pipe_shift"])
def test_fp32_stream_attainable_accuracy(torch, method):
    """FP32-stream form lands within 10x of the oracle's attainable accuracy
    in the same form (binary32 storage emulation, same sigma)."""
    p = problems.poisson2d_manufactured(64)
    g = gpu_solve(torch, p, method, fp32=True, rtol=1e-30, max_iter=400, true_residual_check=False)
    o = oracle_solve(p, method, fp32=True, rtol=1e-30, max_iter=400, ignore_breakdown=True)
    assert g["rel_res_true"] <= 10 * o["rel_res_true"]
    # early history agrees to binary32 resolution
    np.testing.assert_allclose(g["res"][:15], o["res"][:15], rtol=1e-4)


@pytest.mark.parametrize("method", ["cg", "pipe_shift"])
def test_fp32_stream_with_restarts_reaches_fp64_tolerance(torch, method):
    """x and b stay binary64; restarting from x when the explicit residual
    misses the tolerance reaches 1e-10 in the FP32-stream form."""
    p = problems.poisson3d(40, seed=2)
    g = gpu_solve(torch, p, method, fp32=True, rtol=1e-10, max_iter=4000, replace_max=10, hist=False)
    assert g["status"] == "converged"
    assert g["replacements"] >= 1
    assert g["rel_res_true"] <= 1e-10


def test_fp32_stream_csr(torch):
    p = problems.anisotropic_csr(48, seed=5)
    g = gpu_solve(torch, p, "pipe_shift", fp32=True, rtol=1e-30, max_iter=600, true_residual_check=False)
    o = oracle_solve(p, "pipe_shift", fp32=True, rtol=1e-30, max_iter=600, ignore_breakdown=True)
    assert g["rel_res_true"] <= 10 * o["rel_res_true"]


def test_fp32_stream_refinement_reaches_fp64_oracle_attainable_csr(torch):
    """The C3 recipe at 96^2 (anisotropic CSR, Jacobi, sigma = 1): the
    FP32-stream form alone stalls near binary32 accuracy, but restarting
    from the binary64 x whenever the binary64 explicit residual misses the
    tolerance (iterative refinement) ends within 10x of the attainable
    accuracy of the oracle's all-binary64 run (its explicit residual after it
    has stagnated)."""
    p = problems.anisotropic_csr(96, seed=3)
    o = oracle_solve(p, "pipe_shift", sigma=1.0, rtol=1e-30, max_iter=4000, ignore_breakdown=True)
    level = o["rel_res_true"]
    assert level < 1e-13
    alone = gpu_solve(torch, p, "pipe_shift", fp32=True, sigma=1.0, rtol=1e-30, max_iter=4000,
                      true_residual_check=False, hist=False)
    assert alone["rel_res_true"] > 100 * level  # binary32 storage alone cannot get there
    g = gpu_solve(torch, p, "pipe_shift", fp32=True, sigma=1.0, rtol=5 * level, max_iter=40000, replace_max=40,
                  hist=False)
    assert g["status"] == "converged", (g["status"], g["rel_res_true"], level)
    assert g["replacements"] >= 1
    assert g["rel_res_true"] <= 10 * level, (g["rel_res_true"], level)


# ---------------------------------------------------------------- identities, determinism

def test_shift_zero_equals_pipe_bitwise_on_gpu(torch):
    p = problems.poisson3d(30, seed=1)
    a = gpu_solve(torch, p, "pipe", max_iter=80)
    b = gpu_solve(torch, p, "pipe_shift", sigma=0.0, max_iter=80)
    assert np.array_equal(a["x"], b["x"])
    assert np.array_equal(a["res"], b["res"], equal_nan=True)


@pytest.mark.parametrize("method", METHODS)
def test_deterministic_across_runs_graph_and_K(torch, method):
    p = problems.poisson3d(33, seed=4)
    base = gpu_solve(torch, p, method, max_iter=120, rtol=1e-30)
    again = gpu_solve(torch, p, method, max_iter=120, rtol=1e-30)
    nograph = gpu_solve(torch, p, method, max_iter=120, rtol=1e-30, use_graph=False)
    k6 = gpu_solve(torch, p, method, max_iter=120, rtol=1e-30, iters_per_launch=6)
    for other in (again, nograph, k6):
        assert np.array_equal(base["x"], other["x"])
        assert np.array_equal(base["res"], other["res"], equal_nan=True)


# ---------------------------------------------------------------- edge cases

@pytest.mark.parametrize("shape", [(1, 1), (2, 1), (1, 7), (3, 5)])
@pytest.mark.parametrize("method", METHODS)
def test_tiny_grids(torch, method, shape):
    op = problems.stencil2d(*shape)
    b = np.arange(1, op.n + 1, dtype=np.float64)
    p = problems.Problem("tiny", op, b, np.zeros(op.n), None, sigma=4.0, rtol=1e-12, max_iter=50)
    g = gpu_solve(torch, p, method)
    o = oracle_solve(p, method)
    assert g["status"] == "converged"
    xs = np.linalg.solve(problems.to_scipy(op).toarray(), b)
    np.testing.assert_allclose(g["x"], xs, rtol=1e-11)
    assert abs(g["iterations"] - o["iterations"]) <= 1


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("n", [10 ** 6, 2 * 10 ** 6])
def test_builtin_sorted_copy_takes_its_shape(torch, n, fp32):
    """Banded operators of 1e6 and 2e6 rows: set-up keeps the sorted copy and
    the passes run at that copy's built-in shape and grid: binary64 blocks of
    128, four per CU, six beyond 1.5e6 rows when the values are stored as
    binary32 (four with binary64 values); FP32-stream blocks of 256, two per
    CU up to 1.5e6 rows, three beyond."""
    p = problems.banded_csr(n, seed=2)
    cases = [(p, 32)]
    if not fp32 and n > 1500000:
        # the same pattern with values that are not binary32 numbers
        op = problems.csr_operator(p.op.row_ptr, p.op.col, p.op.val / 3.0)
        cases.append((problems.Problem("banded_thirds", op, p.b / 3.0, p.x0, p.x_true, jacobi=True, sigma=1.0), 64))
    for q, vbits in cases:
        g = gpu_solve(torch, q, "pipe_shift", fp32=fp32, max_iter=3, rtol=1e-30, true_residual_check=False,
                      hist=False)
        info = g["info"]
        assert info["csr_form_name"] == "sell_sorted" and info["csr_col_bits"] == 16
        assert info["csr_val_bits"] == (32 if fp32 else vbits)
        if fp32:
            block, per_cu = 256, (2 if n <= 1500000 else 3)
        else:
            block, per_cu = 128, (6 if n > 1500000 and vbits == 32 else 4)
        assert (info["block"], info["ept"]) == (block, 4)
        assert info["ntiles"] == -(-q.op.n // (block * 4))
        assert info["grid"] == min(per_cu * 256, info["ntiles"] & ~7), (q.name, info)


@pytest.mark.parametrize("n", [1, 2, 7, 65, 257])
@pytest.mark.parametrize("fp32", [False, True])
def test_tiny_csr_operators(torch, n, fp32):
    """Banded random CSR operators of a handful of rows (one ragged tile, a
    single partial slice; the built-in choice puts them on a sliced-ELL
    copy): p-CG-sh reaches the dense solution and follows the oracle."""
    p = problems.banded_csr(n, seed=n)
    g = gpu_solve(torch, p, "pipe_shift", fp32=fp32, rtol=1e-12 if not fp32 else 1e-6, max_iter=400,
                  replace_max=8)
    o = oracle_solve(p, "pipe_shift", fp32=fp32, rtol=1e-12 if not fp32 else 1e-6, max_iter=400)
    assert g["status"] == "converged", g["status"]
    assert g["info"]["csr_form_name"] in ("csr", "sell", "sell_sorted")
    xs = np.linalg.solve(problems.to_scipy(p.op).toarray(), p.b)
    np.testing.assert_allclose(g["x"], xs, rtol=0, atol=(1e-9 if not fp32 else 1e-4) * np.abs(xs).max())
    if not fp32:
        # these converge by 11 orders in ~30 iterations: compare the history
        # down to 1e-8, below which it is rounding noise relative to ||b||
        above = np.nonzero(o["res"] < 1e-8)[0]
        check_history(g, o, upto=int(above[0]) if above.size else 50)


def test_zero_iterations_and_exact_start(torch):
    p = problems.poisson2d_manufactured(20)
    g = gpu_solve(torch, p, "pipe_shift", max_iter=0)
    assert g["status"] == "max_iter" and g["iterations"] == 0
    assert np.array_equal(g["x"], p.x0)
    g = gpu_solve(torch, p, "pipe_shift", x0=p.x_true.copy())
    assert g["status"] == "converged" and g["iterations"] == 0


@pytest.mark.parametrize("method", METHODS + ["pipe_rr", "pipe_var"])
@pytest.mark.parametrize("fp32,jacobi", [(False, False), (True, True)])
def test_zero_rhs_converges_at_once(torch, method, fp32, jacobi):
    """b = 0 with x0 = 0: r_0 = 0 meets the stop test before any iteration
    (||r_0|| <= rtol ||b|| = 0), x stays 0 and the residuals are reported
    unnormalised (0, not 0/0)."""
    op = problems.stencil3d(9, 7, 5)
    p = problems.Problem("zero_rhs", op, np.zeros(op.n), np.zeros(op.n), np.zeros(op.n), jacobi=jacobi,
                         sigma=1.0 if jacobi else 6.0, rtol=1e-10, max_iter=100)
    kw = dict(sigma_schedule=[p.sigma, p.sigma]) if method == "pipe_var" else {}
    g = gpu_solve(torch, p, method, fp32=fp32, sigma=p.sigma if method != "cg" else 0.0, **kw)
    assert g["status"] == "converged" and g["iterations"] == 0
    assert g["rel_res_true"] == 0.0 and g["rel_res_recursive"] == 0.0
    assert not np.any(g["x"])


def test_nonfinite_rhs_is_an_error(torch):
    from paper_1706_05988_amd import pcg as P
    p = problems.poisson2d_manufactured(20)
    p.b = p.b.copy()
    p.b[7] = np.inf
    with pytest.raises(P.PcgError) as ei:
        gpu_solve(torch, p, "pipe_shift")
    assert ei.value.status == P.PCG_ERR_NONFINITE


def test_breakdown_on_indefinite_csr(torch):
    n = 40
    vals = np.linspace(-1.0, 3.0, n)
    vals[np.abs(vals) < 1e-3] = 0.5
    op = problems.csr_operator(np.arange(n + 1), np.arange(n, dtype=np.int32), vals)
    p = problems.Problem("indef", op, np.ones(n), np.zeros(n), None, sigma=1.0, rtol=1e-12, max_iter=100)
    for m in METHODS:
        assert gpu_solve(torch, p, m)["status"] == "breakdown"


def test_invalid_csr_rejected_before_any_pass(torch):
    from paper_1706_05988_amd import pcg as P
    n = 10
    op = problems.csr_operator(np.arange(n + 1), np.arange(n, dtype=np.int32), np.ones(n))
    op.col = op.col.copy()
    op.col[3] = 99  # out of range
    opt = P.make_options(method="pipe_shift", sigma=1.0)
    with pytest.raises(P.PcgError) as ei:
        P.Solver(op, opt)
    assert ei.value.status == P.PCG_ERR_INVALID


def test_workspace_too_small_rejected(torch):
    from paper_1706_05988_amd import pcg as P
    op = problems.stencil2d(30)
    dev = P.DeviceOperator(op)
    opt = P.make_options()
    need = P.pcg_workspace_size(dev.struct, opt)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PcgError) as ei:
        P.pcg_create(dev.struct, opt, ws.data_ptr(), need - 256, 0)
    assert ei.value.status == P.PCG_ERR_INVALID


# ---------------------------------------------------------------- full size (configs 2, 3)

def sample_index(n, nxy, nx, seed):
    """Sampled unknowns plus the first and last tiles and the first and last
    grid planes' opening rows."""
    return np.unique(np.concatenate([
        np.random.default_rng(seed).integers(0, n, 4000), np.arange(0, 1024), np.arange(n - 1024, n),
        np.arange(nxy, nxy + nx), np.arange(n - nxy, n - nxy + nx)]))


@pytest.mark.parametrize("method", METHODS)
def test_config2_full_size_fifty_iterations(torch, method):
    """3-D Poisson 256^3 (16.8M unknowns), Jacobi, sigma = 1, FP64, in the
    benchmark's launch configuration: sqrt(rho_i)/||b||, alpha_i and beta_i
    match the oracle's to 1e-10 over the first 50 iterations, and x after
    them matches at sampled unknowns, the first and last tiles and planes
    included."""
    p = problems.poisson3d(256, seed=0)
    o = oracle_solve(p, method, max_iter=50, rtol=1e-30, threads=oracle.max_threads())
    print(f"[parity] 256^3 {method}: oracle 50 iterations done", flush=True)
    g = gpu_solve(torch, p, method, max_iter=50, rtol=1e-30, true_residual_check=False)
    assert g["iterations"] == o["iterations"] == 50
    check_history(g, o, upto=50)
    idx = sample_index(p.op.n, 256 * 256, 256, 2)
    np.testing.assert_allclose(g["x"][idx], o["x"][idx], rtol=1e-10, atol=1e-12 * np.abs(o["x"]).max())


@pytest.mark.parametrize("method", METHODS)
def test_config2_full_solve_final_residual(torch, method):
    """The complete 256^3 solve to 1e-10 with the explicit-residual check and
    restarts from x (the benchmark's options), GPU against the oracle with the
    same restart rule: the same iteration count (within one), and final
    explicit residuals ||b - A x||/||b|| within 1e-12 (p-CG: within a 10x
    band, its attainable level being rounding-determined)."""
    p = problems.poisson3d(256, seed=0)
    o = oracle_solve(p, method, replace_max=4, record=False, threads=oracle.max_threads())
    print(f"[parity] 256^3 {method}: oracle full solve {o['iterations']} iterations, "
          f"true residual {o['rel_res_true']:.3e}", flush=True)
    g = gpu_solve(torch, p, method, hist=False, replace_max=4)
    assert g["status"] == o["status"] == "converged", (g["status"], o["status"])
    assert abs(g["iterations"] - o["iterations"]) <= 1
    assert g["rel_res_true"] <= 1e-10
    if method == "pipe":
        assert g["rel_res_true"] <= 10 * o["rel_res_true"] and o["rel_res_true"] <= 10 * g["rel_res_true"]
    else:
        assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12
    assert np.abs(g["x"] - p.x_true).max() < 1e-6


def test_largest_grid_sampled(torch):
    """3-D Poisson 512^3 (134M unknowns; the solver's workspace is above
    2^32 bytes, so every byte offset past 4 GiB is exercised), Jacobi,
    sigma = 1, FP64: the first three iterations' residual history and
    alphas match the oracle, and x after them matches at sampled unknowns,
    the last tiles and planes included."""
    from paper_1706_05988_amd import pcg as P
    p = problems.poisson3d(512, seed=0)
    o = oracle_solve(p, "pipe_shift", max_iter=3, rtol=1e-30)
    opt = P.make_options(method="pipe_shift", jacobi=True, sigma=p.sigma, rtol=1e-30, max_iter=3,
                         true_residual_check=False, history_cap=5)
    s = P.Solver(p.op, opt)
    assert s.nbytes > (1 << 32)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros_like(b)
    g = s.solve(b, x)
    torch.cuda.synchronize()
    s.close()
    np.testing.assert_allclose(g["res"][:4], o["res"][:4], rtol=1e-12)
    np.testing.assert_allclose(g["alpha"][:3], o["alpha"][:3], rtol=1e-12)
    n, nxy = p.op.n, 512 * 512
    idx = np.concatenate([np.random.default_rng(1).integers(0, n, 2000), np.arange(n - 1024, n),
                          np.arange(n - nxy, n - nxy + 512), np.arange(0, 512)])
    xg = x.cpu().numpy()
    np.testing.assert_allclose(xg[idx], o["x"][idx], rtol=1e-11, atol=1e-14)
    del b, x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fp32", [False, True])
def test_config3_full_size_sampled(torch, fp32):
    """2-D anisotropic diffusion 1024^2 CSR (5.24M nonzeros), Jacobi, sigma = 1,
    in the report's launch configuration, against the oracle in the same
    storage form on the same input.  Binary64: the residual history, alpha
    and beta to 1e-10 over the first 50 iterations and x after them at
    sampled unknowns (the last rows included).  FP32-stream: the first 10
    iterations at binary32 resolution (1e-4; later iterates of the two sides
    part at the binary32 rounding of the stored vectors)."""
    p = problems.anisotropic_csr(1024, seed=0)
    its = 10 if fp32 else 50
    kw = dict(fp32=fp32, sigma=1.0, max_iter=its, rtol=1e-30)
    o = oracle_solve(p, "pipe_shift", threads=oracle.max_threads(), **kw)
    g = gpu_solve(torch, p, "pipe_shift", true_residual_check=False, **kw)
    tol = 1e-4 if fp32 else 1e-10
    if fp32:
        np.testing.assert_allclose(g["res"][: its + 1], o["res"][: its + 1], rtol=tol)
    else:
        assert g["iterations"] == o["iterations"] == its
        check_history(g, o, upto=its)
    n = p.op.n
    idx = np.unique(np.concatenate([np.random.default_rng(1).integers(0, n, 4000), np.arange(n - 2048, n)]))
    np.testing.assert_allclose(g["x"][idx], o["x"][idx], rtol=10 * tol, atol=10 * tol * np.abs(o["x"]).max())


# ---------------------------------------------------------------- kernel variants

VARIANTS = {
    "ept1": 0x01 | 0x10,
    "ept1_nt_xcd": 0x01 | 0x10 | 0x02 | 0x04,
    "ept2": 0x01,
    "ept2_nt_xcd": 0x01 | 0x02 | 0x04,
    "ept4": 0x01 | 0x20,
    "ept4_nt_xcd": 0x01 | 0x20 | 0x02 | 0x04,
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("method", ["cg", "pipe_shift"])
def test_kernel_variants_match_oracle(torch, variant, fp32, method):
    """Every kernel variant follows the oracle (binary64: 1e-10 over 50
    iterations; FP32-stream: binary32 resolution over 15)."""
    p = problems.poisson3d(48, seed=9)
    g = gpu_solve(torch, p, method, fp32=fp32, max_iter=60, rtol=1e-30, true_residual_check=False,
                  variant=VARIANTS[variant], grid_blocks=64)
    o = oracle_solve(p, method, fp32=fp32, max_iter=60, rtol=1e-30)
    if fp32:
        np.testing.assert_allclose(g["res"][:16], o["res"][:16], rtol=1e-4)
    else:
        check_history(g, o)


@pytest.mark.parametrize("n", [511, 512, 513, 1025])
def test_blocked_layout_tile_edges(torch, n):
    """Unknown counts around the 512-unknown tile of the blocked layout."""
    op = problems.Operator("2d5", n, n, 1, 1, 2.0, -1.0, 0.0)  # 1-D Laplacian
    b = np.random.default_rng(n).uniform(-1, 1, n)
    p = problems.Problem("edge", op, b, np.zeros(n), None, sigma=2.0, rtol=1e-12, max_iter=3000)
    for m in METHODS:
        g = gpu_solve(torch, p, m, max_iter=60, rtol=1e-30, true_residual_check=False)
        o = oracle_solve(p, m, max_iter=60, rtol=1e-30)
        check_history(g, o)


# ---------------------------------------------------------------- C3 recipe, every shift

@pytest.mark.parametrize("sigma", [0.0, 0.02, 1.0, 2.0])
@pytest.mark.parametrize("fp32", [False, True])
def test_anisotropic_csr_attainable_accuracy_per_shift(torch, sigma, fp32):
    """The anisotropic-diffusion CSR recipe (reduced to 64^2, Jacobi) run to
    a fixed iteration cap for shifts 0, near lambda_min, the midpoint and the
    lambda_max bound: the explicit residual the GPU attains matches the
    oracle's in the same storage form.  Where the oracle stops at a breakdown
    (its iteration is set by rounding), the GPU's level lies between the
    oracle's level at that breakdown and the level it reaches running on."""
    p = problems.anisotropic_csr(64, seed=0)
    kw = dict(fp32=fp32, sigma=sigma, rtol=1e-30, max_iter=1500)
    g = gpu_solve(torch, p, "pipe_shift", true_residual_check=False, hist=False, **kw)
    o = oracle_solve(p, "pipe_shift", **kw)
    if o["status"] == "max_iter":
        assert g["status"] == "max_iter"
        assert 0.1 * o["rel_res_true"] - 1e-14 <= g["rel_res_true"] <= 10 * o["rel_res_true"] + 1e-14
    else:
        assert o["status"] == "breakdown"
        on = oracle_solve(p, "pipe_shift", ignore_breakdown=True, **kw)
        assert g["status"] in ("breakdown", "max_iter")
        lo, hi = sorted((o["rel_res_true"], on["rel_res_true"]))
        assert lo / 100 <= g["rel_res_true"] <= hi * 100


# ---------------------------------------------------------------- Alg. 4: variable shift

def _sched(count, seed, lo, hi):
    return np.random.default_rng(seed).uniform(lo, hi, count)


@pytest.mark.parametrize("jacobi", [False, True])
def test_variable_shift_constant_schedule_matches_alg3_on_gpu(torch, jacobi):
    """A constant schedule makes every correction term zero: the Alg. 4 pass
    gives Alg. 3's iterates (to the last bits that FMA contraction choices
    can move: the compiler may fuse either product of a sum of two)."""
    p = problems.poisson3d(30, seed=1, jacobi=jacobi)
    sig = 1.0 if jacobi else 6.0
    a = gpu_solve(torch, p, "pipe_shift", sigma=sig, max_iter=120, true_residual_check=False)
    v = gpu_solve(torch, p, "pipe_var", sigma_schedule=[sig], max_iter=120, true_residual_check=False)
    assert v["iterations"] == a["iterations"]
    k = a["iterations"]
    np.testing.assert_allclose(v["res"][: k + 1], a["res"][: k + 1], rtol=1e-12)
    np.testing.assert_allclose(v["x"], a["x"], rtol=1e-10, atol=1e-14)
    assert v["sigma"] == sig


@pytest.mark.parametrize("prob", ["2d_none", "3d_jacobi_ragged", "csr_jacobi"])
def test_variable_shift_history_and_solution(torch, prob):
    """Alg. 4 with a shift that changes every iteration: GPU histories follow
    the oracle's (same schedule) and the solve reaches the oracle's residual."""
    if prob == "2d_none":
        p = problems.poisson2d_manufactured(100)
        sched = _sched(300, 1, 2.0, 6.0)
    elif prob == "3d_jacobi_ragged":
        op = problems.stencil3d(37, 41, 43)
        xt = np.random.default_rng(11).uniform(-1, 1, op.n)
        p = problems.Problem("ragged3d", op, problems.to_scipy(op) @ xt, np.zeros(op.n), xt, jacobi=True,
                             sigma=1.0, rtol=1e-10, max_iter=2000)
        sched = _sched(300, 2, 0.2, 1.8)
    else:
        p = problems.anisotropic_csr(48, seed=5)
        p.rtol, p.max_iter = 1e-10, 5000
        sched = _sched(50, 3, 0.5, 1.5)
    g = gpu_solve(torch, p, "pipe_var", sigma_schedule=sched, true_residual_check=False)
    o = oracle_solve(p, "pipe_var", sigma_schedule=sched)
    assert g["status"] == o["status"] == "converged"
    assert abs(g["iterations"] - o["iterations"]) <= 2
    check_history(g, o)
    assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12
    assert g["sigma"] == sched[min(g["iterations"], len(sched) - 1)]


def test_variable_shift_fp32_stream(torch):
    """FP32-stream form of Alg. 4: early history to binary32 resolution and the
    attainable accuracy within 10x of the oracle's emulation of that form."""
    p = problems.poisson2d_manufactured(64)
    sched = _sched(40, 4, 2.0, 6.0)
    kw = dict(fp32=True, rtol=1e-30, max_iter=400, sigma_schedule=sched)
    g = gpu_solve(torch, p, "pipe_var", true_residual_check=False, **kw)
    o = oracle_solve(p, "pipe_var", ignore_breakdown=True, **kw)
    np.testing.assert_allclose(g["res"][:15], o["res"][:15], rtol=1e-4)
    assert g["rel_res_true"] <= 10 * o["rel_res_true"]


def test_variable_shift_restart_uses_sigma_prev(torch):
    """A restart from x at iteration i rebuilds w_i with sigma_{i-1}: the
    FP32-stream solve with restarts reaches the binary64 tolerance."""
    p = problems.poisson3d(40, seed=2)
    sched = _sched(500, 5, 0.5, 1.5)
    g = gpu_solve(torch, p, "pipe_var", fp32=True, rtol=1e-10, max_iter=4000, replace_max=10, hist=False,
                  sigma_schedule=sched)
    assert g["status"] == "converged"
    assert g["replacements"] >= 1
    assert g["rel_res_true"] <= 1e-10


# ---------------------------------------------------------------- shift selection from a GPU history

def test_select_shift_from_gpu_recorded_history(torch):
    """Section 5.1's workflow: record alpha / beta on the device (500
    iterations of lapl200), then pick sigma from psi_499 on a grid.  The
    library's psi values equal the oracle's on the same coefficients and the
    choice is Table 1's sigma* = 4.00."""
    import oracle.psi as psi_mod
    from paper_1706_05988_amd import pcg as P
    p = problems.lapl200()
    g = gpu_solve(torch, p, "cg", rtol=1e-30, max_iter=500, true_residual_check=False)
    assert g["iterations"] == 500
    a, b = g["alpha"][:500], g["beta"][:500]
    grid = np.arange(0.0, 8.01, 0.5)
    s, vals = P.pcg_select_shift(a, b, 499, grid, slack=2.0)
    so, ovals = psi_mod.select_shift(a, b, grid, 499, slack=2.0)
    np.testing.assert_allclose(vals, ovals, rtol=1e-9)
    assert s == so == 4.0


# ---------------------------------------------------------------- p-CG-rr (residual replacement)

TAU64 = 2.0 ** (-53 / 3)
TAU32 = 2.0 ** -8


@pytest.mark.parametrize("prob", ["lapl200", "3d_jacobi", "csr_jacobi"])
def test_pcg_rr_history_replacements_and_accuracy(torch, prob):
    """p-CG-rr on the GPU follows the oracle: same replacement decisions
    (count), the same early history, the final explicit residual at the
    oracle's level (both near CG's, far below p-CG's where it stagnates)."""
    if prob == "lapl200":
        p = problems.lapl200()
        kw = dict(rtol=1e-30, max_iter=500)
    elif prob == "3d_jacobi":
        op = problems.stencil3d(37, 41, 43)
        xt = np.random.default_rng(11).uniform(-1, 1, op.n)
        p = problems.Problem("ragged3d", op, problems.to_scipy(op) @ xt, np.zeros(op.n), xt, jacobi=True,
                             sigma=1.0, rtol=1e-30, max_iter=400)
        kw = dict(rtol=1e-30, max_iter=400)
    else:
        p = problems.anisotropic_csr(48, seed=5)
        kw = dict(rtol=1e-30, max_iter=800)
    g = gpu_solve(torch, p, "pipe_rr", true_residual_check=False, rr_tau=TAU64, **kw)
    o = oracle_solve(p, "pipe_rr", rr_tau=TAU64, **kw)
    # after stagnation a breakdown (delta <= 0) comes at a rounding-determined
    # iteration; before it both run to the cap
    assert g["status"] in ("max_iter", "breakdown") and o["status"] in ("max_iter", "breakdown")
    if g["status"] == o["status"] == "max_iter":
        assert g["iterations"] == o["iterations"]
    assert g["replacements"] >= 1
    assert abs(g["replacements"] - o["replacements"]) <= 1
    check_history(g, o)
    assert g["rel_res_true"] <= max(10 * o["rel_res_true"], 1e-14)


def test_pcg_rr_no_replacement_equals_pipe(torch):
    p = problems.poisson3d(30, seed=1)
    a = gpu_solve(torch, p, "pipe", max_iter=150, true_residual_check=False)
    b = gpu_solve(torch, p, "pipe_rr", max_iter=150, true_residual_check=False, rr_tau=1e300)
    assert b["replacements"] == 0 and a["iterations"] == b["iterations"]
    k = a["iterations"]
    np.testing.assert_allclose(b["res"][: k + 1], a["res"][: k + 1], rtol=1e-12)


@pytest.mark.parametrize("method", ["pipe", "pipe_shift", "pipe_var"])
def test_x_after_each_stop_parity_matches_oracle(torch, method):
    """The fused pass updates x every other iteration and the host completes
    x when a solve stops after a skipping pass: x after 1..8 iterations (both
    parities) matches the oracle's x_k and the every-iteration update of the
    p-CG-rr pass (no replacement) to rounding."""
    p = problems.poisson3d(23, seed=5)
    kw = {}
    if method == "pipe_var":
        kw["sigma_schedule"] = [0.5, 1.0, 0.8, 1.2, 0.9, 1.1, 1.0]
    for k in range(1, 9):
        g = gpu_solve(torch, p, method, max_iter=k, rtol=1e-30, true_residual_check=False, hist=False, **kw)
        assert g["status"] == "max_iter" and g["iterations"] == k
        o = oracle_solve(p, method, max_iter=k, rtol=1e-30, **kw)
        # the dot products are summed in another order: entries near zero
        # differ at rounding level relative to |x|; a missing or doubled
        # alpha p term would differ by |alpha p|, many orders larger
        np.testing.assert_allclose(g["x"], o["x"], rtol=1e-11, atol=1e-13 * np.abs(o["x"]).max(),
                                   err_msg=f"{method} k={k}")
        if method == "pipe":
            e = gpu_solve(torch, p, "pipe_rr", max_iter=k, rtol=1e-30, true_residual_check=False, hist=False,
                          rr_tau=1e300)
            np.testing.assert_allclose(g["x"], e["x"], rtol=1e-13, atol=1e-15 * np.abs(e["x"]).max())


def test_pcg_rr_replacement_history_matches_oracle_exactly_at_the_reset(torch):
    """At the replacement iteration the recorded residual is the explicit one:
    GPU and oracle agree there too (the dot products were formed again)."""
    p = problems.lapl200()
    g = gpu_solve(torch, p, "pipe_rr", true_residual_check=False, rr_tau=TAU64, rtol=1e-30, max_iter=300)
    o = oracle_solve(p, "pipe_rr", rr_tau=TAU64, rtol=1e-30, max_iter=300, record_true=True)
    rel = np.abs(o["res"] - o["true"]) / o["true"]
    hits = [i for i in range(1, 300) if rel[i] <= 1e-15 and rel[i - 1] >= 1e-9]
    assert hits
    for i in hits:
        assert g["res"][i] == pytest.approx(o["res"][i], rel=1e-6)


def test_pcg_rr_fp32_stream_refines_to_binary64_level(torch):
    """FP32-stream p-CG-rr: replacements recompute r from the binary64 x, so
    the attainable accuracy (the lowest level reached; the recursive residual
    tracks the explicit one under replacement) falls far below binary32 and
    lands within 10x of the oracle's in the same form.  Near the end a
    breakdown can stop either run at a rounding-determined iteration."""
    p = problems.poisson2d_manufactured(64)
    kw = dict(fp32=True, rtol=1e-30, max_iter=400, rr_tau=TAU32)
    g = gpu_solve(torch, p, "pipe_rr", true_residual_check=False, **kw)
    o = oracle_solve(p, "pipe_rr", record_true=True, **kw)
    assert g["replacements"] >= 1
    g_best = np.nanmin(g["res"][: g["iterations"] + 1])
    o_best = np.nanmin(o["true"][: o["iterations"] + 1])
    assert g_best < 1e-11
    assert g_best <= 10 * o_best


# ---------------------------------------------------------------- autotuner

def test_autotuner_shape_solves_like_the_oracle_and_caches(torch, tmp_path, monkeypatch):
    """pcg_tune picks one of its candidate shapes; the solve with it follows
    the oracle; with PCG_TUNE_CACHE set the result is stored and a second call
    returns it without measuring."""
    from paper_1706_05988_amd import pcg as P
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PCG_TUNE_CACHE", str(cache))
    p = problems.poisson3d(48, seed=9)
    base = P.make_options(method="pipe_shift", jacobi=True, sigma=1.0, rtol=1e-30, max_iter=60,
                          true_residual_check=False, history_cap=62)
    tuned, us = P.tune(p.op, base)
    assert us > 0
    assert tuned.block_size in (0, 128, 256) and tuned.grid_blocks >= 0
    lines = cache.read_text().strip().split("\n")
    assert len(lines) == 1
    tuned2, us2 = P.tune(p.op, base)
    assert (tuned2.variant, tuned2.block_size, tuned2.grid_blocks) == (tuned.variant, tuned.block_size,
                                                                        tuned.grid_blocks)
    assert us2 == pytest.approx(us, rel=1e-3)
    assert len(cache.read_text().strip().split("\n")) == 1
    s = P.Solver(p.op, tuned)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros_like(b)
    g = s.solve(b, x)
    s.close()
    o = oracle_solve(p, "pipe_shift", sigma=1.0, rtol=1e-30, max_iter=60)
    check_history(g, o)


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("method", ["pipe", "pipe_shift"])
def test_csr_sliced_ell_operand_gives_the_csr_bits(torch, method, fp32):
    """The fused pass on the sliced-ELL copy of a CSR operator forms every
    row's products and sums in CSR storage order, so at one launch shape a
    solve gives the same bits with either operand form -- on the
    anisotropic operator (rows of 3 to 5 entries, a ragged last slice) and
    on a 3-D 7-point Laplacian assembled as CSR (rows of 4 to 7 entries,
    Jacobi from its diagonal, a last slice of 4 rows), both with 16-bit
    row-relative columns and binary32-stored values, and on a 2-D Laplacian
    scaled by 1/3 with a few couplings 40000 columns away (32-bit columns,
    binary64 values)."""
    from paper_1706_05988_amd import pcg as P
    A = problems.to_scipy(problems.stencil3d(20, 17, 13)).tocsr()
    A.sort_indices()
    op3 = problems.csr_operator(A.indptr, A.indices, A.data)
    xt = np.random.default_rng(8).uniform(-1, 1, op3.n)
    p3 = problems.Problem("lapl3d_csr", op3, A @ xt, np.zeros(op3.n), xt, jacobi=True, sigma=1.0)
    # a 2-D Laplacian scaled by 1/3, with a few couplings 40000 columns away:
    # 32-bit columns and (binary64) 64-bit values
    A6 = problems.to_scipy(problems.stencil2d(300, 300)).tolil()
    for i in (10, 20000, 45000):
        A6[i, i + 40000] = A6[i + 40000, i] = -0.5
        A6[i, i] += 0.5
        A6[i + 40000, i + 40000] += 0.5
    A6 = (A6.tocsr() / 3.0).tocsr()  # values that are not binary32 numbers
    A6.sort_indices()
    op6 = problems.csr_operator(A6.indptr, A6.indices, A6.data)
    xt6 = np.random.default_rng(12).uniform(-1, 1, op6.n)
    p6 = problems.Problem("lapl2d_far_csr", op6, A6 @ xt6, np.zeros(op6.n), xt6, jacobi=True, sigma=1.0)
    for p, bits, vbits in ((problems.anisotropic_csr(90, seed=4), 16, 32), (p3, 16, 32), (p6, 32, 64)):
        base = P.PCG_VAR_SET | P.PCG_VAR_NT | P.PCG_VAR_EPT1
        out = []
        for sell in (0, P.PCG_VAR_CSR_SELL):
            g = gpu_solve(torch, p, method, fp32=fp32, sigma=1.0 if method == "pipe_shift" else 0.0, max_iter=300,
                          rtol=1e-30, true_residual_check=False, variant=base | sell, block_size=256,
                          grid_blocks=64)
            out.append(g)
        a, b = out
        # the copy stores columns as 16-bit offsets from the row when every
        # entry lies within 2^15 of it, and binary64 values as binary32 when
        # they all are binary32 numbers
        assert b["info"]["csr_form_name"] == "sell" and b["info"]["csr_col_bits"] == bits, p.name
        assert b["info"]["csr_val_bits"] == (32 if fp32 else vbits), p.name
        assert a["iterations"] == b["iterations"]
        np.testing.assert_array_equal(a["res"], b["res"])
        np.testing.assert_array_equal(a["x"], b["x"])


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("shape", [(256, 4), (128, 2), (64, 4)])
def test_csr_sorted_sliced_ell_gives_the_csr_bits(torch, shape, fp32):
    """The sorted sliced-ELL copy orders each wave's rows by length and
    routes the products back to their rows through LDS; every row is still
    summed alone in CSR storage order, so at one launch shape a p-CG-sh
    solve gives the same bits as on the CSR arrays -- on banded random
    operators (rows of 4 to 40 entries, ragged last tile), the anisotropic
    operator and 3-D Laplacians assembled as CSR, with the tiles' operand
    columns staged in an LDS window and the columns stored as 16-bit window
    offsets, or gathered directly (planes 1600 columns apart), or a mix of
    the two with 32-bit columns (a banded operator with a few long-range
    couplings)."""
    from paper_1706_05988_amd import pcg as P
    block, ept = shape
    A = problems.to_scipy(problems.stencil3d(19, 17, 13)).tocsr()
    A.sort_indices()
    op3 = problems.csr_operator(A.indptr, A.indices, A.data)
    xt = np.random.default_rng(9).uniform(-1, 1, op3.n)
    p3 = problems.Problem("lapl3d_csr", op3, A @ xt, np.zeros(op3.n), xt, jacobi=True, sigma=1.0)
    # a 3-D Laplacian whose planes are 1600 columns apart: its tiles gather
    # from more columns than fit their LDS window, so they gather directly
    A4 = problems.to_scipy(problems.stencil3d(40, 40, 21)).tocsr()
    A4.sort_indices()
    op4 = problems.csr_operator(A4.indptr, A4.indices, A4.data)
    xt4 = np.random.default_rng(10).uniform(-1, 1, op4.n)
    p4 = problems.Problem("lapl3d_wide_csr", op4, A4 @ xt4, np.zeros(op4.n), xt4, jacobi=True, sigma=1.0)
    # a banded operator with a few long-range couplings: the tiles holding
    # them gather directly, the others from their windows (32-bit columns)
    B5 = problems.to_scipy(problems.banded_csr(20011, seed=6).op).tolil()
    for i in (300, 9000, 15000):
        B5[i, i + 4000] = B5[i + 4000, i] = -0.5
        B5[i, i] += 0.5
        B5[i + 4000, i + 4000] += 0.5
    B5 = B5.tocsr()
    B5.sort_indices()
    op5 = problems.csr_operator(B5.indptr, B5.indices, B5.data)
    xt5 = np.random.default_rng(11).uniform(-1, 1, op5.n)
    p5 = problems.Problem("banded_far_csr", op5, B5 @ xt5, np.zeros(op5.n), xt5, jacobi=True, sigma=1.0)
    for p in (problems.banded_csr(5003, seed=3), problems.banded_csr(20011, seed=5),
              problems.anisotropic_csr(90, seed=4), p3, p4, p5):
        base = P.PCG_VAR_SET | P.PCG_VAR_NT | (P.PCG_VAR_EPT4 if ept == 4 else 0)
        out = []
        for form in (0, P.PCG_VAR_CSR_SELL_SORTED):
            g = gpu_solve(torch, p, "pipe_shift", fp32=fp32, sigma=1.0, max_iter=200, rtol=1e-30,
                          true_residual_check=False, variant=base | form, block_size=block, grid_blocks=48)
            out.append(g)
        a, b = out
        # the copy's size from the sorting rule: each wave's ept x 64 rows of a
        # tile sorted by length cut into slices of 64 as wide as their longest
        lens = np.diff(np.asarray(p.op.row_ptr, dtype=np.int64))
        R = block * ept
        padded = np.zeros(-(-p.op.n // R) * R, np.int64)
        padded[:p.op.n] = lens
        groups = padded.reshape(-1, ept, block // 64, 64).transpose(0, 2, 1, 3).reshape(-1, ept * 64)
        want = 64 * int(np.sort(groups, axis=1)[:, ::-1].reshape(-1, 64).max(axis=1).sum())
        nnz = int(p.op.row_ptr[-1])
        fits = want <= nnz + nnz // 4 + 4096
        print(f"[sorted-sell] {p.name} n={p.op.n} block={block} ept={ept} fp32={fp32}: "
              f"{b['info']['csr_entries']} entries (rule: {want}) for nnz {nnz}", flush=True)
        assert a["info"]["csr_form_name"] == "csr"
        if not fits:  # beyond the reserved capacity: the CSR arrays
            assert b["info"]["csr_form_name"] == "csr"
            continue
        assert b["info"]["csr_form_name"] == "sell_sorted" and b["info"]["csr_entries"] == want
        assert (b["info"]["block"], b["info"]["ept"]) == (block, ept)
        # 16-bit window offsets when every tile's columns (its own rows
        # included) span at most 2048
        rp, cols = np.asarray(p.op.row_ptr, dtype=np.int64), np.asarray(p.op.col)
        spans = []
        for t in range(-(-p.op.n // R)):
            r0, r1 = t * R, min(p.op.n, (t + 1) * R)
            c = cols[rp[r0]:rp[r1]]
            spans.append(max(c.max(initial=r1 - 1), r1 - 1) - min(c.min(initial=r0), r0) + 1)
        windowed = np.array(spans) <= 2048
        assert b["info"]["csr_col_bits"] == (16 if windowed.all() else 32), (p.name, windowed.mean())
        assert b["info"]["csr_val_bits"] == 32  # binary32 numbers in either form
        assert a["iterations"] == b["iterations"]
        np.testing.assert_array_equal(a["res"], b["res"])
        np.testing.assert_array_equal(a["x"], b["x"])


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("form", ["sell", "sell_sorted"])
def test_csr_copies_serve_every_pass(torch, form, fp32):
    """The set-up passes (r_0 = b - A x_0, w_0 = A u_0), the explicit
    residual and the passes of every method read the sliced-ELL copy too,
    each row summed in CSR order: a p-CG-sh solve with the explicit-residual
    check at convergence (a restart from x when it misses the tolerance), an
    Alg. 4 solve, a CG solve, a p-CG-rr solve with residual replacements
    and the explicit residual of a caller's x give the same bits as on the
    CSR arrays, from a nonzero x_0."""
    from paper_1706_05988_amd import pcg as P
    flag, ept_flag, shape = ((P.PCG_VAR_CSR_SELL, P.PCG_VAR_EPT1, (256, 1)) if form == "sell"
                             else (P.PCG_VAR_CSR_SELL_SORTED, P.PCG_VAR_EPT4, (256, 4)))
    runs = [("pipe_shift", dict(sigma=1.0, true_residual_check=True, rtol=1e-9, max_iter=400)),
            ("pipe_var", dict(sigma=1.0, sigma_schedule=[1.0, 0.5, 1.0], rtol=1e-30, max_iter=120,
                              true_residual_check=False)),
            ("cg", dict(sigma=0.0, rtol=1e-30, max_iter=120, true_residual_check=False)),
            # thresholds that let every gap check (each 8 iterations) replace
            ("pipe_rr", dict(sigma=0.0, rtol=1e-30, max_iter=120, true_residual_check=False, rr_period=8,
                             rr_tau=1e-300, rr_floor=1e-300)),
            # the default thresholds over a longer run: the gap check's
            # rounding scale |A||x| + |b| decides with the measured gap
            ("pipe_rr", dict(sigma=0.0, rtol=1e-30, max_iter=600, true_residual_check=False))]
    # the in-place copy needs rows of even length (padding within a quarter);
    # the sorted copy takes the banded random rows of 4 to 40 entries
    A = problems.to_scipy(problems.stencil3d(20, 17, 13)).tocsr()
    A.sort_indices()
    op3 = problems.csr_operator(A.indptr, A.indices, A.data)
    xt = np.random.default_rng(8).uniform(-1, 1, op3.n)
    p3 = problems.Problem("lapl3d_csr", op3, A @ xt, np.zeros(op3.n), xt, jacobi=True, sigma=1.0)
    first = p3 if form == "sell" else problems.banded_csr(20011, seed=5)
    for p in (first, problems.anisotropic_csr(90, seed=4)):
        x0 = np.random.default_rng(13).uniform(-1, 1, p.op.n)
        xu = torch.from_numpy(np.random.default_rng(14).uniform(-1, 1, p.op.n)).cuda()
        b = torch.from_numpy(p.b).cuda()
        for method, kw in runs:
            out = []
            for var in (0, flag):
                mi = kw["max_iter"]
                opt = P.make_options(method=method, jacobi=True, fp32=fp32, history_cap=mi + 2,
                                     variant=P.PCG_VAR_SET | P.PCG_VAR_NT | ept_flag | var,
                                     block_size=shape[0], grid_blocks=48, **kw)
                s = P.Solver(p.op, opt)
                x = torch.from_numpy(x0).clone().cuda()
                r = s.solve(b, x)
                r["x"] = x.cpu().numpy()
                r["info"] = s.info()
                r["user_res"] = s.true_residual(b, xu)
                torch.cuda.synchronize()
                s.close()
                out.append(r)
            a, c = out
            print(f"[csr-copies] {p.name} {method} {form} fp32={fp32}: {a['status']} {a['iterations']} it, "
                  f"{a['replacements']} restarts", flush=True)
            assert a["info"]["csr_form_name"] == "csr" and c["info"]["csr_form_name"] == form, (p.name, method)
            assert (c["info"]["block"], c["info"]["ept"]) == shape
            assert a["iterations"] == c["iterations"] and a["status"] == c["status"]
            assert a["replacements"] == c["replacements"]
            np.testing.assert_array_equal(a["res"], c["res"])
            np.testing.assert_array_equal(a["x"], c["x"])
            assert a["rel_res_true"] == c["rel_res_true"] and a["user_res"] == c["user_res"]
            if method == "pipe_rr" and kw.get("rr_tau") == 1e-300:
                assert a["replacements"] > 0
