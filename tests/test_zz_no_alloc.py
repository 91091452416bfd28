"""pcg_solve_static (the entry point that allocates nothing: its workspace is
a static device array inside the library) against pcg_create + pcg_solve on
caller memory: the same kernels and launch shape, so the same bits, on two
calls in a row with the second one smaller (the scratch keeps the first
call's contents).  The binary64 cases also meet the oracle's parity bar:
recursive residual history to 1e-10 over the first 50 iterations and the
final explicit residual to 1e-12."""
import numpy as np
import pytest

import oracle
import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def rect3d(nx, ny, nz, seed):
    op = problems.stencil3d(nx, ny, nz)
    xt = np.random.default_rng(seed).uniform(-1, 1, op.n)
    return op, problems.to_scipy(op) @ xt


def rect2d(nx, ny, seed):
    op = problems.stencil2d(nx, ny)
    xt = np.random.default_rng(seed).uniform(-1, 1, op.n)
    return op, problems.to_scipy(op) @ xt


def aniso(n, seed):
    p = problems.anisotropic_csr(n, seed=seed)
    return p.op, p.b


# (method, jacobi, fp32, sigma, first system, second smaller system)
CASES = {
    "pipe_shift_fp64_jacobi": ("pipe_shift", True, False, 1.0, lambda: rect3d(80, 78, 76, 1), lambda: rect3d(21, 17, 13, 2)),
    "cg_fp64": ("cg", False, False, 0.0, lambda: rect2d(200, 150, 3), lambda: rect2d(33, 29, 4)),
    "pipe_fp64_jacobi_csr": ("pipe", True, False, 0.0, lambda: aniso(96, 5), lambda: aniso(40, 6)),
    "pipe_shift_fp32_csr": ("pipe_shift", True, True, 1.0, lambda: aniso(128, 7), lambda: aniso(48, 8)),
}


def options(P, method, jac, fp32, sigma, n):
    # binary64: no restarts, as the oracle runs; FP32-stream: restarts from
    # the binary64 x until the explicit residual meets 1e-8
    return P.make_options(method=method, jacobi=jac, fp32=fp32, sigma=sigma, rtol=1e-8 if fp32 else 1e-10,
                          max_iter=3000, history_cap=3002, use_graph=False, true_residual_check=fp32,
                          replace_max=10)


@pytest.mark.parametrize("case", sorted(CASES))
def test_static_solve_matches_workspace_solve(torch, case):
    from paper_1706_05988_amd import pcg as P
    method, jac, fp32, sigma, first, second = CASES[case]
    for k, make in enumerate((first, second)):
        op, b_np = make()
        print(f"[no_alloc] {case} call {k + 1}: n = {op.n}", flush=True)
        b = torch.from_numpy(b_np).cuda()
        x_ref = torch.zeros_like(b)
        s = P.Solver(op, options(P, method, jac, fp32, sigma, op.n))
        assert s.nbytes <= P.PCG_STATIC_SCRATCH_BYTES
        ref = s.solve(b, x_ref)
        s.close()
        x = torch.full_like(b, 0.0)
        got = P.solve_static(op, options(P, method, jac, fp32, sigma, op.n), b, x)
        torch.cuda.synchronize()
        assert got["status"] == ref["status"] == "converged", (got["status"], ref["status"])
        assert got["iterations"] == ref["iterations"]
        assert got["replacements"] == ref["replacements"]
        assert got["rel_res_true"] == ref["rel_res_true"]
        np.testing.assert_array_equal(got["res"], ref["res"])
        np.testing.assert_array_equal(got["alpha"], ref["alpha"])
        np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        if not fp32:
            o = oracle.solve(op, b_np, np.zeros(op.n), method=method, sigma=sigma, rtol=1e-10, max_iter=3000,
                             jacobi=jac, threads=8)
            kk = min(50, o["iterations"], got["iterations"])
            np.testing.assert_allclose(got["res"][: kk + 1], o["res"][: kk + 1], rtol=1e-10)
            if method == "pipe":  # its stagnation level is rounding-determined: a 10x band
                assert got["rel_res_true"] <= 10 * max(o["rel_res_true"], 1e-10)
            else:
                assert abs(got["rel_res_true"] - o["rel_res_true"]) <= 1e-12
        else:
            assert got["rel_res_true"] <= 1e-8


def test_static_solve_rejects_a_solve_beyond_the_scratch(torch):
    from paper_1706_05988_amd import pcg as P
    op = problems.stencil3d(128, 128, 128)
    b = torch.ones(op.n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(P.PcgError) as ei:
        P.solve_static(op, P.make_options(jacobi=True), b, x)
    assert ei.value.status == P.PCG_ERR_INVALID
    assert "static scratch" in str(ei.value)
    assert float(x.abs().max()) == 0.0  # nothing ran
