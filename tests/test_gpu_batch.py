"""The batched persistent pass (pcg_batch_solve) against the oracle, and the
independence of each system's result from the rest of the batch."""
import numpy as np
import pytest

import oracle
import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def opts_for(P, p, fp32=False, hist=True, **kw):
    mi = kw.pop("max_iter", p.max_iter)
    return P.make_options(method=kw.pop("method", "pipe_shift"), jacobi=p.jacobi, fp32=fp32, sigma=p.sigma,
                          rtol=kw.pop("rtol", p.rtol), max_iter=mi, history_cap=(mi + 2) if hist else 0, **kw)


def run_batch(torch, probs, fp32=False, **kw):
    from paper_1706_05988_amd import pcg as P
    opts = [opts_for(P, p, fp32=fp32, **dict(kw)) for p in probs]
    B = P.Batch([p.op for p in probs], opts)
    bs = [torch.from_numpy(p.b).cuda() for p in probs]
    xs = [torch.from_numpy(p.x0).clone().cuda() for p in probs]
    res = B.solve(bs, xs)
    torch.cuda.synchronize()
    for r, x in zip(res, xs):
        r["x"] = x.cpu().numpy()
    return res


def mixed_set():
    ps = []
    for k, (nx, ny) in enumerate([(37, 11), (64, 64), (5, 3), (130, 41)]):
        op = problems.stencil2d(nx, ny, shift=0.01 * (k + 1))
        b = np.random.default_rng(k).uniform(-1, 1, op.n)
        ps.append(problems.Problem(f"r{k}", op, b, np.zeros(op.n), None, sigma=4.0 + op.shift, rtol=1e-10,
                                   max_iter=3000))
    ps.append(problems.poisson3d(19, seed=3))
    ps.append(problems.anisotropic_csr(24, seed=2))
    ps[-1].rtol, ps[-1].max_iter = 1e-10, 5000
    ps.append(problems.banded_csr(3001, seed=4))
    ps[-1].rtol = 1e-10
    return ps


def test_batch_matches_oracle_fp64(torch):
    ps = mixed_set()
    res = run_batch(torch, ps, true_residual_check=False)
    for p, g in zip(ps, res):
        o = oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma, rtol=p.rtol, max_iter=p.max_iter,
                         jacobi=p.jacobi)
        assert g["status"] == o["status"] == "converged", p.name
        assert abs(g["iterations"] - o["iterations"]) <= 2, p.name
        k = min(50, o["iterations"], g["iterations"])
        below = np.nonzero(o["res"][: k + 1] < 1e-12)[0]
        if below.size:
            k = max(1, int(below[0]) - 1)
        np.testing.assert_allclose(g["res"][: k + 1], o["res"][: k + 1], rtol=1e-10, err_msg=p.name)
        assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12, p.name


def test_batch_result_independent_of_batch_mix(torch):
    """A system's tiling and reduction order depend only on itself: solved
    alone or inside a batch it gives the same bits."""
    ps = mixed_set()
    together = run_batch(torch, ps)
    for k in (0, 4, 5, 6):  # 5, 6: CSR on the in-place and the sorted sliced-ELL copy
        alone = run_batch(torch, [ps[k]])[0]
        assert np.array_equal(alone["x"], together[k]["x"]), ps[k].name
        assert alone["iterations"] == together[k]["iterations"]
        assert np.array_equal(alone["res"], together[k]["res"], equal_nan=True)


def test_batch_result_independent_of_launch_mode(torch):
    """A large batch (more than 4096 tile items) starts in the split launch
    mode (transition kernel + pass) and moves to the fused mode as systems
    finish; a system solved alone runs fused all the way.  Both modes take
    the same transition with the same reduction: identical bits."""
    ps = []
    for k in range(40):
        op = problems.stencil2d(256, 256 - k, shift=0.02)
        b = np.random.default_rng(100 + k).uniform(-1, 1, op.n)
        ps.append(problems.Problem(f"big{k}", op, b, np.zeros(op.n), None, sigma=4.02, rtol=1e-8, max_iter=3000))
    small = mixed_set()[1]
    ps.append(small)
    assert sum((p.op.n + 511) // 512 for p in ps) > 4096
    together = run_batch(torch, ps, fp32=True, hist=False)
    for k in (0, 17, len(ps) - 1):
        alone = run_batch(torch, [ps[k]], fp32=True, hist=False)[0]
        assert together[k]["status"] == "converged", ps[k].name
        assert np.array_equal(alone["x"], together[k]["x"]), ps[k].name
        assert alone["iterations"] == together[k]["iterations"]
        assert alone["rel_res_true"] == together[k]["rel_res_true"]


def test_config4_full_batch_sampled(torch):
    """The 512-rectangle batch of the benchmark (FP32-stream p-CG-sh to 1e-8
    with the binary64 explicit check): every system converges to <= 1e-8, and
    three sampled systems (smallest, median, largest) reach within 10x of the
    oracle's level in the same storage form at the iteration count the GPU
    took."""
    ps = problems.batch_rectangles(512, seed=0)
    res = run_batch(torch, ps, fp32=True, rtol=1e-8, max_iter=20000, replace_max=8, hist=False)
    assert all(r["status"] == "converged" and r["rel_res_true"] <= 1e-8 for r in res)
    sizes = np.array([p.op.n for p in ps])
    for k in (int(sizes.argmin()), int(np.argsort(sizes)[len(sizes) // 2]), int(sizes.argmax())):
        p, g = ps[k], res[k]
        o = oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma, rtol=1e-8, max_iter=20000,
                         fp32_storage=True, replace_max=8, threads=8)
        assert o["status"] == "converged", p.name
        assert abs(g["iterations"] - o["iterations"]) <= max(3, 0.05 * o["iterations"]), p.name
        assert g["rel_res_true"] <= 10 * max(o["rel_res_true"], 1e-9), p.name


def _oracle_all(ps, **kw):
    """The oracle on every system, several at once (each single-threaded;
    the library call releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(lambda p: oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma,
                                                  threads=1, **kw), ps))


def test_config4_every_system_binary64_matches_the_oracle(torch):
    """The 512 rectangles of the benchmark batch solved in binary64 in one
    batch, each system against the oracle at the parity bar: sqrt(rho_i)/||b||,
    alpha_i and beta_i to 1e-10 over the first 50 iterations, the same
    iteration count (within one) and the final explicit residual to 1e-12."""
    from paper_1706_05988_amd import pcg as P
    ps = problems.batch_rectangles(512, seed=0)
    opts = [P.make_options(method="pipe_shift", sigma=p.sigma, rtol=1e-8, max_iter=3000,
                           true_residual_check=False, history_cap=52) for p in ps]
    B = P.Batch([p.op for p in ps], opts)
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    res = B.solve(bs, xs)
    torch.cuda.synchronize()
    orc = _oracle_all(ps, rtol=1e-8, max_iter=3000)
    for p, g, o in zip(ps, res, orc):
        assert g["status"] == o["status"] == "converged", p.name
        assert abs(g["iterations"] - o["iterations"]) <= 1, p.name
        k = min(50, g["iterations"], o["iterations"])
        np.testing.assert_allclose(g["res"][: k + 1], o["res"][: k + 1], rtol=1e-10, err_msg=p.name)
        np.testing.assert_allclose(g["alpha"][:k], o["alpha"][:k], rtol=1e-10, err_msg=p.name)
        np.testing.assert_allclose(g["beta"][1:k], o["beta"][1:k], rtol=1e-10, err_msg=p.name)
        assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12, p.name


def test_config4_every_system_fp32_stream_within_the_oracle_level(torch):
    """The benchmark's FP32-stream batch (to 1e-8, binary64 explicit check and
    restarts): every one of the 512 systems converges, and ends within 10x of
    the oracle's level in the same storage form with the same restart rule."""
    ps = problems.batch_rectangles(512, seed=0)
    res = run_batch(torch, ps, fp32=True, rtol=1e-8, max_iter=20000, replace_max=8, hist=False)
    orc = _oracle_all(ps, rtol=1e-8, max_iter=20000, fp32_storage=True, replace_max=8)
    for p, g, o in zip(ps, res, orc):
        assert g["status"] == o["status"] == "converged", p.name
        assert g["rel_res_true"] <= 1e-8, p.name
        assert g["rel_res_true"] <= 10 * o["rel_res_true"], p.name


def test_batch_fp32_stream_with_restarts(torch):
    """FP32-stream batch: every system reaches the tolerance through
    restarts from its binary64 x."""
    ps = problems.batch_rectangles(24, seed=3, side_min=16, side_max=80)
    res = run_batch(torch, ps, fp32=True, replace_max=10, hist=False)
    for p, g in zip(ps, res):
        assert g["status"] == "converged", p.name
        assert g["rel_res_true"] <= 1e-8, (p.name, g["rel_res_true"])


def test_batch_fp32_attainable_accuracy_vs_oracle_emulation(torch):
    ps = problems.batch_rectangles(6, seed=5, side_min=20, side_max=60)
    res = run_batch(torch, ps, fp32=True, rtol=1e-30, max_iter=300, true_residual_check=False)
    for p, g in zip(ps, res):
        o = oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma, rtol=1e-30, max_iter=300,
                         fp32_storage=True, ignore_breakdown=True)
        assert g["rel_res_true"] <= 10 * o["rel_res_true"], p.name


def test_batch_status_edge_cases(torch):
    ps = mixed_set()[:3]
    ps[1] = problems.Problem("capped", ps[1].op, ps[1].b, ps[1].x0, None, sigma=ps[1].sigma, rtol=1e-12,
                             max_iter=5)
    res = run_batch(torch, ps)
    assert res[1]["status"] == "max_iter" and res[1]["iterations"] == 5
    assert res[0]["status"] == "converged" and res[2]["status"] == "converged"


def test_batch_tune_picks_a_candidate_caches_it_and_keeps_the_bits(torch, tmp_path, monkeypatch):
    """pcg_batch_tune times every candidate (1..4 blocks per CU x 16/32/64
    passes per launch) on the caller's batch, writes the fastest into the
    options and the cache file, and a second call reads it back without
    measuring.  A solve with the chosen shape gives the same bits as one with
    the default shape: a system's tiling and reduction order do not depend on
    the grid or the graph length."""
    from paper_1706_05988_amd import pcg as P
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("PCG_TUNE_CACHE", str(cache))
    ps = problems.batch_rectangles(24, seed=7, side_min=16, side_max=96)

    def make():
        opts = [opts_for(P, p, fp32=True, hist=False, rtol=1e-8, max_iter=5000, replace_max=8) for p in ps]
        return P.Batch([p.op for p in ps], opts)

    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    x0s = [torch.from_numpy(p.x0).cuda() for p in ps]
    xs = [torch.empty_like(x) for x in x0s]
    B = make()
    t = B.tune(bs, x0s, xs)
    torch.cuda.synchronize()
    assert (t["grid_blocks"], t["iters_per_launch"]) == (0, 0) or \
        (t["grid_blocks"] in (256, 512, 768, 1024) and t["iters_per_launch"] in (16, 32, 64))
    assert t["solve_ms"] > 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch_p1_c24_")
    B2 = make()
    t2 = B2.tune(bs, x0s, xs)
    assert (t2["grid_blocks"], t2["iters_per_launch"]) == (t["grid_blocks"], t["iters_per_launch"])
    assert len(cache.read_text().splitlines()) == 1
    # tuned shape against the default shape
    ys = [x.clone() for x in x0s]
    tuned = B.solve(bs, ys)
    zs = [x.clone() for x in x0s]
    default = make().solve(bs, zs)
    torch.cuda.synchronize()
    for k in range(len(ps)):
        assert tuned[k]["status"] == default[k]["status"] == "converged"
        assert tuned[k]["iterations"] == default[k]["iterations"]
        assert torch.equal(ys[k], zs[k])


def test_batch_failures_stay_in_their_system(torch):
    """Systems that end in a breakdown (indefinite operator) or on a
    non-finite right-hand side, or that need no iteration (b = 0, an exact
    start), end with their own status, and the other systems of the batch
    keep the bits they get in a batch without them."""
    good = mixed_set()[:2]
    n = 40
    vals = np.linspace(-1.0, 3.0, n)
    vals[np.abs(vals) < 1e-3] = 0.5
    indef = problems.Problem("indef", problems.csr_operator(np.arange(n + 1), np.arange(n, dtype=np.int32), vals),
                             np.ones(n), np.zeros(n), None, sigma=1.0, rtol=1e-12, max_iter=100)
    nanb = good[0].b.copy()
    nanb[5] = np.nan
    bad_rhs = problems.Problem("nan_rhs", good[0].op, nanb, np.zeros(good[0].op.n), None, sigma=good[0].sigma,
                               rtol=1e-10, max_iter=3000)
    zero = problems.Problem("zero_rhs", good[1].op, np.zeros(good[1].op.n), np.zeros(good[1].op.n), None,
                            sigma=good[1].sigma, rtol=1e-10, max_iter=3000)
    man = problems.poisson2d_manufactured(20)
    exact = problems.Problem("exact_start", man.op, man.b, man.x_true.copy(), man.x_true, sigma=man.sigma,
                             rtol=1e-10, max_iter=3000)
    res = run_batch(torch, [good[0], indef, bad_rhs, good[1], zero, exact])
    alone = run_batch(torch, good)
    assert res[1]["status"] == "breakdown"
    assert res[2]["status"] == "nonfinite"
    assert res[4]["status"] == "converged" and res[4]["iterations"] == 0 and not np.any(res[4]["x"])
    assert res[5]["status"] == "converged" and res[5]["iterations"] == 0
    np.testing.assert_array_equal(res[5]["x"], man.x_true)
    for g, a in zip((res[0], res[3]), alone):
        assert g["status"] == a["status"] == "converged"
        assert g["iterations"] == a["iterations"]
        np.testing.assert_array_equal(g["x"], a["x"])


def test_large_system_chunked_reduction_matches_oracle_and_alone(torch):
    """A system with more than 1024 partials (here 700 x 600: 411 work tiles,
    1644 partials, two chunks) has its partials summed in fixed chunks by
    the chunk pass; beside small systems it gives the bits it gives alone,
    and it follows the oracle at the parity bar (binary64)."""
    op = problems.stencil2d(700, 600, shift=0.03)
    b = np.random.default_rng(21).uniform(-1, 1, op.n)
    big = problems.Problem("big700x600", op, b, np.zeros(op.n), None, sigma=4.03, rtol=1e-10, max_iter=4000)
    ps = [big] + mixed_set()[:3]
    together = run_batch(torch, ps, true_residual_check=False)
    alone = run_batch(torch, [big], true_residual_check=False)[0]
    assert np.array_equal(alone["x"], together[0]["x"])
    assert alone["iterations"] == together[0]["iterations"]
    np.testing.assert_array_equal(alone["res"], together[0]["res"])
    o = oracle.solve(big.op, big.b, big.x0, method="pipe_shift", sigma=big.sigma, rtol=big.rtol,
                     max_iter=big.max_iter, threads=8)
    g = together[0]
    assert g["status"] == o["status"] == "converged"
    assert abs(g["iterations"] - o["iterations"]) <= 1
    k = min(50, g["iterations"], o["iterations"])
    np.testing.assert_allclose(g["res"][: k + 1], o["res"][: k + 1], rtol=1e-10)
    assert abs(g["rel_res_true"] - o["rel_res_true"]) <= 1e-12
