"""The continuously batching server: results equal the same solve alone,
requests join while others run, admission respects the HBM budget."""
import threading
import time

import numpy as np
import pytest

import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def request_set():
    ps = []
    for k, (nx, ny) in enumerate([(40, 17), (64, 64), (9, 7), (100, 30)]):
        op = problems.stencil2d(nx, ny, shift=0.02 * (k + 1))
        b = np.random.default_rng(10 + k).uniform(-1, 1, op.n)
        ps.append(problems.Problem(f"r{k}", op, b, np.zeros(op.n), None, sigma=4.0 + op.shift, rtol=1e-8,
                                   max_iter=4000))
    ps.append(problems.poisson3d(21, seed=8))
    ps[-1].rtol = 1e-8
    ps.append(problems.banded_csr(4000, seed=9))
    ps.append(problems.anisotropic_csr(20, seed=3))
    ps[-1].rtol = 1e-8
    return ps


def opts(P, p, fp32=True):
    return P.make_options(method="pipe_shift", jacobi=p.jacobi, fp32=fp32, sigma=p.sigma, rtol=p.rtol,
                          max_iter=p.max_iter, replace_max=8, history_cap=64)


def solve_alone(torch, P, p):
    srv = P.Server(64 << 20, max_slots=4)
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros_like(b)
    r = srv.wait(srv.submit(p.op, opts(P, p), b, x))
    r["x"] = x.cpu().numpy()
    srv.close()
    return r


def test_server_results_equal_alone(torch):
    from paper_1706_05988_amd import pcg as P
    ps = request_set()
    srv = P.Server(256 << 20, max_slots=16)
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    tickets = [srv.submit(p.op, opts(P, p), b, x) for p, b, x in zip(ps, bs, xs)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for p, r, x in zip(ps, res, xs):
        assert r["status"] == "converged", p.name
        assert r["rel_res_true"] <= 1e-8, (p.name, r["rel_res_true"])
        alone = solve_alone(torch, P, p)
        assert np.array_equal(alone["x"], x.cpu().numpy()), p.name
        assert alone["iterations"] == r["iterations"]


def test_server_admits_while_running_and_respects_budget(torch):
    """Arrivals spread in time join the running batch; a small arena holds
    only a few systems at once, so the rest wait for memory."""
    from paper_1706_05988_amd import pcg as P
    ps = request_set() * 3
    srv = P.Server(6 << 20, max_slots=64)  # a few MB: admission by footprint matters
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    tickets = []

    def producer():
        for p, b, x in zip(ps, bs, xs):
            tickets.append(srv.submit(p.op, opts(P, p), b, x))
            time.sleep(0.002)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    res = [srv.wait(t) for t in tickets]
    info = srv.info()
    srv.close()
    for p, r in zip(ps, res):
        assert r["status"] == "converged", p.name
        assert r["rel_res_true"] <= 1e-8
    assert info["completed"] == len(ps) and info["failed"] == 0
    assert info["running"] == 0 and info["queued"] == 0
    assert info["arena_free"] == info["arena_bytes"]  # every range returned
    # identical requests give identical bits whenever they ran
    n = len(request_set())
    for k in range(n):
        assert np.array_equal(xs[k].cpu().numpy(), xs[k + n].cpu().numpy())
        assert np.array_equal(xs[k].cpu().numpy(), xs[k + 2 * n].cpu().numpy())


def test_server_budget_error_and_poll(torch):
    from paper_1706_05988_amd import pcg as P
    srv = P.Server(2 << 20, max_slots=4)
    big = problems.poisson3d(64, seed=1)  # needs far more than 2 MB
    b = torch.from_numpy(big.b).cuda()
    x = torch.zeros_like(b)
    with pytest.raises(P.PcgError) as ei:
        srv.submit(big.op, opts(P, big), b, x)
    assert ei.value.status == P.PCG_ERR_BUDGET
    p = request_set()[2]
    b = torch.from_numpy(p.b).cuda()
    x = torch.zeros_like(b)
    t = srv.submit(p.op, opts(P, p), b, x)
    r = None
    for _ in range(2000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.001)
    assert r is not None and r["status"] == "converged"
    srv.close()


def test_server_failed_request_leaves_the_others_alone(torch):
    """A request with a non-finite right-hand side and one on an indefinite
    operator end with their own status; the requests served beside them get
    the bits they get alone."""
    from paper_1706_05988_amd import pcg as P
    good = request_set()[:2]
    nanb = good[0].b.copy()
    nanb[3] = np.inf
    bad_rhs = problems.Problem("inf_rhs", good[0].op, nanb, np.zeros(good[0].op.n), None, sigma=good[0].sigma,
                               rtol=1e-8, max_iter=4000)
    n = 40
    vals = np.linspace(-1.0, 3.0, n)
    vals[np.abs(vals) < 1e-3] = 0.5
    indef = problems.Problem("indef", problems.csr_operator(np.arange(n + 1), np.arange(n, dtype=np.int32), vals),
                             np.ones(n), np.zeros(n), None, sigma=1.0, rtol=1e-8, max_iter=100)
    ps = [good[0], bad_rhs, indef, good[1]]
    srv = P.Server(64 << 20, max_slots=8)
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    tickets = [srv.submit(p.op, opts(P, p), b, x) for p, b, x in zip(ps, bs, xs)]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    assert res[1]["status"] == "nonfinite"
    assert res[2]["status"] == "breakdown"
    for k in (0, 3):
        alone = solve_alone(torch, P, ps[k])
        assert res[k]["status"] == alone["status"] == "converged"
        assert res[k]["iterations"] == alone["iterations"]
        assert np.array_equal(alone["x"], xs[k].cpu().numpy())


def test_server_fp64_requests_match_the_oracle_in_a_mixed_stream(torch):
    """Binary64 requests of every operator kind, submitted one by one while
    the others run: each result follows the oracle on the same system --
    sqrt(rho_i)/||b||, alpha_i and beta_i to 1e-10 over the first 50
    iterations and the final explicit residual to 1e-12."""
    import oracle
    from paper_1706_05988_amd import pcg as P
    ps = request_set()
    for p in ps:
        p.rtol = 1e-10
    srv = P.Server(256 << 20, max_slots=16)
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    tickets = []
    for p, b, x in zip(ps, bs, xs):
        o = P.make_options(method="pipe_shift", jacobi=p.jacobi, sigma=p.sigma, rtol=p.rtol, max_iter=p.max_iter,
                           true_residual_check=False, history_cap=p.max_iter + 2)
        tickets.append(srv.submit(p.op, o, b, x))
        time.sleep(0.003)
    res = [srv.wait(t) for t in tickets]
    srv.close()
    assert any(r["admitted_at"] > 0 for r in res)  # some joined a running batch
    for p, r, x in zip(ps, res, xs):
        o = oracle.solve(p.op, p.b, p.x0, method="pipe_shift", sigma=p.sigma, rtol=p.rtol, max_iter=p.max_iter,
                         jacobi=p.jacobi, threads=8)
        assert r["status"] == o["status"] == "converged", p.name
        assert abs(r["iterations"] - o["iterations"]) <= 1, p.name
        k = min(50, o["iterations"], r["iterations"])
        np.testing.assert_allclose(r["res"][: k + 1], o["res"][: k + 1], rtol=1e-10, err_msg=p.name)
        np.testing.assert_allclose(r["alpha"][:k], o["alpha"][:k], rtol=1e-10, err_msg=p.name)
        np.testing.assert_allclose(r["beta"][1:k], o["beta"][1:k], rtol=1e-10, err_msg=p.name)
        assert abs(r["rel_res_true"] - o["rel_res_true"]) <= 1e-12, (p.name, r["rel_res_true"], o["rel_res_true"])


def test_server_launch_failure_returns_slots_and_memory(torch, monkeypatch):
    """A launch that fails (injected from the host: the server issues no
    device work for it) fails the requests then running with PCG_ERR_HIP;
    their slots and arena ranges come back, and the same requests submitted
    afterwards get the bits they get alone."""
    from paper_1706_05988_amd import pcg as P
    ps = request_set()[:4]
    monkeypatch.setenv("PCG_SERVER_FAIL_AT_LAUNCH", "1")
    srv = P.Server(16 << 20, max_slots=4)
    monkeypatch.delenv("PCG_SERVER_FAIL_AT_LAUNCH")
    bs = [torch.from_numpy(p.b).cuda() for p in ps]
    xs = [torch.zeros_like(b) for b in bs]
    tickets = [srv.submit(p.op, opts(P, p), b, x) for p, b, x in zip(ps, bs, xs)]
    outcome = []
    for t in tickets:
        try:
            outcome.append(srv.wait(t)["status"])
        except P.PcgError as e:
            outcome.append(e.status)
    failed = [o for o in outcome if o == P.PCG_ERR_HIP]
    assert failed, outcome  # the slow ones were still running at launch 1
    info = srv.info()
    assert info["failed"] == len(failed)
    assert info["running"] == 0 and info["arena_free"] == info["arena_bytes"]
    # the server goes on: every slot and the whole arena are usable again
    xs2 = [torch.zeros_like(b) for b in bs]
    res = [srv.wait(srv.submit(p.op, opts(P, p), b, x)) for p, b, x in zip(ps, bs, xs2)]
    info = srv.info()
    srv.close()
    assert info["arena_free"] == info["arena_bytes"] and info["running"] == 0
    for p, r, x in zip(ps, res, xs2):
        assert r["status"] == "converged", p.name
        alone = solve_alone(torch, P, p)
        assert np.array_equal(alone["x"], x.cpu().numpy()), p.name


def test_server_joins_requests_into_a_running_batch(torch):
    """Continuous batching: requests submitted while a long solve is on the
    device join its batch at a later launch (the long one still iterating),
    run beside it, and give the bits they give alone."""
    from paper_1706_05988_amd import pcg as P
    op = problems.stencil2d(300, 280)  # no preconditioner: ~1000 iterations, many launches
    b_long = np.random.default_rng(5).uniform(-1, 1, op.n)
    long_p = problems.Problem("long", op, b_long, np.zeros(op.n), None, sigma=4.0, rtol=1e-8, max_iter=20000)
    short = request_set()[:3]
    srv = P.Server(256 << 20, max_slots=8)
    bl = torch.from_numpy(long_p.b).cuda()
    xl = torch.zeros_like(bl)
    bs = [torch.from_numpy(p.b).cuda() for p in short]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    t_long = srv.submit(long_p.op, opts(P, long_p), bl, xl)
    for _ in range(20000):  # until the long solve has run two launches
        if srv.info()["launches"] >= 2:
            break
        time.sleep(0.0005)
    tickets = [srv.submit(p.op, opts(P, p), b, x) for p, b, x in zip(short, bs, xs)]
    res = [srv.wait(t) for t in tickets]
    r_long = srv.wait(t_long)
    info = srv.info()
    srv.close()
    assert r_long["status"] == "converged" and r_long["admitted_at"] == 0
    end_long = r_long["admitted_at"] + r_long["launches"]
    for p, r, x in zip(short, res, xs):
        assert r["status"] == "converged", p.name
        assert 2 <= r["admitted_at"] < end_long, (r["admitted_at"], end_long)
        alone = solve_alone(torch, P, p)
        assert np.array_equal(alone["x"], x.cpu().numpy()), p.name
    assert info["max_running"] >= 2
    assert np.array_equal(solve_alone(torch, P, long_p)["x"], xl.cpu().numpy())


def test_server_admission_is_first_in_first_out_under_a_full_arena(torch):
    """A queue far larger than the arena for a long time: the arena holds the
    large request alone, or small ones, never the large one beside a small
    one.  Requests are admitted in submission order (the queue head is never
    skipped, so the large request does not starve behind small ones submitted
    after it, and those wait until it is done), every request finishes with
    the bits it gets alone, and all memory comes back."""
    from paper_1706_05988_amd import pcg as P
    op = problems.stencil2d(200, 160)
    big = problems.Problem("big", op, np.random.default_rng(1).uniform(-1, 1, op.n), np.zeros(op.n), None,
                           sigma=4.0, rtol=1e-8, max_iter=20000)
    small = request_set()[:2]
    order = [small[0], small[1], big] + [small[k % 2] for k in range(12)]
    k_big = 2
    ob = opts(P, big)
    hb = np.zeros((ob.history_cap, P.PCG_HISTORY_FIELDS))  # the size query checks the history buffer
    ob.history = hb.ctypes.data
    foot_big = P.pcg_batch_workspace_size([P.DeviceOperator(big.op, ob.prec).struct], [ob])
    srv = P.Server(foot_big + (16 << 10), max_slots=16)  # no small request fits beside the big one
    bs = [torch.from_numpy(p.b).cuda() for p in order]
    xs = [torch.zeros_like(b) for b in bs]
    torch.cuda.synchronize()
    tickets = [srv.submit(p.op, opts(P, p), b, x) for p, b, x in zip(order, bs, xs)]
    res = [srv.wait(t) for t in tickets]
    info = srv.info()
    srv.close()
    adm = [r["admitted_at"] for r in res]
    assert adm == sorted(adm), adm  # first in, first admitted
    end_big = adm[k_big] + res[k_big]["launches"]
    assert adm[k_big] >= max(adm[j] + res[j]["launches"] for j in range(k_big)) - 1  # waited for memory
    assert all(a >= end_big for a in adm[k_big + 1:]), (adm, end_big)
    assert all(r["status"] == "converged" for r in res)
    assert info["completed"] == len(order) and info["arena_free"] == info["arena_bytes"]
    assert np.array_equal(solve_alone(torch, P, big)["x"], xs[k_big].cpu().numpy())
    assert np.array_equal(solve_alone(torch, P, small[1])["x"], xs[-1].cpu().numpy())
