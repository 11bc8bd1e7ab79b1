"""GPU tests of the serving form: continuous batching on resident matrices.

Each request's result in the mix must equal the same request run alone
(ilu_smooth) bit for bit, and the oracle's; admission respects the workspace
arena; every request completes (no starvation), including requests that
arrive while others are running.  Both scheduling modes: one batched launch
per sweep (stepwise), and one persistent launch per admitted batch whose
requests chain their sweeps through device-side counters."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


@pytest.fixture(scope="module")
def pool(orc, B, ctx):
    """Resident matrices of different sizes (ragged row counts included)."""
    out = []
    for j, N in enumerate((6, 9, 13, 16, 21)):
        A = W.vardens7(N, seed_rho=5 + j, with_cuts=False)
        Ls, U = orc.ilu0(A)
        d, dinv, Us = orc.scale_rows(U)
        Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(Ls), B.Csr.from_host(U)
        F = ctx.ilu_scale_factors(Ld, Ud)
        out.append(dict(A=A, Ls=Ls, Us=Us, dinv=dinv, Ad=Ad, Ud=Ud, F=F))
    torch.cuda.synchronize()
    return out


def _requests(pool, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        mid = int(rng.integers(0, len(pool)))
        n = pool[mid]["A"].n
        outer = int(rng.integers(1, 5))
        mL, mU = [(3, 3), (2, 4), (1, 3), (4, 1), (3, 2)][k % 5]
        reqs.append(dict(mid=mid, b=W.rhs(n, 100 + k), x0=W.rhs(n, 500 + k) * (k % 2), outer=outer, mL=mL, mU=mU))
    return reqs


def _alone(ctx, pool, r):
    p = pool[r["mid"]]
    x = dev(r["x0"])
    ctx.ilu_smooth(p["Ad"], p["F"], dev(r["b"]), x, r["outer"], r["mL"], r["mU"])
    return host(x)


def _drain(server, tickets, max_steps=100000, per_call=1):
    """Step the server until every ticket is done; per_call > 1: that many
    scheduling steps per call (silu_server_run, which enqueues several steps
    at once while nothing waits for admission)."""
    left = set(tickets)
    steps = 0
    while left:
        if per_call > 1:
            server.run(per_call)
        else:
            server.step()
        steps += 1
        for t in list(left):
            if server.poll(t) == server.DONE:
                left.discard(t)
        assert steps < max_steps, "requests starved"
    return steps


# The persistent mode is switched off in the library (set_mode refuses it):
# its launches did not finish on MI355X, and the cause is not yet found.
OFF = pytest.mark.skip(reason="persistent serving mode switched off: its launches did not finish on MI355X "
                              "(counters at agent and at system scope); cause not yet found")
MODES = [False, pytest.param(True, marks=OFF)]


@pytest.mark.parametrize("persistent", MODES, ids=["stepwise", "persistent"])
def test_mix_equals_alone_and_oracle(orc, B, ctx, pool, persistent):
    say(f"serving: mix vs alone, persistent={persistent}")
    reqs = _requests(pool, 60, seed=1)
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=64, persistent=persistent)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
    _drain(server, tickets)
    for i, r in enumerate(reqs):
        got = host(xs[i])
        np.testing.assert_array_equal(got, _alone(ctx, pool, r))
        if i < 12:
            p = pool[r["mid"]]
            ref = orc.smooth(p["A"], p["Ls"], p["Us"], p["dinv"], r["b"], r["x0"], r["outer"], r["mL"], r["mU"])
            np.testing.assert_array_equal(got, ref)
    server.close()


@pytest.mark.parametrize("persistent", MODES, ids=["stepwise", "persistent"])
def test_admission_by_workspace_budget(B, ctx, pool, persistent):
    """An arena that holds exactly two of the largest requests: never more
    active than fit, and everything completes in order of arrival."""
    say(f"serving: admission, persistent={persistent}")
    big = len(pool) - 1
    server = B.Server(ctx, arena_bytes=1 << 30, max_active=1000)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    per = server.request_bytes(mids[big])
    server.close()
    server = B.Server(ctx, arena_bytes=2 * per, max_active=1000, persistent=persistent)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    n = pool[big]["A"].n
    tickets, xs = [], []
    for k in range(7):
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        xs.append(x)
        tickets.append(server.submit(mids[big], dev(W.rhs(n, k)), x, 2, 3, 3))
    max_active = 0
    finished_order = []
    left = list(tickets)
    while left:
        active, queued = server.step()
        max_active = max(max_active, active)
        for t in list(left):
            if server.poll(t) == server.DONE:
                finished_order.append(t)
                left.remove(t)
    assert max_active <= 2
    # first come, first admitted: the arena holds two, so requests run in
    # pairs (0,1), (2,3), ...; a pair finishes at one step and polling may
    # notice its two members in either order
    pairs = [sorted(finished_order[i:i + 2]) for i in range(0, len(finished_order), 2)]
    assert pairs == [[0, 1], [2, 3], [4, 5], [6]]
    with pytest.raises(B.SiluError) as e:  # one request larger than the whole arena
        small = B.Server(ctx, arena_bytes=per // 2, max_active=4)
        m = small.register(pool[big]["Ad"], pool[big]["F"])
        small.submit(m, dev(W.rhs(n, 0)), xs[0], 1, 3, 3)
    assert e.value.status == -6
    server.close()


@pytest.mark.parametrize("persistent", MODES, ids=["stepwise", "persistent"])
def test_arrivals_while_running(B, ctx, pool, persistent):
    """Requests submitted between steps join running ones; each still equals
    its lone run."""
    say(f"serving: staggered arrivals, persistent={persistent}")
    reqs = _requests(pool, 40, seed=7)
    server = B.Server(ctx, arena_bytes=32 << 20, max_active=16, persistent=persistent)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    xs, tickets = [], []
    for i, r in enumerate(reqs):
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
        for _ in range(i % 3):
            server.step()
    _drain(server, tickets)
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, pool, r))
    server.close()


def test_serving_errors(B, ctx, pool):
    say("serving: errors")
    server = B.Server(ctx, arena_bytes=8 << 20, max_active=4)
    mid = server.register(pool[0]["Ad"], pool[0]["F"])
    n = pool[0]["A"].n
    b, x = dev(W.rhs(n, 0)), dev(np.zeros(n))
    with pytest.raises(B.SiluError) as e:
        server.submit(mid, b, x, 1, 1, 1)
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        server.submit(mid + 5, b, x, 1, 3, 3)
    assert e.value.status == -1
    Fu = ctx.ilu_scale_factors(pool[0]["F"].Ls, pool[0]["Ud"], scale=False)
    with pytest.raises(B.SiluError) as e:
        server.register(pool[0]["Ad"], Fu)
    assert e.value.status == -8
    server.close()


@pytest.fixture(scope="module")
def big_pool(orc, B, ctx):
    """Two larger matrices (1,024 and 432 row tiles of 256 rows), so that a
    persistent launch has many workgroups waiting on each other's tiles."""
    out = []
    for j, N in enumerate((64, 48)):
        A = W.vardens7(N, seed_rho=20 + j, with_cuts=False)
        Ls, U = orc.ilu0(A)
        Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(Ls), B.Csr.from_host(U)
        out.append(dict(A=A, Ad=Ad, F=ctx.ilu_scale_factors(Ld, Ud)))
    torch.cuda.synchronize()
    return out


@OFF
@pytest.mark.parametrize("max_wg", [1, 7, 300, 0])
def test_persistent_large_equals_alone(B, ctx, big_pool, max_wg):
    """Any workgroup cap (one workgroup runs the queue in order; 0 = the
    default) gives the lone results bit for bit, with requests on both
    matrices in one launch and further launches overlapping it."""
    say(f"serving: persistent large, max_wg={max_wg}")
    server = B.Server(ctx, arena_bytes=512 << 20, max_active=64, persistent=True, max_workgroups=max_wg)
    mids = [server.register(p["Ad"], p["F"]) for p in big_pool]
    reqs, xs, tickets = [], [], []
    for k in range(6):
        mid = k % 2
        n = big_pool[mid]["A"].n
        r = dict(mid=mid, b=W.rhs(n, 900 + k), x0=W.rhs(n, 950 + k) * (k % 3 == 0), outer=1 + k % 3, mL=3, mU=3)
        reqs.append(r)
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[mid], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
        if k % 2:
            server.step()
    _drain(server, tickets)
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, big_pool, r))
    server.close()


@OFF
def test_persistent_wait_limit_reports_timeout(B, ctx, big_pool):
    """The failure path, forced from the host: with a wait limit of one poll
    nearly every dependent tile gives up at once, the launch still drains, and
    poll reports SILU_ERR_TIMEOUT; the server then serves normally again."""
    say("serving: persistent wait limit")
    server = B.Server(ctx, arena_bytes=512 << 20, max_active=64, persistent=True, max_workgroups=1024)
    mid = server.register(big_pool[0]["Ad"], big_pool[0]["F"])
    n = big_pool[0]["A"].n
    server.set_wait_limit(1)
    tickets = [server.submit(mid, dev(W.rhs(n, k)), dev(np.zeros(n)), 2, 3, 3) for k in range(4)]
    server.step()
    torch.cuda.synchronize()
    timeouts = 0
    left = set(tickets)
    for _ in range(100000):
        for t in list(left):
            try:
                if server.poll(t) == server.DONE:
                    left.discard(t)
            except B.SiluError as e:
                assert e.status == -9
                timeouts += 1
                left.discard(t)
        if not left:
            break
    assert not left and timeouts >= 1
    server.set_wait_limit(0)
    r = dict(mid=0, b=W.rhs(n, 77), x0=np.zeros(n), outer=2, mL=3, mU=3)
    x = dev(r["x0"])
    t = server.submit(mid, dev(r["b"]), x, 2, 3, 3)
    _drain(server, [t])
    np.testing.assert_array_equal(host(x), _alone(ctx, big_pool, r))
    server.close()


def test_set_mode_rules(B, ctx, pool):
    say("serving: set_mode rules")
    server = B.Server(ctx, arena_bytes=8 << 20, max_active=4)
    mid = server.register(pool[0]["Ad"], pool[0]["F"])
    n = pool[0]["A"].n
    for bad in [(2, 0), (1, -1), (1, 70000)]:
        with pytest.raises(B.SiluError) as e:
            server.set_mode(*bad)
        assert e.value.status == -1
    t = server.submit(mid, dev(W.rhs(n, 0)), dev(np.zeros(n)), 1, 3, 3)
    with pytest.raises(B.SiluError) as e:  # a request is queued
        server.set_mode(server.PERSISTENT)
    assert e.value.status == -1
    _drain(server, [t])
    torch.cuda.synchronize()
    with pytest.raises(B.SiluError) as e:  # switched off in the library
        server.set_mode(server.PERSISTENT, 16)
    assert e.value.status == -8
    server.set_mode(server.STEPWISE)
    server.close()


def test_completed_reports_each_ticket_once(B, ctx, pool):
    """silu_server_completed returns every finished ticket exactly once, only
    after poll would report it done, with results equal to the lone runs."""
    say("serving: completed()")
    reqs = _requests(pool, 30, seed=11)
    server = B.Server(ctx, arena_bytes=16 << 20, max_active=8)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    xs, tickets = [], []
    seen = []
    for i, r in enumerate(reqs):
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
        server.step()
        seen += server.completed()
    for _ in range(100000):
        if len(seen) == len(tickets):
            break
        server.step()
        got = server.completed(capacity=3)
        assert len(got) <= 3
        for t in got:
            assert server.poll(t) == server.DONE
        seen += got
    assert sorted(seen) == sorted(tickets)
    assert server.completed() == []
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, pool, r))
    server.close()


def test_run_several_steps_per_call(B, ctx, pool):
    """silu_server_run: several scheduling steps per call, same results."""
    reqs = _requests(pool, 20, seed=13)
    server = B.Server(ctx, arena_bytes=16 << 20, max_active=8)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
    done = []
    for _ in range(10000):
        active, queued = server.run(5)
        done += server.completed()
        if len(done) == len(tickets):
            break
    assert sorted(done) == sorted(tickets)
    with pytest.raises(B.SiluError) as e:
        server.run(0)
    assert e.value.status == -1
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, pool, r))
    server.close()


def test_wait_and_times(B, ctx, pool):
    """silu_server_wait drives the server until the request is done; the
    submit and completion times are ordered; results equal the lone runs."""
    reqs = _requests(pool, 12, seed=17)
    server = B.Server(ctx, arena_bytes=16 << 20, max_active=4)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
    t0, d0 = server.times(tickets[-1])
    assert d0 is None
    server.wait(tickets[-1])  # the last one: everything before it is admitted first
    assert server.poll(tickets[-1]) == server.DONE
    for t in tickets:
        server.wait(t)
        a, d = server.times(t)
        assert d is not None and d >= a
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, pool, r))
    with pytest.raises(B.SiluError):
        server.times(10 ** 6)
    server.close()


def test_sliced_and_streamed_matrices_in_one_batch(orc, B, ctx):
    """A randomly permuted operator (no diagonal or offset structure: its
    batched sweeps stream the CSR arrays), a 27-point ILUT one and a
    variable-density one with cut cells (both swept through the server's
    sliced copies) served in the same steps: every result equals the request
    alone bit for bit, and the oracle's."""
    say("serving: sliced and streamed in one batch")
    mats = [(W.permuted_longrange7(7, seed=2), "ilu0", {}), (W.aniso27(8), "ilut", {"tau": 1e-3, "p": 20}),
            (W.vardens7(11, seed_rho=4), "iluk", {"k": 1})]
    pool = []
    for A, kind, params in mats:
        Ls, U = orc.factor(A, kind, params)
        _, dinv, Us = orc.scale_rows(U)
        Ad = B.Csr.from_host(A)
        F = ctx.ilu_scale_factors(B.Csr.from_host(Ls), B.Csr.from_host(U))
        pool.append(dict(A=A, Ls=Ls, Us=Us, dinv=dinv, Ad=Ad, F=F))
    server = B.Server(ctx, arena_bytes=32 << 20, max_active=16)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    reqs = []
    for k in range(12):
        mid = k % 3
        n = pool[mid]["A"].n
        reqs.append(dict(mid=mid, b=W.rhs(n, 40 + k), x0=W.rhs(n, 70 + k) * (k % 2), outer=1 + k % 3, mL=3, mU=2))
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
    _drain(server, tickets)
    for i, r in enumerate(reqs):
        p = pool[r["mid"]]
        got = host(xs[i])
        np.testing.assert_array_equal(got, _alone(ctx, pool, r))
        ref = orc.smooth(p["A"], p["Ls"], p["Us"], p["dinv"], r["b"], r["x0"], r["outer"], r["mL"], r["mU"])
        np.testing.assert_array_equal(got, ref)
    server.close()


def _tol_with_margin(hist_fn, tol):
    """A tolerance at least 1e-6 (relative) away from every residual the
    oracle's run checks, so that the two sides' different summation orders
    cannot flip a decision."""
    for _ in range(20):
        k, x, hist = hist_fn(tol)
        if np.all(np.abs(hist / tol - 1.0) > 1e-6):
            return tol, (k, x, hist)
        tol *= 1.37
    raise AssertionError("no tolerance with a margin")


@pytest.mark.parametrize("per_call", [1, 16], ids=["step", "run16"])
def test_solve_requests_match_the_oracle(orc, B, ctx, pool, per_call):
    """Solve requests (iterate until eq. relres < tol) in the same steps as
    smoother requests: the outer-step count and x equal the oracle's
    smooth_until bit for bit, the reported relative residual to rounding;
    including x0 already converged (0 steps), max_outer = 0, a request that
    never converges (max_outer + 1) and m_L = 1 (the residual fused with
    D^{-1}); driven one step per call and 16 per call (several steps
    enqueued at once)."""
    say("serving: solve requests")
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=64)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    # (matrix, m_L, m_U, tol, max_outer): the two smallest pool matrices converge
    # (tens of steps), the larger ones do not within these limits
    plan = [(0, 3, 3, 1e-3, 60), (0, 6, 6, 1e-8, 80), (1, 4, 4, 1e-6, 200), (1, 1, 6, 1e-4, 200),
            (0, 6, 1, 1e-5, 120), (3, 3, 3, 1e-8, 5), (4, 2, 2, 1e-6, 0), (2, 4, 2, 1e-12, 3), (1, 3, 3, 1e-2, 50),
            (0, 2, 4, 1e-7, 100)]
    cases = []
    for k, (mid, mL, mU, tol, max_outer) in enumerate(plan):
        p = pool[mid]
        n = p["A"].n
        b = W.rhs(n, 300 + k)
        x0 = W.rhs(n, 400 + k) * (k % 2)
        if k == 7:  # already converged: b = A x0 exactly
            x0 = W.rhs(n, 400 + k)
            b = orc.spmv(p["A"], x0)

        def run(t, p=p, b=b, x0=x0, mL=mL, mU=mU, max_outer=max_outer):
            return orc.smooth_until(p["A"], p["Ls"], p["Us"], p["dinv"], b, x0, mL, mU, t, max_outer)

        tol, ref = (tol, run(tol)) if k == 7 else _tol_with_margin(run, tol)
        cases.append(dict(mid=mid, b=b, x0=x0, mL=mL, mU=mU, tol=tol, max_outer=max_outer, ref=ref))
    tickets, xs = [], []
    for k, c in enumerate(cases):
        x = dev(c["x0"])
        xs.append(x)
        tickets.append(server.submit_solve(mids[c["mid"]], dev(c["b"]), x, c["tol"], c["max_outer"], c["mL"], c["mU"]))
        # a smoother request between the solve requests shares their steps
        n = pool[c["mid"]]["A"].n
        server.submit(mids[c["mid"]], dev(W.rhs(n, 900 + k)), torch.zeros(n, dtype=torch.float64, device="cuda"),
                      2, 3, 3)
    _drain(server, tickets, per_call=per_call)
    seen = set()
    for k, c in enumerate(cases):
        k_ref, x_ref, hist = c["ref"]
        steps, rel = server.solve_result(tickets[k])
        seen.add(k_ref if k_ref <= c["max_outer"] else "never")
        assert steps == k_ref, f"case {k}: {steps} steps, oracle {k_ref}"
        np.testing.assert_array_equal(host(xs[k]), x_ref)
        assert rel == pytest.approx(hist[-1], rel=1e-12)
    assert 0 in seen and "never" in seen and len(seen) >= 6
    with pytest.raises(B.SiluError) as e:  # not a solve request
        t = server.submit(mids[0], dev(W.rhs(pool[0]["A"].n, 1)), dev(np.zeros(pool[0]["A"].n)), 1, 3, 3)
        server.wait(t)
        server.solve_result(t)
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        server.submit_solve(mids[0], dev(W.rhs(pool[0]["A"].n, 1)), dev(np.zeros(pool[0]["A"].n)), 0.0, 5, 3, 3)
    assert e.value.status == -1
    server.close()


def test_solve_request_finishes_when_converged(orc, B, ctx, pool):
    """A solve request with a step limit far beyond what it needs is retired
    a few steps after the device's check passes (the host reads the request's
    stop flag), not after max_outer steps; with and without other work in the
    server, and the result still equals the oracle's."""
    say("serving: solve request retired when converged")
    p = pool[0]
    n = p["A"].n
    b = W.rhs(n, 11)
    k_ref, x_ref, _ = orc.smooth_until(p["A"], p["Ls"], p["Us"], p["dinv"], b, np.zeros(n), 3, 3, 1e-6, 1 << 20)
    assert k_ref < 100
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=8)
    mid = server.register(p["Ad"], p["F"])
    other = server.register(pool[4]["Ad"], pool[4]["F"])
    for busy in (False, True):
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        t = server.submit_solve(mid, dev(b), x, 1e-6, 1 << 20, 3, 3)
        if busy:
            n4 = pool[4]["A"].n
            server.submit(other, dev(W.rhs(n4, 3)), torch.zeros(n4, dtype=torch.float64, device="cuda"), 4, 3, 3)
        steps = _drain(server, [t], max_steps=5 * k_ref + 200)
        assert steps <= 5 * k_ref + 40
        k, _ = server.solve_result(t)
        assert k == k_ref
        np.testing.assert_array_equal(host(x), x_ref)
    server.close()


@pytest.mark.parametrize("per_call", [1, 8], ids=["step", "run8"])
def test_more_than_64_requests_in_one_step(B, ctx, pool, per_call):
    """Over 64 requests active at once (the launch finds a workgroup's op by
    bisection there, by one ballot per wave up to 64): each result equals the
    request alone; with 8 steps per call their staged op tables of several
    steps share one copy."""
    say("serving: > 64 active requests")
    server = B.Server(ctx, arena_bytes=256 << 20, max_active=160)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    reqs = []
    for k in range(150):
        mid = k % 3  # the small matrices, so that all fit at once
        n = pool[mid]["A"].n
        reqs.append(dict(mid=mid, b=W.rhs(n, 1000 + k), x0=W.rhs(n, 2000 + k) * (k % 3 == 0), outer=1 + k % 3,
                         mL=3, mU=3))
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"]))
    a, q = server.step()
    assert a > 64 and q == 0
    _drain(server, tickets, per_call=per_call)
    for i, r in enumerate(reqs):
        np.testing.assert_array_equal(host(xs[i]), _alone(ctx, pool, r))
    server.close()


@pytest.mark.parametrize("per_call", [1, 16], ids=["step", "run16"])
def test_fp32_inner_requests_equal_the_single_call(orc, B, ctx, per_call):
    """FP32-inner requests (L and U~ sweeps on FP32 factor values) mixed in the
    same steps with FP64 ones, on sliced and streamed matrices: each equals
    ilu_smooth(mixed=True) alone bit for bit (the FP64 ones ilu_smooth), and
    stays within the mixed form's 1e-5 of the FP64 oracle; the first step's 30
    FP64 residuals (more than 24 ops of one precision) take the staged op
    tables beside the kernel-argument batch of the others; a matrix
    registered without FP32 values refuses them."""
    say("serving: FP32-inner requests")
    mats = [(W.vardens7(9, seed_rho=6, with_cuts=False), "ilu0", {}), (W.aniso27(7), "ilut", {"tau": 1e-3, "p": 20}),
            (W.permuted_longrange7(6, seed=3), "ilu0", {})]
    pool = []
    for A, kind, params in mats:
        Ls, U = orc.factor(A, kind, params)
        _, dinv, Us = orc.scale_rows(U)
        Ad = B.Csr.from_host(A)
        F = ctx.ilu_scale_factors(B.Csr.from_host(Ls), B.Csr.from_host(U), fp32=True)
        pool.append(dict(A=A, Ls=Ls, Us=Us, dinv=dinv, Ad=Ad, F=F))
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=64)
    mids = [server.register(p["Ad"], p["F"]) for p in pool]
    reqs = []
    for k in range(40):
        mid = k % 3
        n = pool[mid]["A"].n
        mL, mU = [(3, 3), (1, 3), (4, 2), (2, 1)][k % 4]
        reqs.append(dict(mid=mid, b=W.rhs(n, 60 + k), x0=W.rhs(n, 80 + k) * (k % 2), outer=1 + k % 3, mL=mL, mU=mU,
                         mixed=k % 5 != 0))
    xs, tickets = [], []
    for r in reqs:
        x = dev(r["x0"])
        xs.append(x)
        tickets.append(server.submit(mids[r["mid"]], dev(r["b"]), x, r["outer"], r["mL"], r["mU"], mixed=r["mixed"]))
    _drain(server, tickets, per_call=per_call)
    for i, r in enumerate(reqs):
        p = pool[r["mid"]]
        xa = dev(r["x0"])
        ctx.ilu_smooth(p["Ad"], p["F"], dev(r["b"]), xa, r["outer"], r["mL"], r["mU"], mixed=r["mixed"])
        got = host(xs[i])
        np.testing.assert_array_equal(got, host(xa))
        ref = orc.smooth(p["A"], p["Ls"], p["Us"], p["dinv"], r["b"], r["x0"], r["outer"], r["mL"], r["mU"])
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= (1e-5 if r["mixed"] else 0.0)
    plain = B.Server(ctx, arena_bytes=8 << 20, max_active=4)
    m0 = plain.register(pool[0]["Ad"], ctx.ilu_scale_factors(B.Csr.from_host(pool[0]["Ls"]),
                                                             B.Csr.from_host(orc.factor(pool[0]["A"], "ilu0", {})[1])))
    n0 = pool[0]["A"].n
    with pytest.raises(B.SiluError) as e:
        plain.submit(m0, dev(W.rhs(n0, 1)), dev(np.zeros(n0)), 1, 3, 3, mixed=True)
    assert e.value.status == -8
    plain.close()
    server.close()


def test_solve_request_on_a_streamed_matrix(orc, B, ctx):
    """A randomly permuted operator of 42^3 rows: its column offsets span more
    than 16-bit codes reach and it has no diagonal structure, so the server
    streams its CSR arrays, and the convergence checks take their row values
    from the stream body.  Step count and x equal the oracle's."""
    say("serving: solve request on a streamed matrix")
    A = W.permuted_longrange7(42, seed=4)
    Ls, U = orc.ilu0(A)
    _, dinv, Us = orc.scale_rows(U)
    F = ctx.ilu_scale_factors(B.Csr.from_host(Ls), B.Csr.from_host(U))
    b = W.rhs(A.n, 7)
    k_ref, x_ref, hist = orc.smooth_until(A, Ls, Us, dinv, b, np.zeros(A.n), 3, 3, 1e-6, 200)
    assert k_ref < 200 and np.all(np.abs(hist / 1e-6 - 1.0) > 1e-6)
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=4)
    mid = server.register(B.Csr.from_host(A), F)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    t = server.submit_solve(mid, dev(b), x, 1e-6, 200, 3, 3)
    server.wait(t)
    k, rel = server.solve_result(t)
    assert k == k_ref
    np.testing.assert_array_equal(host(x), x_ref)
    assert rel == pytest.approx(hist[-1], rel=1e-12)
    server.close()


def test_per_ticket_state_stays_bounded(B, ctx, pool):
    """A long-running request loop keeps bounded per-ticket state: after more
    than 65,536 finished requests the oldest records are dropped (poll and wait
    report those tickets done, times refuses them), the latest are kept, and
    the pinned slots for solve-request results are reused rather than grown."""
    say("serving: bounded per-ticket state")
    p = pool[0]
    n = p["A"].n
    server = B.Server(ctx, arena_bytes=64 << 20, max_active=1024)
    mid = server.register(p["Ad"], p["F"])
    b = dev(W.rhs(n, 1))
    xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(1024)]
    first = last = None
    total = 0
    while total < 70000:
        tickets = [server.submit(mid, b, xs[k], 1, 2, 1) for k in range(1024)]
        first = tickets[0] if first is None else first
        last = tickets[-1]
        server.wait(last)  # admitted in order, same length: the last one done means all are
        total += len(tickets)
    records, slots, unreported = server.footprint()
    say(f"  {total} requests: records {records}, result slots {slots}, unreported {unreported}")
    assert records <= 65536 and unreported <= 65536
    assert server.poll(first) == server.DONE
    server.wait(first)
    with pytest.raises(B.SiluError):
        server.times(first)
    t_sub, t_done = server.times(last)
    assert t_done is not None and t_done >= t_sub
    # solve requests in waves: the pinned result slots do not grow with their number
    seen = []
    for wave in range(4):
        tickets = [server.submit_solve(mid, b, xs[k], 1e-300, 2, 2, 2) for k in range(1024)]
        server.wait(tickets[-1])
        for t in tickets:
            server.wait(t)
        k, rel = server.solve_result(tickets[-1])
        assert k == 3 and rel > 0.0  # never below 1e-300: max_outer + 1
        seen.append(server.footprint()[1])
    say(f"  pinned result slots after each wave of 1,024 solve requests: {seen}")
    assert seen[-1] == seen[1] and seen[-1] <= 16 * 1024
    server.close()
