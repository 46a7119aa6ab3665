"""Scheduler of the encode server on a fake backend (no GPU): admission by memory
budget, fair chunking, completion, and codes identical alone and in the mix."""
import numpy as np
import pytest

from paper_1806_04374_amd import serve


class FakeBackend(serve.Backend):
    """Codes a window by a deterministic function of its pixels; steps finish after
    ``lag`` polls; uploads become visible after ``upload_lag`` queries."""

    def __init__(self, N=3, K=2, lag=1, upload_lag=0, capacity=None):
        self.N, self.K, self.lag, self.upload_lag = N, K, lag, upload_lag
        self.capacity = capacity          # windows a step buffer holds (as the device slots)
        self.pixels = {}
        self.queries = {}
        self.steps = []

    def request_elems(self, req):
        return req.H * req.W

    def upload(self, req, block):
        self.pixels[req.rid] = np.asarray(req.pixels, np.float64)
        self.queries[req.rid] = 0
        req.codes = np.full((req.windows, self.K), -7.0)

    def uploaded(self, req):
        self.queries[req.rid] += 1
        return self.queries[req.rid] > self.upload_lag

    @staticmethod
    def code_window(win, K):
        s = win.sum()
        return np.array([s * (j + 1) + win[0, 0] for j in range(K)])

    def launch(self, chunks):
        n = sum(c.rows * (c.req.W - self.N + 1) for c in chunks)
        if self.capacity is not None and n > self.capacity:
            raise ValueError(f"step of {n} windows exceeds the slot capacity {self.capacity}")
        self.steps.append(n)
        for c in chunks:
            img = self.pixels[c.req.rid]
            wc = c.req.W - self.N + 1
            for y in range(c.y0, c.y0 + c.rows):
                for x in range(wc):
                    c.req.codes[y * wc + x] = self.code_window(img[y:y + self.N, x:x + self.N], self.K)
        return {"left": self.lag}

    def finished(self, tok):
        tok["left"] -= 1
        return tok["left"] < 0

    def wait(self, tok):
        pass


def alone(be, img):
    N = be.N
    H, W = img.shape
    out = []
    for y in range(H - N + 1):
        for x in range(W - N + 1):
            out.append(FakeBackend.code_window(img[y:y + N, x:x + N], be.K))
    return np.array(out).reshape(-1, be.K)


def make_requests(n, seed=0, lo=1, hi=40):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        H, W = rng.integers(lo, hi, 2)
        reqs.append(serve.Request(i, 0.0, rng.standard_normal((H, W)), int(H), int(W)))
    return reqs


def test_every_window_coded_once_and_equal_alone():
    be = FakeBackend(lag=2, upload_lag=1, capacity=300)
    sch = serve.Scheduler(be, budget_elems=10_000, step_windows=300, clock=lambda: 0.0)
    reqs = make_requests(40)
    for r in reqs:
        sch.submit(r)
    sch.drain(len(reqs))
    assert len(sch.finished) == len(reqs)
    for r in reqs:
        if r.windows:
            assert np.array_equal(r.codes, alone(be, r.pixels))
        assert r.done_rows == max(r.H - be.N + 1, 0) or r.windows == 0
    assert sch.arena.used == 0
    assert max(be.steps) <= 300                  # never past the step size


@pytest.mark.parametrize("step,shapes", [
    (2100, [(200, 114), (20, 2048)]),        # wide rows that used to overshoot the step
    (3000, [(20, 4000)]),                    # one row wider than a step: rejected
    (50, [(9, 40), (9, 45), (12, 50), (5, 52)]),
])
def test_steps_never_exceed_the_slot_capacity(step, shapes):
    be = FakeBackend(N=3, lag=1, capacity=step)
    sch = serve.Scheduler(be, budget_elems=10**7, step_windows=step, clock=lambda: 0.0)
    rng = np.random.default_rng(5)
    reqs = [serve.Request(i, 0.0, rng.standard_normal(s), s[0], s[1]) for i, s in enumerate(shapes)]
    for r in reqs:
        sch.submit(r)
    sch.drain(len(reqs))
    wide = {r.rid for r in reqs if r.W - be.N + 1 > step}
    assert {r.rid for r in sch.rejected} == wide
    assert max(be.steps, default=0) <= step
    for r in reqs:
        if r.rid not in wide:
            assert np.array_equal(r.codes, alone(be, r.pixels))


def test_admission_respects_budget_and_order():
    be = FakeBackend(lag=3)
    budget = 2_000
    sch = serve.Scheduler(be, budget_elems=budget, step_windows=500, clock=lambda: 0.0)
    reqs = make_requests(30, seed=1, lo=10, hi=40)
    big = serve.Request(99, 0.0, np.zeros((60, 60)), 60, 60)     # 3,600 > budget: rejected
    for r in reqs[:10] + [big] + reqs[10:]:
        sch.submit(r)
    peak = 0
    admitted_order = []
    while len(sch.finished) + len(sch.rejected) < 31:
        sch.poll()
        peak = max(peak, sch.arena.used)
        for r in sch.active:
            if r.rid not in admitted_order:
                admitted_order.append(r.rid)
    assert peak <= budget
    assert [r.rid for r in sch.rejected] == [99]
    assert admitted_order == sorted(admitted_order)              # arrival order kept
    for r in reqs:
        assert np.array_equal(r.codes, alone(be, r.pixels))


def test_small_requests_not_blocked_by_a_huge_one():
    be = FakeBackend(lag=0)
    sch = serve.Scheduler(be, budget_elems=10**6, step_windows=400, clock=lambda: 0.0)
    huge = serve.Request(0, 0.0, np.zeros((400, 400)), 400, 400)
    small = [serve.Request(i, 0.0, np.ones((5, 6)), 5, 6) for i in range(1, 6)]
    sch.submit(huge)
    for r in small:
        sch.submit(r)
    order = []
    while len(sch.finished) < 6:
        sch.poll()
        for r in sch.finished:
            if r.rid not in order:
                order.append(r.rid)
    assert order[-1] == 0                                         # the huge one finishes last
    assert set(order[:5]) == {1, 2, 3, 4, 5}


def test_arena_first_fit_and_merge():
    a = serve.Arena(1000, align=10)
    b1, b2, b3 = a.alloc(95), a.alloc(200), a.alloc(300)
    assert b1 == (0, 100) and b2 == (100, 200) and b3 == (300, 300)
    assert a.alloc(500) is None
    a.release(b2)
    a.release(b1)
    assert a.free[0] == (0, 300)
    assert a.alloc(250) == (0, 250)
    a.release((0, 250))
    a.release(b3)
    assert a.free == [(0, 1000)] and a.used == 0


def test_latency_report_and_replay():
    t = [0.0]
    be = FakeBackend(lag=0)
    sch = serve.Scheduler(be, budget_elems=10**6, step_windows=1000, clock=lambda: t[0])
    reqs = make_requests(5, seed=3)
    for i, r in enumerate(reqs):
        r.arrival = 0.1 * i
        sch.submit(r)
        t[0] = 0.1 * i
        sch.poll()
        t[0] += 0.05
        sch.poll()
    sch.drain(len(reqs))
    rep = serve.latency_report(reqs)
    assert rep["requests"] == 5 and rep["p99_s"] >= rep["p50_s"] >= 0


def test_wide_request_not_starved_by_a_stream_of_small_ones():
    be = FakeBackend(N=3, lag=0, capacity=100)
    sch = serve.Scheduler(be, budget_elems=10**7, step_windows=100, clock=lambda: 0.0)
    wide = serve.Request(0, 0.0, np.ones((12, 92)), 12, 92)        # 10 rows of 90 windows
    sch.submit(wide)
    rid = 1
    for _ in range(200):                                          # a new small request every round
        sch.submit(serve.Request(rid, 0.0, np.ones((6, 8)), 6, 8))
        rid += 1
        sch.poll()
        if wide in sch.finished:
            break
    assert wide in sch.finished
    assert sch.steps <= 40                                        # served at least every other step
    assert max(be.steps) <= 100
