"""Scheduling logic of the serving loop on the CPU, with the library replaced
by a stand-in whose "solution" is a known function of each request's sources:
every request gets its own result, requests that arrive while others are
being solved join the running batch (continuous batching), the resident
footprint never exceeds the budget, idle operators are evicted least
recently used first, and a context is destroyed before the next one is
built.  No GPU and no library calls."""
import threading
import time
import types

import numpy as np
import pytest

from paper_2304_01728_amd import serving


class FakeLib:
    DPG_MIXED, DPG_FP64, DPG_OK = 1, 0, 0

    def __init__(self, nbytes_per_element=1000, solve_s=0.02):
        self.lock = threading.Lock()
        self.live = {}            # ctx id -> bytes
        self.peak = 0
        self.events = []
        self.per = nbytes_per_element
        self.solve_s = solve_s
        self.batches = []         # running columns at every batch iteration
        self.adds = 0
        self.next_id = 0

    # --- the calls the server makes ---
    def dpg_default_options(self, **kw):
        return kw

    def dpg_setup(self, N, p, omega, loads, dp=1, c=None, options=None):
        with self.lock:
            self.next_id += 1
            ctx = types.SimpleNamespace(id=self.next_id, N=N, loads=None, lib=self)
            ctx.close = lambda ctx=ctx: self._close(ctx)
            self.live[ctx.id] = self.per * N ** 3
            self.peak = max(self.peak, sum(self.live.values()))
            self.events.append(("build", N))
            return ctx

    def _close(self, ctx):
        with self.lock:
            self.live.pop(ctx.id, None)
            self.events.append(("close", ctx.N))

    def dpg_assemble(self, ctx):
        pass

    def dpg_build_hierarchy(self, ctx):
        pass

    def dpg_release_setup(self, ctx):
        pass

    def dpg_info(self, ctx):
        return types.SimpleNamespace(resident_bytes=self.per * ctx.N ** 3)

    def dpg_load_rhs(self, ctx, loads, want=True):
        ctx.loads = loads

    # a batch: slot -> [load, iterations left]; each step is one iteration
    def dpg_batch_open(self, ctx, slots):
        ctx.nslots, ctx.cols, ctx.done = slots, {}, []

    def dpg_batch_add(self, ctx, rhs=None, load_col=0, tol=1e-8):
        k = min(set(range(ctx.nslots)) - set(ctx.cols))
        ld = ctx.loads[load_col]
        ctx.cols[k] = [ld, 3 + int(ld["sources"].shape[0])]
        with self.lock:
            self.adds += 1
        return k

    def dpg_batch_step(self, ctx, max_iters):
        for _ in range(max_iters):
            running = [k for k, c in ctx.cols.items() if c[1] > 0]
            if not running:
                break
            time.sleep(self.solve_s / 5)
            with self.lock:
                self.batches.append(len(running))
            fin = []
            for k in running:
                ctx.cols[k][1] -= 1
                if ctx.cols[k][1] == 0:
                    fin.append(k)
            ctx.done += fin
            if fin:
                break
        return list(ctx.done)

    def dpg_batch_take(self, ctx, k):
        ld, _ = ctx.cols.pop(k)
        ctx.done.remove(k)
        return np.array([ld["sources"].sum() + ctx.N]), 5, 1e-9, 0

    def dpg_batch_close(self, ctx):
        ctx.cols = {}


def _ops():
    return [serving.Operator(k, N, 2, 1.0) for k, N in enumerate([4, 6, 8])]


def _reqs(n, gap, seed=0):
    rng = np.random.default_rng(seed)
    return [serving.Request(i, int(rng.integers(3)), rng.uniform(0, 1, size=(int(rng.integers(1, 5)), 6)),
                            gap * i) for i in range(n)]


@pytest.fixture
def fake(monkeypatch):
    lib = FakeLib()
    monkeypatch.setattr(serving, "D", lib)
    return lib


def test_every_request_gets_its_own_result(fake):
    ops = _ops()
    srv = serving.Server(ops, budget_bytes=1 << 40, max_active=2)
    reqs = _reqs(40, 0.001)
    try:
        wall, lat = serving.run_stream(srv, reqs)
    finally:
        srv.close()
    N = {op.key: op.N for op in ops}
    for r in reqs:
        assert r.x[0] == pytest.approx(r.sources.sum() + N[r.op_key])
    assert len(lat) == 40 and np.all(lat > 0)
    assert max(fake.batches) > 1                  # requests joined running batches
    assert fake.adds == 40
    assert srv.builds == 3 and srv.evictions == 0
    assert not fake.live                          # every context destroyed on close


def test_late_request_joins_the_running_batch(fake):
    """One operator: the second request arrives while the first is part-way
    through its iterations and joins it; it finishes before a solve that waited
    for the whole batch could have started."""
    ops = _ops()[:1]
    srv = serving.Server(ops, budget_bytes=1 << 40, max_active=1)
    src = np.ones((12, 6))
    a = serving.Request(0, 0, src, 0.0)             # 15 iterations of solve_s / 5
    b = serving.Request(1, 0, src[:1], 0.012)       # 4 iterations, arrives mid-way
    try:
        serving.run_stream(srv, [a, b])
    finally:
        srv.close()
    assert b.batch == 2 and a.batch == 2
    assert b.t_done < a.t_done                      # left the batch before the first
    assert b.x[0] == pytest.approx(src[:1].sum() + ops[0].N)


def test_budget_is_respected_with_eviction(fake):
    ops = _ops()
    budget = fake.per * (8 ** 3 + 4 ** 3)         # room for N = 8 and N = 4, not N = 6 too
    srv = serving.Server(ops, budget_bytes=budget, max_active=2)
    srv.estimate = lambda op: fake.per * op.N ** 3
    reqs = _reqs(30, 0.01, seed=1)
    try:
        serving.run_stream(srv, reqs)
    finally:
        srv.close()
    assert fake.peak <= budget
    assert srv.evictions >= 1
    # a build never happens while the evicted context is still alive beyond the budget
    held, limit = 0, budget
    for ev, N in fake.events:
        held += fake.per * N ** 3 if ev == "build" else -fake.per * N ** 3
        assert held <= limit


def test_single_operator_larger_than_budget_still_runs(fake):
    ops = _ops()
    srv = serving.Server(ops, budget_bytes=1, max_active=1)
    reqs = _reqs(9, 0.0, seed=2)
    try:
        serving.run_stream(srv, reqs)
    finally:
        srv.close()
    assert all(r.x is not None for r in reqs)
    assert not fake.live


def test_layered_speed_assigns_z_layers():
    c = serving.layered_speed(4, (0.25, 0.5, 0.75), (1.0, 2.0, 3.0, 4.0))
    assert c.shape == (64,)
    # element e = i + 4 (j + 4 k): layer by k
    for e in range(64):
        assert c[e] == [1.0, 2.0, 3.0, 4.0][e // 16]


def test_pool_and_requests_are_seeded():
    a = serving.draw_pool(seed=4)
    b = serving.draw_pool(seed=4)
    assert [(o.N, o.p, o.omega) for o in a] == [(o.N, o.p, o.omega) for o in b]
    for o in a:
        h = 1.0 / o.N
        assert o.omega == pytest.approx(2 * np.pi * o.c.min() / (5 * h))
        assert 1.0 <= o.c.min() and o.c.max() <= 4.0 and len(np.unique(o.c)) <= 4
    r = serving.draw_requests(a, 50, rate=10.0, seed=4)
    t = np.array([q.t_arrival for q in r])
    assert np.all(np.diff(t) > 0)
    assert all(1 <= len(q.sources) <= 16 for q in r)
