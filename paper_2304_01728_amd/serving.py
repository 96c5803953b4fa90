"""Continuous-batching solve server over resident DPG multigrid hierarchies.

A request names an operator (mesh size N, order p, frequency, layered wave
speed) and carries one to sixteen Gaussian point sources.  The server

* keeps one library context (assembled element matrices and multigrid
  hierarchy) per operator resident on the GPU while the HBM budget allows,
  admitting an operator by its footprint and evicting the least recently
  used idle one when room is needed;
* gives each resident operator a host worker thread and the context its own
  stream, so that solves of different operators overlap on the device (the
  library releases the interpreter lock inside its calls);
* runs every operator's solves as one continuous batch (dpg_batch_*): a
  request that arrives while others are being solved joins the running
  block solve at the next iteration, in a free column slot (up to 32), and
  leaves it as soon as its own column converges, so no request waits for a
  whole batch to finish.  Each column keeps its own CG recurrence, so a
  request's result is the same alone and in the mix.

Latency is measured from a request's arrival to its result on the host.
Every step of a solve runs in the library's kernels; this module only
schedules calls to it.
"""
import collections
import math
import threading
import time

import numpy as np

from . import dpgmg as D

MAX_BATCH = 32      # column slots of a batch in the library


class Operator:
    """Problem data of one operator: N^3 mesh of the unit cube, order p, omega,
    wave speed per element (c), precision and tolerance of its solves."""

    def __init__(self, key, N, p, omega, c=None, precision="mixed", tol=1e-8, dp=1):
        self.key, self.N, self.p, self.omega, self.dp = key, N, p, omega, dp
        self.c = None if c is None else np.ascontiguousarray(np.asarray(c, dtype=float))
        self.precision, self.tol = precision, tol

    def build(self, batch_slots=0):
        """Context with its hierarchy; with batch_slots > 0 a batch of that many
        column slots is opened on it (its buffers count in the footprint)."""
        opt = D.dpg_default_options(
            precision=D.DPG_MIXED if self.precision == "mixed" else D.DPG_FP64)
        ctx = D.dpg_setup(self.N, self.p, self.omega, [dict(dir=(0.0, 0.0, 1.0), amp=0.0)],
                          dp=self.dp, c=self.c, options=opt)
        D.dpg_assemble(ctx)
        D.dpg_build_hierarchy(ctx)
        D.dpg_release_setup(ctx)   # keep only what solves and new loads need
        if batch_slots > 0:
            D.dpg_batch_open(ctx, batch_slots)
        return ctx


def layered_speed(N, interfaces, speeds):
    """Wave speed per element (e = i + N (j + N k)) of a medium in z-layers:
    layer l holds the elements whose centre lies between interfaces l-1 and l."""
    zc = (np.arange(N) + 0.5) / N
    layer = np.searchsorted(np.sort(np.asarray(interfaces, dtype=float)), zc)
    ck = np.asarray(speeds, dtype=float)[layer]
    return np.repeat(ck, N * N)


class Request:
    def __init__(self, rid, op_key, sources, t_arrival=0.0):
        self.rid, self.op_key, self.t_arrival = rid, op_key, t_arrival
        self.sources = np.asarray(sources, dtype=float).reshape(-1, 6)
        self.x = None
        self.iters = None
        self.relres = None
        self.status = None
        self.t_done = None
        self.batch = 0               # most columns its batch ran while it was in it
        self.joined_running = False  # admitted while other requests were part-way through
        self.error = None
        self.done = threading.Event()

    def load(self):
        return dict(dir=(0.0, 0.0, 1.0), amp=0.0, sources=self.sources)


class _Resident:
    def __init__(self, op, ctx, nbytes):
        self.op, self.ctx, self.nbytes = op, ctx, nbytes
        self.pending = collections.deque()
        self.busy = False
        self.last_used = time.perf_counter()
        self.stop = False
        self.thread = None


class Server:
    """budget_bytes: device memory the resident contexts may hold together.
    max_active: operators whose batches step on the device at once.
    max_batch: column slots of each operator's batch.  step_iters: block PCG
    iterations between two looks at the queue (admissions happen there)."""

    def __init__(self, operators, budget_bytes, max_active=8, max_batch=8, step_iters=1):
        self.ops = {op.key: op for op in operators}
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.step_iters = step_iters
        self.cv = threading.Condition()
        self.slots = threading.Semaphore(max_active)
        self.resident = {}
        self.waiting = collections.deque()   # requests of operators not admitted yet
        self.bytes_per_element = {}          # (p, precision) -> largest seen
        self.builds = 0
        self.evictions = 0
        self.closed = False
        self.error = None
        self.admitter = threading.Thread(target=self._admit_loop, daemon=True)
        self.admitter.start()

    # ---- footprint ----------------------------------------------------------------------
    def estimate(self, op):
        """A-priori footprint: the largest bytes per element seen for this
        order and precision, else a conservative default per order."""
        default = {2: 0.6e6, 3: 1.6e6, 4: 4.0e6}.get(op.p, 6.0e6)
        if op.precision == "mixed":
            default *= 0.8
        per = self.bytes_per_element.get((op.p, op.precision), default)
        return int(per * op.N ** 3) + (256 << 20)

    def _held(self):
        return sum(r.nbytes for r in self.resident.values())

    # ---- requests -----------------------------------------------------------------------
    def submit(self, req):
        with self.cv:
            if self.closed:
                raise RuntimeError("server closed")
            res = self.resident.get(req.op_key)
            if res is not None:
                res.pending.append(req)
            else:
                self.waiting.append(req)
            self.cv.notify_all()

    def _admit_loop(self):
        """Admits the operators of waiting requests in arrival order, evicting
        idle operators (least recently used first) to make room; an evicted
        context is destroyed before the next one is built."""
        while True:
            victims = []
            admit = None
            with self.cv:
                while not self.closed and not self.waiting:
                    self.cv.wait()
                if self.closed:
                    return
                req = self.waiting[0]
                res = self.resident.get(req.op_key)
                if res is not None:           # admitted meanwhile
                    self.waiting.popleft()
                    res.pending.append(req)
                    self.cv.notify_all()
                    continue
                op = self.ops[req.op_key]
                need = self.estimate(op)
                while self._held() + need > self.budget:
                    idle = [r for r in self.resident.values() if not r.busy and not r.pending]
                    if not idle:
                        break
                    victim = min(idle, key=lambda r: r.last_used)
                    self._evict(victim)
                    victims.append(victim)
                if self._held() + need <= self.budget or not self.resident:
                    admit = _Resident(op, None, need)
                    admit.busy = True
                    self.resident[op.key] = admit
                    for r in [r for r in self.waiting if r.op_key == op.key]:
                        self.waiting.remove(r)
                        admit.pending.append(r)
                elif not victims:
                    self.cv.wait(0.01)        # wait until a resident operator falls idle
            for v in victims:
                v.thread.join()
            if admit is None:
                continue
            try:
                ctx = op.build(self.max_batch)
                nbytes = D.dpg_info(ctx).resident_bytes
            except Exception as exc:          # reported on every request of this operator
                with self.cv:
                    self.resident.pop(op.key, None)
                    for r in admit.pending:
                        r.error = exc
                        r.done.set()
                    self.cv.notify_all()
                continue
            with self.cv:
                self.builds += 1
                kp = (op.p, op.precision)
                self.bytes_per_element[kp] = max(self.bytes_per_element.get(kp, 0.0),
                                                 nbytes / op.N ** 3)
                admit.ctx, admit.nbytes = ctx, nbytes
                admit.busy = False
                admit.thread = threading.Thread(target=self._worker, args=(admit,), daemon=True)
                admit.thread.start()
                self.cv.notify_all()

    def _evict(self, res):
        res.stop = True
        self.resident.pop(res.op.key, None)
        self.evictions += 1
        self.cv.notify_all()

    def _worker(self, res):
        ctx = res.ctx                  # built with a batch of max_batch slots open
        slots = {}                     # batch slot -> request being solved
        while True:
            with self.cv:
                while not res.stop and not res.pending and not slots:
                    self.cv.wait()
                if res.stop and not res.pending and not slots:
                    break
                free = self.max_batch - len(slots)
                new = [res.pending.popleft() for _ in range(min(free, len(res.pending)))]
                res.busy = True
            finished = []
            self.slots.acquire()
            try:
                if new:
                    # the loads of the newcomers, then each joins the running batch
                    D.dpg_load_rhs(ctx, [r.load() for r in new], want=False)
                    running = bool(slots)
                    for j, r in enumerate(new):
                        r.joined_running = running
                        slots[D.dpg_batch_add(ctx, None, load_col=j, tol=res.op.tol)] = r
                for r in slots.values():
                    r.batch = max(r.batch, len(slots))
                for k in D.dpg_batch_step(ctx, self.step_iters):
                    x, it, rel, code = D.dpg_batch_take(ctx, k)
                    finished.append((slots.pop(k), x.copy(), it, rel, code, None))
            except Exception as exc:   # reported on every request of the batch
                finished += [(r, None, None, None, None, exc) for r in slots.values()]
                slots.clear()
                D.dpg_batch_open(ctx, self.max_batch)
            finally:
                self.slots.release()
            t = time.perf_counter()
            with self.cv:
                for r, x, it, rel, code, err in finished:
                    if err is None:
                        r.x, r.iters, r.relres, r.status = x, int(it), float(rel), code
                    else:
                        r.error = err
                    r.t_done = t
                    r.done.set()
                res.busy = bool(slots)
                res.last_used = t
                self.cv.notify_all()
        D.dpg_batch_close(ctx)
        res.ctx = None
        ctx.close()

    def close(self):
        with self.cv:
            self.closed = True
            for r in list(self.resident.values()):
                r.stop = True
            self.cv.notify_all()
        self.admitter.join()
        for r in list(self.resident.values()):
            if r.thread is not None:
                r.thread.join()
        self.resident.clear()


def run_stream(server, requests):
    """Submits requests at their arrival times (seconds from now) and waits for
    all of them; returns (wall seconds, latencies in seconds)."""
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.t_arrival):
        delay = t0 + r.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        r.t_submit = time.perf_counter()
        server.submit(r)
    for r in requests:
        r.done.wait()
    wall = time.perf_counter() - t0
    errs = [r for r in requests if r.error is not None]
    if errs:
        raise RuntimeError(f"request {errs[0].rid} failed: {errs[0].error}")
    lat = np.array([r.t_done - r.t_submit for r in requests])
    return wall, lat


# ---- the layered-medium point-source stream -----------------------------------------------

def draw_pool(seed=4, n_ops=8, Ns=(8, 12, 16, 24, 32), ps=(2, 3, 4), precision="mixed",
              tol=1e-8):
    """Operators drawn once: N and p uniformly, three interfaces at distinct
    multiples of 1/8 (four z-layers), layer speeds U[1, 4], and omega giving
    five elements per shortest wavelength, omega = 2 pi c_min / (5 h)."""
    rng = np.random.default_rng(seed)
    ops = []
    for k in range(n_ops):
        N = int(rng.choice(Ns))
        p = int(rng.choice(ps))
        interfaces = np.sort(rng.choice(np.arange(1, 8), size=3, replace=False)) / 8.0
        speeds = rng.uniform(1.0, 4.0, size=4)
        omega = 2 * math.pi * speeds.min() / (5.0 / N)
        ops.append(Operator(k, N, p, omega, layered_speed(N, interfaces, speeds),
                            precision=precision, tol=tol))
    return ops


def draw_requests(ops, n_req, rate, seed=4, sigma=0.02, max_sources=16):
    """Poisson arrivals at `rate` per second; each request picks an operator
    and 1..max_sources sources with centres U[0.1, 0.9]^3 and unit amplitude."""
    rng = np.random.default_rng(seed + 1)
    t = 0.0
    reqs = []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        op = ops[int(rng.integers(len(ops)))]
        ns = int(rng.integers(1, max_sources + 1))
        c = rng.uniform(0.1, 0.9, size=(ns, 3))
        src = np.column_stack([c, np.full(ns, sigma), np.ones(ns), np.zeros(ns)])
        reqs.append(Request(i, op.key, src, t))
    return reqs


def percentile(lat, q):
    return float(np.percentile(lat, q)) if len(lat) else float("nan")
