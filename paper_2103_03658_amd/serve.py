"""Serving loop: continuous batching of fractional-Poisson solve requests.

Requests arrive over time (each: d, N, alpha, degree, right-hand sides).  A
pool of worker threads drives the GPU: each worker takes the oldest queued
request whose operator is idle, merges every other queued request for the
same operator (up to `max_batch_rhs` right-hand sides) into one batched
fl_solve, and returns each request's solution.  Different operators are
solved concurrently (each operator runs on its own HIP stream, so kernels
from several requests overlap on the device).

* Operator cache: operators (weights, generator, symbol and their solver
  buffers) are kept by key (d, N, alpha, degree, kernel) and evicted least
  recently used when the cache exceeds its byte budget (by default the free
  device memory less the in-flight budget); evicted operators are closed
  outside the server's lock.
* Admission by HBM footprint: a request is dispatched only while the
  estimated device bytes of all in-flight batches plus its own fit in
  `hbm_budget`; a request that can never fit is rejected.
* Per request: latency (arrival to completion), queueing time, batch size,
  iterations and final FP64 relative residual.
* Precision: FP64 PCG by default (`mixed=1` selects FP32 CG with FP64
  reliable updates); on the serving stream (N = 64 ... 512) FP64 has the
  lower latency, since the mixed path's extra iterations and reliable steps
  outweigh its cheaper passes at these sizes.
* Warm-up: with `warm` shapes, each worker first solves one right-hand side
  of each shape on its own stream (first kernel launches, its thread's and
  stream's first library calls), and the server takes requests only once
  every worker is done; `warmup_s` reports the time it took.

The solver and every kernel are the library's (fl_solve through the C ABI);
this module only schedules.  ctypes releases the GIL during library calls,
so the worker threads run the GPU concurrently.
"""

import collections
import threading
import time

import numpy as np


def op_bytes(d, N):
    """Device bytes an operator holds without solver buffers: the generator
    (FP64) and the symbol and its inverse in FP64 and FP32, each (N + 1)^d
    values on a cube."""
    return (N + 1) ** d * (8 + 2 * (8 + 4))


def batch_bytes(d, N, nrhs):
    """Device bytes of the solver buffers of a solve (FP64 or mixed) of nrhs
    right-hand sides (transform workspace, vectors, reduction partials)."""
    n, M = N - 1, 2 * N
    nd = n ** d
    h = M // 2 + 1
    ws = (h * n if d == 2 else (h * n * n + h * M * n if d == 3 else 0)) * 16 * nrhs
    vecs = nd * nrhs * (3 * 8 + 5 * 4)
    io = nd * nrhs * 8 * 2            # caller's f and u
    part = 2 * 8192 * 8 * nrhs * 2
    return ws + vecs + io + part


class Request:
    __slots__ = ("id", "d", "N", "alpha", "degree", "kernel", "lam", "f", "t_arrive",
                 "t_dispatch", "t_done", "u", "info", "batch_rhs", "status", "cache_hit")

    def __init__(self, rid, d, N, alpha, degree, f, t_arrive=0.0, kernel="fractional", lam=0.0):
        self.id, self.d, self.N, self.alpha, self.degree = rid, d, N, alpha, degree
        self.kernel, self.lam, self.f, self.t_arrive = kernel, lam, f, t_arrive
        self.t_dispatch = self.t_done = None
        self.u = self.info = None
        self.batch_rhs = 0
        self.status = "queued"
        self.cache_hit = None

    @property
    def key(self):
        return (self.d, self.N, round(self.alpha, 12), self.degree, self.kernel, self.lam)

    @property
    def nrhs(self):
        return int(self.f.shape[0])


class Server:
    def __init__(self, workers=4, hbm_budget=64 << 30, cache_bytes=None, max_batch_rhs=64,
                 tol=1e-10, mixed=0, maxiter=20000, keep_solutions=False, device=0, warm=(),
                 graphs=1):
        self.workers = workers
        # HIP graphs of the operators' CG chunks (fl_set_graphs mode): 1
        # captures a chunk at its first run; 2 at its second, so that an
        # operator solved once never pays for capture (on the 4096-request
        # stream the two measured the same within run-to-run spread)
        self.graphs = graphs
        self.warm = list(warm)                     # (d, N, degree) solved once per worker
        self._warmed = threading.Barrier(workers + 1)
        self.hbm_budget = hbm_budget
        if cache_bytes is None:
            cache_bytes = self.default_cache_bytes(device, hbm_budget)
        self.cache_bytes = cache_bytes
        self.max_batch_rhs = max_batch_rhs
        self.tol, self.mixed, self.maxiter = tol, mixed, maxiter
        # True: keep every request's solution; a set of request ids: keep those
        self.keep = keep_solutions
        self.device = device
        self._cv = threading.Condition()
        self._queue = collections.deque()
        self._busy = set()
        self._inflight = 0
        self._ops = collections.OrderedDict()      # key -> (Operator, bytes)
        self._cached = 0
        self._arrivals_done = False
        self.done = []
        self.rejected = []
        self.admission_waits = 0
        self.batches = []
        self.errors = []

    # -- operator cache -------------------------------------------------------
    @staticmethod
    def default_cache_bytes(device, hbm_budget):
        """Operator cache budget: three quarters of the device memory free at
        start-up less the in-flight budget (about 150 GB on a 288 GB device),
        at least 4 GiB.  Evicting an operator frees device memory, which waits
        for every stream of the device, so a cache that holds the working set
        keeps those waits out of the serving loop."""
        import torch
        free, _ = torch.cuda.mem_get_info(device)
        return max(4 << 30, int(0.75 * free) - hbm_budget)

    def _get_op(self, req, nrhs):
        import paper_2103_03658_amd as fl
        k = req.key
        with self._cv:
            if k in self._ops:
                self._ops.move_to_end(k)
                op, b = self._ops[k]
                need = op_bytes(req.d, req.N) + batch_bytes(req.d, req.N, nrhs)
                if need > b:
                    self._cached += need - b
                    self._ops[k] = (op, need)
                return op, True
        op = fl.Operator(req.d, req.alpha, req.degree, N=req.N, kernel=req.kernel, lam=req.lam)
        if self.graphs != 1:     # 1 is the library's default
            op.set_graphs(self.graphs)
        b = op_bytes(req.d, req.N) + batch_bytes(req.d, req.N, nrhs)
        with self._cv:
            self._ops[k] = (op, b)
            self._cached += b
            gone = self._evict_locked()
        self._close(gone)
        return op, False

    def _evict_locked(self):
        """Drop least recently used idle operators until the cache fits its
        budget; returns them for _close, which runs outside the lock (freeing
        device memory waits for the whole device, and other workers must not
        wait for the lock meanwhile)."""
        gone = []
        for k in list(self._ops):
            if self._cached <= self.cache_bytes:
                break
            if k in self._busy:
                continue
            op, b = self._ops.pop(k)
            self._cached -= b
            gone.append(op)
        return gone

    @staticmethod
    def _close(ops):
        for op in ops:
            op.close()

    # -- scheduling -----------------------------------------------------------
    def submit(self, req):
        with self._cv:
            need = op_bytes(req.d, req.N) + batch_bytes(req.d, req.N, req.nrhs)
            if need > self.hbm_budget:
                req.status = "rejected"
                self.rejected.append(req)
            else:
                self._queue.append(req)
            self._cv.notify_all()

    def _take_locked(self):
        """Oldest queued request with an idle operator, plus queued requests
        for the same operator; None if nothing can start now."""
        blocked_by_memory = False
        for i, req in enumerate(self._queue):
            if req.key in self._busy:
                continue
            group, rhs = [req], req.nrhs
            for other in list(self._queue)[i + 1:]:
                if other.key == req.key and rhs + other.nrhs <= self.max_batch_rhs:
                    group.append(other)
                    rhs += other.nrhs
            need = op_bytes(req.d, req.N) + batch_bytes(req.d, req.N, rhs)
            if self._inflight + need > self.hbm_budget:
                blocked_by_memory = True
                continue
            for g in group:
                self._queue.remove(g)
            self._busy.add(req.key)
            self._inflight += need
            return group, need
        if blocked_by_memory:
            self.admission_waits += 1
        return None

    def _tensor_device(self):
        return f"cuda:{self.device}"

    def _open_stream(self):
        """The worker's own stream on the server's device."""
        import torch
        torch.cuda.set_device(self.device)
        return torch.cuda.Stream()

    def _worker(self):
        stream = self._open_stream()
        try:
            self._warm_up(stream)
        except Exception as exc:
            self.errors.append(f"warm-up: {exc!r}")
        finally:
            self._warmed.wait()
        while True:
            with self._cv:
                item = None
                while item is None:
                    item = self._take_locked()
                    if item is None:
                        if self._arrivals_done and not self._queue:
                            return
                        self._cv.wait(0.05)
            group, need = item
            try:
                self._run_batch(group, stream)
            except Exception as exc:  # a failed batch fails its requests
                for r in group:
                    r.status = f"error: {exc}"
                self.errors.append(repr(exc))
            finally:
                with self._cv:
                    self._busy.discard(group[0].key)
                    self._inflight -= need
                    self.done.extend(group)
                    gone = self._evict_locked()
                    self._cv.notify_all()
                self._close(gone)

    def _warm_up(self, stream):
        import torch
        import paper_2103_03658_amd as fl
        for d, N, degree in self.warm:
            op = fl.Operator(d, 1.0, degree, N=N)
            f = torch.ones((1,) + (N - 1,) * d, dtype=torch.float64,
                           device=self._tensor_device())
            with torch.cuda.stream(stream):
                op.solve(f, tol=self.tol, mixed=self.mixed, maxiter=self.maxiter,
                         stream=stream, raise_on_fail=False)
            op.close()

    def _run_batch(self, group, stream):
        import torch
        t0 = time.perf_counter()
        rhs = sum(r.nrhs for r in group)
        op, hit = self._get_op(group[0], rhs)
        with torch.cuda.stream(stream):
            f = torch.cat([r.f for r in group]).contiguous() if len(group) > 1 else group[0].f
            u, info = op.solve(f, tol=self.tol, mixed=self.mixed, maxiter=self.maxiter,
                               stream=stream, raise_on_fail=False)
            # copies on the worker stream, where u was allocated and written:
            # the allocator may hand u's block to the next batch on this
            # stream as soon as u is dropped
            kept = []
            if self.keep:
                off = 0
                for r in group:
                    kept.append(u[off:off + r.nrhs].clone() if self._keeps(r) else None)
                    off += r.nrhs
        t1 = time.perf_counter()
        self.batches.append((len(group), rhs, t1 - t0, group[0].N))
        off = 0
        for k, r in enumerate(group):
            r.t_dispatch = t0
            r.t_done = t1
            r.cache_hit = hit
            r.batch_rhs = rhs
            r.info = info[off:off + r.nrhs]
            if self.keep and kept[k] is not None:
                r.u = kept[k]
            r.status = "ok" if all(i["converged"] for i in r.info) else "noconv"
            off += r.nrhs

    def _keeps(self, r):
        return self.keep is True or (not isinstance(self.keep, bool) and r.id in self.keep)

    # -- driver ---------------------------------------------------------------
    def run(self, requests, realtime=True):
        """Feed requests (sorted by t_arrive) and serve until all are done.
        realtime: arrivals follow t_arrive on the wall clock; otherwise all
        arrive at once.  Returns a statistics dict."""
        threads = [threading.Thread(target=self._worker, daemon=True)
                   for _ in range(self.workers)]
        t_warm = time.perf_counter()
        for t in threads:
            t.start()
        self._warmed.wait()
        start = time.perf_counter()
        self.warmup_s = start - t_warm
        for req in requests:
            if realtime:
                delay = start + req.t_arrive - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            req.t_arrive = time.perf_counter()
            self.submit(req)
        with self._cv:
            self._arrivals_done = True
            self._cv.notify_all()
        for t in threads:
            t.join()
        end = time.perf_counter()
        self.device_bytes_in_use = self._device_bytes_in_use()
        return self.stats(start, end)

    def _device_bytes_in_use(self):
        """Device memory in use (operator cache included) at the end of a run."""
        import torch
        free, total = torch.cuda.mem_get_info(self.device)
        return total - free

    def stats(self, start, end):
        ok = [r for r in self.done if r.status == "ok"]
        lat = np.array([r.t_done - r.t_arrive for r in self.done if r.t_done]) * 1e3
        qwait = np.array([r.t_dispatch - r.t_arrive for r in self.done if r.t_dispatch]) * 1e3
        rhs = sum(r.nrhs for r in self.done if r.t_done)
        hits = [r.cache_hit for r in self.done if r.cache_hit is not None]
        worst = max((i["relres_true"] for r in self.done if r.info for i in r.info),
                    default=0.0)
        return {
            "requests": len(self.done) + len(self.rejected),
            "served": len(self.done), "ok": len(ok), "rejected": len(self.rejected),
            "wall_s": end - start,
            "warmup_s": getattr(self, "warmup_s", None),
            "rhs_solves_per_s": rhs / (end - start),
            "requests_per_s": len(self.done) / (end - start),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "queue_p50_ms": float(np.percentile(qwait, 50)) if len(qwait) else None,
            "cache_hit_rate": float(np.mean(hits)) if hits else None,
            "batches": len(self.batches),
            "mean_requests_per_batch": float(np.mean([b[0] for b in self.batches]))
            if self.batches else None,
            "admission_waits": self.admission_waits,
            "operators_cached": len(self._ops),
            "device_gb_in_use_at_end": getattr(self, "device_bytes_in_use", 0) / 1e9,
            "max_relres_true": worst,
            "errors": self.errors[:5],
        }
