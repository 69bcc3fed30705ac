"""Serving SAR scenes: continuous batching under an HBM budget.

Requests (one raw scene each, already on the device) arrive at any time.  The
HBM budget is one device region (an arena) of that many bytes, allocated once
when the server starts; every request is placed inside it, so the serving loop
never calls the device allocator and the budget is a hard limit.  A scheduler
thread admits requests in arrival order as soon as a slot (one HIP stream per
slot) is free and the arena can place the request's two blocks:

    image    8 bytes per pixel, held until the client releases the result;
    scratch  16 bytes per pixel (staging copy of the raw scene + workspace),
             held until the request's work has finished on the device.

Admitted requests run concurrently on their slots' streams, so a request that
arrives while others are on the GPU starts as soon as a slot and memory free
up, and its kernels overlap theirs (continuous batching, not a queue in front
of one stream).  When a request's work has finished its scratch block returns
to the arena and its future resolves with a Result whose image (a view into
the arena) stays valid until Result.release() or until the Result is garbage
collected.  A client must not release an image while work of its own that
reads it is still queued on the device.

The scheduling is independent of the device: an executor enqueues and polls
the work.  GpuExecutor runs each scene through libsar_rda.so
(sar_rda_execute on the slot's stream, plans cached per parameter set);
tests drive the same scheduler with a CPU executor that models durations.

Per-request errors (invalid parameters, a failed launch, a scene larger than
the whole budget) resolve that request's future with the exception and leave
the others untouched.  A request still on the device after ``timeout``
seconds has its future failed with ``TimeoutError``; its memory stays
allocated until the device work has really finished.
"""
from __future__ import annotations

import bisect
import collections
import concurrent.futures as cf
import dataclasses
import threading
import time
import weakref

import numpy as np

ALIGN = 256


class ServerError(RuntimeError):
    pass


class Arena:
    """First-fit allocator over [0, size) with a coalescing free list
    (thread-safe).  Offsets and sizes are multiples of ``align``.
    release_later() may be called from any thread at any time (also from a
    garbage-collection finalizer while the arena's lock is held): the block is
    queued and freed by the next operation."""

    def __init__(self, size: int, align: int = ALIGN):
        self.size = size // align * align
        self.align = align
        self._lock = threading.Lock()
        self._free_off = [0] if self.size else []      # sorted offsets of free blocks
        self._free_len = {0: self.size} if self.size else {}
        self._live: dict[int, int] = {}
        self._pending: collections.deque[int] = collections.deque()
        self._used = 0
        self._max_used = 0

    def _round(self, n: int) -> int:
        return max(self.align, (n + self.align - 1) // self.align * self.align)

    def _drain(self):
        while self._pending:
            self._free_locked(self._pending.popleft())

    def alloc(self, n: int):
        n = self._round(n)
        with self._lock:
            self._drain()
            for i, off in enumerate(self._free_off):
                ln = self._free_len[off]
                if ln < n:
                    continue
                del self._free_off[i]
                del self._free_len[off]
                if ln > n:
                    self._free_off.insert(i, off + n)
                    self._free_len[off + n] = ln - n
                self._live[off] = n
                self._used += n
                self._max_used = max(self._max_used, self._used)
                return off
        return None

    def free(self, off: int):
        with self._lock:
            self._drain()
            self._free_locked(off)

    def release_later(self, off: int):
        self._pending.append(off)

    def _free_locked(self, off: int):
        n = self._live.pop(off)
        self._used -= n
        i = bisect.bisect_left(self._free_off, off)
        if i < len(self._free_off) and self._free_off[i] == off + n:     # merge next
            n += self._free_len.pop(self._free_off.pop(i))
        if i > 0 and self._free_off[i - 1] + self._free_len[self._free_off[i - 1]] == off:
            self._free_len[self._free_off[i - 1]] += n                    # merge previous
        else:
            self._free_off.insert(i, off)
            self._free_len[off] = n

    @property
    def used(self) -> int:
        with self._lock:
            self._drain()
            return self._used

    @property
    def max_used(self) -> int:
        return self._max_used

    def live_blocks(self):
        with self._lock:
            self._drain()
            return sorted(self._live.items())

    def free_blocks(self):
        with self._lock:
            self._drain()
            return [(o, self._free_len[o]) for o in self._free_off]


def scene_blocks(cfg: dict) -> tuple[int, int]:
    """(image bytes, scratch bytes) of a request: complex64 image; staging
    copy of the raw scene plus the workspace (one complex64 scene, or for
    half storage two FP16 scenes and 4 (Na + Nr) bytes of exponents, each
    block 256-byte aligned)."""
    na, nr = int(cfg["Na"]), int(cfg["Nr"])
    px = na * nr
    return 8 * px, 16 * px + 4 * (na + nr) + 1024


def footprint_bytes(cfg: dict) -> int:
    return sum(scene_blocks(cfg))


class Result:
    """A finished request.  ``image`` lives in the server's arena until
    release() (or until this object is garbage collected)."""

    def __init__(self, rid, image, arrival, admitted, done, release_cb):
        self.id = rid
        self.image = image
        self.arrival = arrival
        self.admitted = admitted
        self.done = done
        self._fin = weakref.finalize(self, release_cb)

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queued(self) -> float:
        return self.admitted - self.arrival

    def release(self):
        """Return the image's memory to the arena (idempotent)."""
        self.image = None
        self._fin()


@dataclasses.dataclass
class Request:
    id: int
    cfg: dict
    raw: object
    precision: str
    arrival: float
    blocks: tuple
    future: cf.Future
    ready: object = None        # executor's marker: raw's producer has finished
    admitted: float = 0.0
    img_off: int = -1
    scratch_off: int = -1
    token: object = None
    timed_out: bool = False


class Server:
    """Continuous-batching server.

    hbm_budget: bytes of the arena all admitted requests live in.
    slots: requests that may be on the device at once (one stream each).
    executor: GpuExecutor(slots, hbm_budget) by default.
    timeout: seconds a request may stay on the device (None: no limit).
    on_result: called as on_result(result) in the scheduler thread when a
        request finishes, before its future resolves (e.g. to copy the image
        out and release it).
    """

    def __init__(self, hbm_budget: int, slots: int = 4, executor=None, timeout=None,
                 on_result=None, poll_interval: float = 20e-6):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.arena = Arena(int(hbm_budget))
        self.budget = self.arena.size
        self.slots = slots
        self.executor = executor if executor is not None else GpuExecutor(slots, self.budget)
        cap = getattr(self.executor, "capacity", None)
        if cap is not None and cap < self.budget:
            raise ValueError(f"executor arena of {cap} bytes is smaller than the budget")
        self.timeout = timeout
        self.on_result = on_result
        self.poll = poll_interval
        self._queue: collections.deque[Request] = collections.deque()
        self._inflight: dict[int, Request] = {}            # slot -> request
        self._free_slots = list(range(slots))[::-1]
        self._next_id = 0
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._closing = False
        self.max_concurrent = 0
        self.admission_order: list[int] = []
        self._thread = threading.Thread(target=self._loop, name="sar-server", daemon=True)
        self._thread.start()

    @property
    def max_used(self) -> int:
        return self.arena.max_used

    @property
    def used_bytes(self) -> int:
        return self.arena.used

    # ---- client side ----
    def submit(self, cfg: dict, raw, precision: str = "fp32") -> cf.Future:
        """Queue one scene; returns a future of Result.  ``raw`` is the
        scene's device tensor (Na, Nr) complex64; it is only read."""
        fut: cf.Future = cf.Future()
        now = time.perf_counter()
        blocks = scene_blocks(cfg)
        # taken in the caller's thread, on the caller's current stream: work
        # the client queued to fill raw is ordered before the request's copy
        prepare = getattr(self.executor, "prepare", None)
        ready = prepare(raw) if prepare is not None else None
        with self._lock:
            if self._closing:
                raise ServerError("server is closed")
            rid = self._next_id
            self._next_id += 1
            need = sum(self.arena._round(b) for b in blocks)
            if need > self.budget:
                fut.set_exception(ServerError(
                    f"request {rid}: footprint {need} bytes exceeds the HBM budget {self.budget}"))
                return fut
            self._queue.append(Request(rid, cfg, raw, precision, now, blocks, fut, ready))
            self._wake.notify()
        return fut

    def close(self, wait: bool = True):
        """Stop accepting requests; with wait, finish every queued one."""
        with self._lock:
            self._closing = True
            self._wake.notify()
        if wait:
            self._thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---- scheduler ----
    def _loop(self):
        while True:
            progressed = self._complete()
            progressed |= self._admit()
            with self._lock:
                if self._closing and not self._queue and not self._inflight:
                    return
                if not progressed:
                    # with requests waiting, memory may come back from a
                    # client's release at any time: poll
                    busy = self._inflight or self._queue
                    self._wake.wait(self.poll if busy else 0.05)

    def _retire(self, slot: int, req: Request):
        with self._lock:
            del self._inflight[slot]
            self._free_slots.append(slot)
        self.arena.free(req.scratch_off)
        req.token = None

    def _complete(self) -> bool:
        progressed = False
        with self._lock:
            items = list(self._inflight.items())
        now = time.perf_counter()
        for slot, req in items:
            err = None
            try:
                finished = self.executor.done(req.token)
            except Exception as e:        # noqa: BLE001 -- isolate the request
                finished, err = True, e
            if not finished:
                if (self.timeout is not None and not req.timed_out
                        and now - req.admitted > self.timeout):
                    req.timed_out = True
                    req.future.set_exception(TimeoutError(
                        f"request {req.id} still running after {self.timeout} s"))
                continue
            done_t = time.perf_counter()
            value = None
            if err is None:
                try:
                    value = self.executor.finish(req.token)
                except Exception as e:    # noqa: BLE001
                    err = e
            self._retire(slot, req)
            if req.timed_out or err is not None:
                self.arena.free(req.img_off)
                if not req.timed_out:
                    req.future.set_exception(err)
            else:
                res = Result(req.id, value, req.arrival, req.admitted, done_t,
                             _Releaser(self.arena, req.img_off))
                if self.on_result is not None:
                    try:
                        self.on_result(res)
                    except Exception as e:    # noqa: BLE001
                        res.release()
                        req.future.set_exception(e)
                        progressed = True
                        continue
                req.future.set_result(res)
            progressed = True
        return progressed

    def _admit(self) -> bool:
        progressed = False
        while True:
            with self._lock:
                if not self._queue or not self._free_slots:
                    return progressed
                req = self._queue[0]
                img_off = self.arena.alloc(req.blocks[0])
                scr_off = self.arena.alloc(req.blocks[1]) if img_off is not None else None
                if scr_off is None:
                    if img_off is not None:
                        self.arena.free(img_off)
                    return progressed             # arrival order: wait for memory
                self._queue.popleft()
                slot = self._free_slots.pop()
                self.admission_order.append(req.id)
            req.img_off, req.scratch_off = img_off, scr_off
            req.admitted = time.perf_counter()
            try:
                req.token = self.executor.launch(req, slot)
            except Exception as e:        # noqa: BLE001
                with self._lock:
                    self._free_slots.append(slot)
                self.arena.free(img_off)
                self.arena.free(scr_off)
                req.future.set_exception(e)
                progressed = True
                continue
            with self._lock:
                self._inflight[slot] = req
                self.max_concurrent = max(self.max_concurrent, len(self._inflight))
            progressed = True


class _Releaser:
    """Returns an image block to the arena (the finalizer of a Result)."""

    def __init__(self, arena: Arena, off: int):
        self.arena, self.off = arena, off

    def __call__(self):
        self.arena.release_later(self.off)


PLAN_KEYS = ("Nr", "Na", "range_len", "range_tbp", "az_model", "az_len", "az_tbp", "lam", "v",
             "r_near", "rcmc_taps", "rcmc_beta")


class GpuExecutor:
    """Runs requests through libsar_rda.so, one torch stream per slot, every
    buffer carved out of one device arena of ``arena_bytes``."""

    def __init__(self, slots: int, arena_bytes: int, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.capacity = arena_bytes // ALIGN * ALIGN
        self.arena = torch.empty(self.capacity, dtype=torch.uint8, device=self.device)
        self.plans: dict = {}
        self._plan_lock = threading.Lock()

    def plan(self, cfg: dict, precision: str, stream):
        """Cached plan for a parameter set (built once, then shared)."""
        from . import Plan
        key = (precision,) + tuple((k, cfg[k]) for k in PLAN_KEYS if k in cfg)
        with self._plan_lock:
            p = self.plans.get(key)
            if p is None:
                p = Plan(cfg, precision=precision, stream=stream)
                stream.synchronize()          # tables ready for every slot's stream
                self.plans[key] = p
        return p

    def _view(self, off: int, shape):
        n = int(np.prod(shape))
        return self.arena[off:off + 8 * n].view(self.torch.complex64).view(shape)

    def prepare(self, raw):
        """Called by submit() in the client's thread: an event on the client's
        current stream, after whatever work the client queued to produce
        ``raw`` (e.g. a non-blocking host-to-device copy)."""
        if raw is None or not getattr(raw, "is_cuda", False):
            return None
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(raw.device))
        return ev

    def launch(self, req: Request, slot: int):
        from ._lib import sar_rda_execute
        s = self.streams[slot]
        p = self.plan(req.cfg, req.precision, s)
        px = p.Na * p.Nr
        img = self._view(req.img_off, p.image_shape())
        raw = self._view(req.scratch_off, (p.Na, p.Nr))
        work = self._view(req.scratch_off + 8 * px, ((p.workspace_bytes + 7) // 8,))
        with self.torch.cuda.stream(s):
            if req.ready is not None:
                s.wait_event(req.ready)                 # raw's producer first
            if getattr(req.raw, "is_cuda", False):
                req.raw.record_stream(s)                # keep raw's memory until the copy ran
            raw.copy_(req.raw, non_blocking=True)       # stage into the request's buffer
            sar_rda_execute(p.handle, raw, img, work, s)
            ev = self.torch.cuda.Event()
            ev.record(s)
        return (ev, img)

    def done(self, token) -> bool:
        return token[0].query()

    def finish(self, token):
        return token[1]

    def close(self):
        self.torch.cuda.synchronize(self.device)
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def replay(server: Server, requests, arrivals):
    """Submit ``requests`` (a list of (cfg, raw, precision)) at the offsets
    ``arrivals`` (seconds, increasing) from now, in real time, and wait for
    all.  Returns (results, exceptions-by-index, wall seconds)."""
    futs = []
    t0 = time.perf_counter()
    for (cfg, raw, prec), at in zip(requests, arrivals):
        while True:
            dt = t0 + at - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(min(dt, 1e-3) if dt > 2e-4 else 0)
        futs.append(server.submit(cfg, raw, prec))
    results, errors = [], {}
    for i, f in enumerate(futs):
        try:
            results.append(f.result())
        except Exception as e:            # noqa: BLE001
            errors[i] = e
    return results, errors, time.perf_counter() - t0


def release_on_result(res: Result):
    """on_result hook for clients that only measure: drop the image."""
    res.release()


def latency_summary(results) -> dict:
    lat = np.array([r.latency for r in results]) * 1e3
    q = np.array([r.queued for r in results]) * 1e3
    return {"n": len(results), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "queue_p50_ms": float(np.percentile(q, 50)),
            "queue_p99_ms": float(np.percentile(q, 99))}
