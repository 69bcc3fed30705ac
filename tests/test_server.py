"""Scheduling logic of the continuous-batching server on the CPU, with an
executor that models each request's duration (no GPU): the HBM budget is
never exceeded, oversize requests are rejected, admission follows arrival
order, admitted requests overlap, errors and time-outs stay with their
request, and concurrent submitters are safe."""
import threading
import time

import numpy as np
import pytest

from paper_2604_03585_amd.server import (Arena, Server, ServerError, footprint_bytes,
                                         latency_summary, release_on_result, replay)


class FakeExecutor:
    """Completes a request ``cfg['dur']`` seconds after its launch; checks
    slot exclusivity and that the request's blocks lie inside the arena and
    overlap no other live block."""

    def __init__(self, budget):
        self.budget = budget
        self.lock = threading.Lock()
        self.server = None
        self.slots_busy = set()
        self.max_running = 0
        self.launched = 0

    def launch(self, req, slot):
        if req.cfg.get("bad_launch"):
            raise ValueError(f"bad parameters in request {req.id}")
        with self.lock:
            assert slot not in self.slots_busy, "slot handed out twice"
            self.slots_busy.add(slot)
            self.max_running = max(self.max_running, len(self.slots_busy))
            self.launched += 1
        if self.server is not None:
            check_blocks(self.server.arena)
            live = dict(self.server.arena.live_blocks())
            assert live[req.img_off] >= req.blocks[0] and live[req.scratch_off] >= req.blocks[1]
        return (req, slot, time.perf_counter() + req.cfg.get("dur", 0.001))

    def done(self, token):
        return time.perf_counter() >= token[2]

    def finish(self, token):
        req, slot, _ = token
        with self.lock:
            self.slots_busy.discard(slot)
        if req.cfg.get("bad_result"):
            raise RuntimeError("device error")
        return ("image", req.id)


def cfg(na, nr, dur=0.002, **kw):
    return dict(Na=na, Nr=nr, dur=dur, **kw)


def check_blocks(arena):
    blocks = arena.live_blocks()
    end = 0
    for off, n in blocks:
        assert off >= end and off % arena.align == 0, "overlapping or misaligned blocks"
        end = off + n
    assert end <= arena.size


def make(budget, slots=4, **kw):
    ex = FakeExecutor(budget)
    kw.setdefault("on_result", release_on_result)
    srv = Server(budget, slots=slots, executor=ex, **kw)
    ex.server = srv
    return srv, ex


def test_footprint():
    px = 1024 * 2048
    assert footprint_bytes(cfg(1024, 2048)) == 24 * px + 4 * (1024 + 2048) + 1024


def test_arena_against_brute_force():
    """Random allocations and frees: blocks never overlap, first fit takes
    the lowest hole, and freeing everything coalesces back to one block."""
    rng = np.random.default_rng(1)
    size = 1 << 20
    a = Arena(size, align=256)
    owner = np.zeros(size // 256, dtype=np.int64)     # 0 free, else block id + 1
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            n = live.pop(off)
            if rng.random() < 0.5:
                a.free(off)
            else:
                a.release_later(off)
            owner[off // 256:(off + n) // 256] = 0
        else:
            n = int(rng.integers(1, 40)) * 256 - int(rng.integers(0, 200))
            off = a.alloc(n)
            n = (n + 255) // 256 * 256
            holes = np.flatnonzero(np.convolve(owner == 0, np.ones(n // 256, int), "valid")
                                   == n // 256)
            if off is None:
                assert holes.size == 0
            else:
                assert holes.size and off == holes[0] * 256       # first fit
                assert not owner[off // 256:(off + n) // 256].any()
                owner[off // 256:(off + n) // 256] = step + 1
                live[off] = n
        assert a.used == sum(live.values())
    for off in list(live):
        a.free(off)
    assert a.free_blocks() == [(0, size)] and a.used == 0


def test_release_by_garbage_collection():
    srv, _ = make(1 << 30, on_result=None)
    r = srv.submit(cfg(512, 512), None).result(5)
    assert srv.used_bytes == 8 * 512 * 512
    del r
    assert srv.used_bytes == 0
    srv.close()


def test_budget_never_exceeded_under_random_load():
    rng = np.random.default_rng(0)
    sizes = [(512, 512), (1024, 1024), (2048, 1024), (2048, 2048)]
    budget = 2 * footprint_bytes(cfg(2048, 2048)) + footprint_bytes(cfg(1024, 1024))
    srv, ex = make(budget, slots=4)
    futs = []
    for i in range(200):
        na, nr = sizes[rng.integers(len(sizes))]
        futs.append(srv.submit(cfg(na, nr, dur=float(rng.uniform(0.0002, 0.003))), None))
        if rng.random() < 0.3:
            time.sleep(0.0005)
    res = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [r.id for r in res] == list(range(200))
    assert srv.max_used <= budget
    assert srv.max_concurrent <= 4 and ex.max_running <= 4
    assert srv.used_bytes == 0
    assert srv.admission_order == list(range(200))          # arrival order


def test_oversize_rejected_others_served():
    budget = footprint_bytes(cfg(1024, 1024))
    srv, _ = make(budget, on_result=None)
    f_big = srv.submit(cfg(2048, 1024), None)
    f_ok = srv.submit(cfg(1024, 1024), None)
    with pytest.raises(ServerError, match="exceeds the HBM budget"):
        f_big.result(timeout=5)
    r = f_ok.result(timeout=5)
    assert r.image == ("image", 1)
    r.release()
    assert r.image is None and srv.used_bytes == 0
    r.release()                                           # idempotent
    srv.close()


def test_budget_exhaustion_queues_in_arrival_order():
    big = footprint_bytes(cfg(2048, 2048))
    srv, ex = make(big + footprint_bytes(cfg(256, 256)) - 1, slots=4)
    fa = srv.submit(cfg(2048, 2048, dur=0.05), None)
    fb = srv.submit(cfg(2048, 2048, dur=0.01), None)
    fc = srv.submit(cfg(256, 256, dur=0.001), None)      # fits, but must not pass b
    ra, rb, rc = fa.result(5), fb.result(5), fc.result(5)
    srv.close()
    assert srv.admission_order == [0, 1, 2]
    assert rb.admitted >= ra.done - 1e-3                  # b waited for a's memory
    assert rb.queued > 0.03
    assert rc.admitted >= rb.admitted


def test_admitted_requests_overlap():
    srv, ex = make(1 << 40, slots=4)
    t0 = time.perf_counter()
    futs = [srv.submit(cfg(512, 512, dur=0.05), None) for _ in range(8)]
    for f in futs:
        f.result(5)
    wall = time.perf_counter() - t0
    srv.close()
    assert srv.max_concurrent == 4
    assert wall < 0.3                                     # 8 x 50 ms in two waves, not serial


def test_launch_and_result_errors_are_isolated():
    srv, ex = make(1 << 40, slots=2)
    f1 = srv.submit(cfg(256, 256), None)
    f2 = srv.submit(cfg(256, 256, bad_launch=True), None)
    f3 = srv.submit(cfg(256, 256, bad_result=True), None)
    f4 = srv.submit(cfg(256, 256), None)
    assert f1.result(5).id == 0
    with pytest.raises(ValueError):
        f2.result(5)
    with pytest.raises(RuntimeError, match="device error"):
        f3.result(5)
    assert f4.result(5).id == 3
    srv.close()
    assert srv.used_bytes == 0


def test_timeout_fails_future_but_keeps_memory_until_done():
    fp = footprint_bytes(cfg(512, 512))
    srv, ex = make(fp, slots=2, timeout=0.02)
    f_slow = srv.submit(cfg(512, 512, dur=0.3), None)
    with pytest.raises(TimeoutError):
        f_slow.result(5)
    # the slow request still holds its memory: the next one waits for it
    f_next = srv.submit(cfg(512, 512, dur=0.001), None)
    r = f_next.result(5)
    assert r.admitted - r.arrival > 0.1
    srv.close()
    assert srv.used_bytes == 0 and srv.max_used <= fp


def test_concurrent_submitters():
    srv, ex = make(1 << 40, slots=4)
    futs, lock = [], threading.Lock()

    def client():
        for _ in range(50):
            f = srv.submit(cfg(256, 256, dur=0.0002), None)
            with lock:
                futs.append(f)

    ts = [threading.Thread(target=client) for _ in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    ids = sorted(f.result(10).id for f in futs)
    srv.close()
    assert ids == list(range(400))


def test_closed_server_refuses():
    srv, _ = make(1 << 30)
    srv.close()
    with pytest.raises(ServerError):
        srv.submit(cfg(256, 256), None)


def test_replay_poisson_and_summary():
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(0.002, size=100))
    reqs = [(cfg(512, 512, dur=0.001), None, "fp32") for _ in arrivals]
    srv, _ = make(1 << 40, slots=4)
    results, errors, wall = replay(srv, reqs, arrivals)
    srv.close()
    assert not errors and len(results) == 100
    s = latency_summary(results)
    assert s["n"] == 100
    assert 0.001 <= s["p50_ms"] / 1e3 + 1e-4 and s["p99_ms"] >= s["p50_ms"]
    assert wall >= arrivals[-1]
