"""The server's scheduling core on the CPU (no HIP), driven by a simulated clock:
budget admission, queue limits, chunked epochs with a fair share for every active
request, completion only after every tile, cancellation, failure reclaim, stats."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_14827_amd", "csrc")

OK, BUDGET, QUEUE_FULL, DEVICE, CANCELLED, STATE = 0, -3, -4, -5, -7, -9
PENDING_ST, ADMITTED, DONE, CANCELLED_ST, FAILED = 0, 1, 2, 3, 4


@pytest.fixture(scope="module")
def L(tmp_path_factory):
    d = tmp_path_factory.mktemp("core")
    so = str(d / "libcore.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-Wall", "-I", CSRC,
                    os.path.join(CSRC, "serve_core.cpp"), os.path.join(ROOT, "tests", "serve_core_shim.cpp"),
                    "-o", so], check=True)
    lib = C.CDLL(so)
    lib.core_new.restype = C.c_void_p
    lib.core_new.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.c_double, C.c_uint64, C.c_int32,
                             C.c_int32]
    lib.core_free.argtypes = [C.c_void_p]
    lib.core_submit.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_double, C.c_double,
                                C.POINTER(C.c_uint64)]
    lib.core_admit.argtypes = [C.c_void_p, C.c_double]
    lib.core_build.argtypes = [C.c_void_p, C.c_double, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                               C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.c_int32]
    lib.core_finish.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.c_double, C.POINTER(C.c_uint64),
                                C.c_int32]
    lib.core_cancel.argtypes = [C.c_void_p, C.c_uint64, C.c_double]
    lib.core_fail_all.argtypes = [C.c_void_p, C.c_double]
    lib.core_state.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.core_stats.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double)]
    return lib


class Core:
    def __init__(self, L, budget=1000, max_inflight=64, max_pending=100, epoch_work=100.0,
                 epoch_pixels=1 << 20, max_chunks=256, oldest_first=False):
        self.L = L
        self.h = L.core_new(budget, max_inflight, max_pending, epoch_work, epoch_pixels, max_chunks,
                            1 if oldest_first else 0)

    def submit(self, nbytes, tiles, now=0.0, tile_px=64, wpt=1.0):
        t = C.c_uint64()
        st = self.L.core_submit(self.h, nbytes, tiles, tile_px, wpt, now, C.byref(t))
        return st, t.value

    def admit(self, now=0.0):
        self.L.core_admit(self.h, now)

    def build(self, now=0.0, cap=512):
        eid = C.c_uint64()
        tk = (C.c_uint64 * cap)()
        bg = (C.c_uint32 * cap)()
        nt = (C.c_uint32 * cap)()
        n = self.L.core_build(self.h, now, C.byref(eid), tk, bg, nt, cap)
        if n == 0:
            return None
        return eid.value, [(tk[i], bg[i], nt[i]) for i in range(n)]

    def finish(self, eid, ok=True, now=0.0):
        fin = (C.c_uint64 * 512)()
        n = self.L.core_finish(self.h, eid, 1 if ok else 0, now, fin, 512)
        return [fin[i] for i in range(n)]

    def cancel(self, t, now=0.0):
        return self.L.core_cancel(self.h, t, now)

    def state(self, t):
        st, ta, td, ch = C.c_int32(), C.c_double(), C.c_double(), C.c_int32()
        s = self.L.core_state(self.h, t, C.byref(st), C.byref(ta), C.byref(td), C.byref(ch))
        return s, st.value, ta.value, td.value, ch.value

    def stats(self):
        c = (C.c_uint64 * 10)()
        l = (C.c_double * 4)()
        self.L.core_stats(self.h, c, l)
        keys = ["submitted", "admitted", "completed", "cancelled", "failed", "rejected", "epochs",
                "resident", "pending", "active"]
        d = dict(zip(keys, list(c)))
        d.update(dict(zip(["p50", "p99", "max", "mean"], list(l))))
        return d

    def __del__(self):
        self.L.core_free(self.h)


def run_to_completion(core, now=0.0, limit=10000):
    for _ in range(limit):
        core.admit(now)
        e = core.build(now)
        if e is None:
            return now
        core.finish(e[0], True, now + 1.0)
        now += 1.0
    raise AssertionError("did not drain")


def test_budget_admission_and_reclaim(L):
    c = Core(L, budget=250)
    assert c.submit(300, 4)[0] == BUDGET          # alone above the budget
    ts = [c.submit(100, 4)[1] for _ in range(3)]
    c.admit()
    assert [c.state(t)[0] for t in ts] == [ADMITTED, ADMITTED, PENDING_ST]
    assert c.stats()["resident"] == 200
    e = c.build()
    for _, (eid, chunks) in [(0, e)]:
        c.finish(eid)
    assert c.state(ts[0])[0] == DONE and c.state(ts[1])[0] == DONE
    assert c.stats()["resident"] == 0
    c.admit(2.0)
    assert c.state(ts[2])[0] == ADMITTED
    run_to_completion(c, 3.0)
    assert c.state(ts[2])[0] == DONE and c.stats()["completed"] == 3


def test_queue_full_and_inflight_cap(L):
    c = Core(L, budget=10 ** 9, max_inflight=2, max_pending=3)
    ts = [c.submit(1, 10)[1] for _ in range(3)]
    assert c.submit(1, 10)[0] == QUEUE_FULL
    c.admit()
    assert sum(c.state(t)[0] == ADMITTED for t in ts) == 2
    assert c.stats()["rejected"] == 1


def test_every_tile_once_and_fair_share(L):
    c = Core(L, epoch_work=100.0)
    _, big = c.submit(1, 1000)
    c.admit()
    seen = {}
    eid, ch = c.build()
    assert ch == [(big, 0, 100)]                  # one epoch's worth of the big request
    c.finish(eid)
    _, small = c.submit(1, 5, now=1.0)
    c.admit(1.0)
    eid, ch = c.build(1.0)
    d = {t: (b, n) for t, b, n in ch}
    assert d[small] == (0, 5)                     # the newcomer is in the very next epoch
    assert d[big][0] == 100
    fin = c.finish(eid, True, 2.0)
    assert small in fin and c.state(small)[0] == DONE and c.state(big)[0] == ADMITTED
    # drain and check the big request's tiles were handed out contiguously, once each
    nxt = 100 + d[big][1]
    while True:
        e = c.build(3.0)
        if e is None:
            break
        for t, b, n in e[1]:
            assert t == big and b == nxt
            nxt += n
        c.finish(e[0], True, 3.0)
    assert nxt == 1000 and c.state(big)[0] == DONE


def test_oldest_first_policy(L):
    # epochs are filled oldest request first: a newcomer waits until the older request's
    # remaining tiles fit, then shares the epoch with it
    c = Core(L, epoch_work=100.0, oldest_first=True)
    _, big = c.submit(1, 250)
    _, small = c.submit(1, 5)
    c.admit()
    eid, ch = c.build()
    assert ch == [(big, 0, 100)]
    c.finish(eid, True, 1.0)
    eid, ch = c.build(1.0)
    assert ch == [(big, 100, 100)]
    c.finish(eid, True, 2.0)
    eid, ch = c.build(2.0)
    assert ch == [(big, 200, 50), (small, 0, 5)]
    fin = c.finish(eid, True, 3.0)
    assert set(fin) == {big, small}


def test_pixel_and_chunk_caps(L):
    c = Core(L, epoch_work=1e9, epoch_pixels=64 * 10, max_chunks=2)
    ts = [c.submit(1, 8)[1] for _ in range(3)]
    c.admit()
    eid, ch = c.build()
    assert len(ch) <= 2 and sum(n for _, _, n in ch) <= 10


def test_completion_waits_for_all_chunks(L):
    c = Core(L, epoch_work=10.0)
    _, t = c.submit(1, 25)
    c.admit()
    e1 = c.build()
    e2 = c.build()
    e3 = c.build()
    assert c.build() is None                      # everything assigned, three epochs in flight
    c.finish(e3[0])
    c.finish(e1[0])
    assert c.state(t)[0] == ADMITTED
    c.finish(e2[0], True, 5.0)
    s = c.state(t)
    assert s[0] == DONE and s[4] == 3 and s[3] == 5.0


def test_cancel_pending_and_running(L):
    c = Core(L, budget=100, epoch_work=10.0)
    _, a = c.submit(100, 50)
    _, b = c.submit(100, 5)
    c.admit()
    e = c.build()
    assert c.state(b)[0] == PENDING_ST
    assert c.cancel(b) == OK and c.state(b)[0] == CANCELLED_ST and c.state(b)[1] == CANCELLED
    assert c.cancel(a) == OK and c.state(a)[0] == ADMITTED      # its chunk is still in flight
    assert c.build() is None                                     # nothing more of it is launched
    c.finish(e[0])
    assert c.state(a)[0] == CANCELLED_ST and c.stats()["resident"] == 0
    assert c.cancel(a) == STATE


def test_launch_failure_reclaims_and_later_requests_succeed(L):
    c = Core(L, budget=100, epoch_work=1000.0)
    _, a = c.submit(60, 4)
    _, b = c.submit(60, 4)
    c.admit()
    e = c.build()
    fin = c.finish(e[0], ok=False)
    assert a in fin and c.state(a)[0] == FAILED and c.state(a)[1] == DEVICE
    assert c.stats()["resident"] == 0
    run_to_completion(c, 1.0)
    assert c.state(b)[0] == DONE


def test_fail_all(L):
    c = Core(L, budget=100)
    ts = [c.submit(60, 4)[1] for _ in range(3)]
    c.admit()
    c.build()
    assert L.core_fail_all(c.h, 1.0) == 3
    assert all(c.state(t)[0] == FAILED for t in ts)
    assert c.stats()["resident"] == 0 and c.stats()["pending"] == 0


def test_latency_stats(L):
    c = Core(L, epoch_work=1e9)
    for i in range(100):
        _, t = c.submit(1, 1, now=0.0)
        c.admit(0.0)
        e = c.build(0.0)
        c.finish(e[0], True, (i + 1) / 100.0)
    s = c.stats()
    assert abs(s["p50"] - 0.50) < 1e-12 and abs(s["p99"] - 0.99) < 1e-12 and s["max"] == 1.0
    assert abs(s["mean"] - 0.505) < 1e-12


def test_random_load_invariants(L):
    rng = np.random.default_rng(7)
    budget = 5000
    c = Core(L, budget=budget, max_inflight=8, max_pending=64, epoch_work=200.0, max_chunks=16)
    inflight = []
    now = 0.0
    tiles_of = {}
    done_tiles = {}
    for step in range(3000):
        now += 0.001
        if rng.random() < 0.3:
            nb = int(rng.integers(1, 3000))
            nt = int(rng.integers(1, 400))
            st, t = c.submit(nb, nt, now=now, wpt=float(rng.uniform(0.5, 3)))
            if st == OK:
                tiles_of[t] = nt
                done_tiles[t] = 0
        c.admit(now)
        assert c.stats()["resident"] <= budget
        if len(inflight) < 3:
            e = c.build(now)
            if e is not None:
                inflight.append(e)
        if inflight and rng.random() < 0.5:
            eid, ch = inflight.pop(int(rng.integers(0, len(inflight))))
            for t, b, n in ch:
                done_tiles[t] += n
            c.finish(eid, True, now)
    while inflight or c.build(now) is not None:
        while inflight:
            eid, ch = inflight.pop()
            for t, b, n in ch:
                done_tiles[t] += n
            c.finish(eid, True, now)
        c.admit(now)
        e = c.build(now)
        if e is not None:
            inflight.append(e)
    for t, n in tiles_of.items():
        assert c.state(t)[0] == DONE, t
        assert done_tiles[t] == n
