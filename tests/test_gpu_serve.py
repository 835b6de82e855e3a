"""GPU request server: every served result equals the same request rendered alone
(bit for bit: arithmetic is deterministic and pixels are independent, so chunking
and co-scheduling cannot change a pixel), served results meet the oracle bar of
their precision, and refusals, cancellation and time-outs behave as documented."""
import sys
import time

import numpy as np
import pytest

import workloads
from parity import assert_parity, compare, sample_pixels, to_numpy

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dqj():
    import torch
    assert torch.cuda.is_available()
    import paper_2303_14827_amd as m
    m.lib()
    return m


def mix(precision, n=14, seed=3):
    rng = np.random.default_rng(seed)
    ps = []
    for i in range(n):
        side = int(rng.choice([48, 64, 96, 128, 160, 256, 320]))
        N = int(rng.integers(8, 40))
        p = workloads.Params(c=workloads.seeded_c(500 + i, 0.6), width=side,
                             height=int(side * rng.choice([1.0, 0.75])), max_iter=N,
                             march_steps=2 * N * 8, bisect_steps=10, precision=precision)
        if i % 5 == 0:
            p = p.replace(c=workloads.PAPER_C[7])
        ps.append(p)
    return ps


@pytest.mark.parametrize("precision", [workloads.PREC_SPLIT, workloads.PREC_FP32])
def test_alone_equals_mixed(dqj, precision):
    import torch
    ps = mix(precision)
    alone = []
    for p in ps:
        o = dqj.render(p)
        torch.cuda.synchronize()
        alone.append(to_numpy(o))
    say("alone done", len(ps))
    # small epochs so requests are cut into several chunks and share epochs
    with dqj.Server(precision=precision, epoch_work=2e7, slots=3) as srv:
        outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
        tickets = [srv.submit(p, o) for p, o in zip(ps, outs)]
        res = [srv.wait(t, timeout_ms=60000) for t in tickets]
        st = srv.stats()
    say("served", st)
    assert all(r["status"] == dqj.OK for r in res), res
    assert st["completed"] == len(ps) and st["epochs"] >= 2
    assert max(r["chunks"] for r in res) >= 2            # some request spanned several epochs
    for p, o, a in zip(ps, outs, alone):
        g = to_numpy(o)
        for k in ("mask", "depth", "shade", "normal", "first_hit", "flags", "image8"):
            np.testing.assert_array_equal(g[k], a[k], err_msg=k)
    for r in res:
        assert r["t_submit"] <= r["t_admit"] <= r["t_first_launch"] <= r["t_done"]


def test_served_split_against_oracle(dqj):
    import oracle
    ps = [workloads.serve_stream(duration_s=0.2)[i].params for i in range(3)]
    with dqj.Server(precision=workloads.PREC_SPLIT) as srv:
        outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
        tickets = [srv.submit(p, o) for p, o in zip(ps, outs)]
        for t in tickets:
            assert srv.wait(t, 60000)["status"] == dqj.OK
    for p, o in zip(ps, outs):
        g = to_numpy(o)
        pix = sample_pixels(p, 1500, 1)
        hits = np.nonzero(g["mask"].reshape(-1))[0]
        if hits.size:
            pix = np.union1d(pix, np.random.default_rng(2).choice(hits, min(800, hits.size), replace=False))
        ora = oracle.render(p, pixels=pix)
        rep = compare(p, g, ora, pixels=pix)
        say(p.width, p.max_iter, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep, 0.999, 0.999)


def test_refusals_cancel_timeout(dqj):
    import torch
    base = workloads.plain_128()[0].replace(precision=workloads.PREC_SPLIT)
    # budget below one 512x512 framebuffer (9 B/pixel without extras)
    with dqj.Server(precision=workloads.PREC_SPLIT, hbm_budget_bytes=1 << 20, max_inflight=1,
                    max_pending=2) as srv:
        big = base.replace(width=512, height=512)
        st, _ = srv.submit_status(big, dqj.alloc_outputs(512, 512, extras=False))
        assert st == dqj.E_BUDGET
        st, _ = srv.submit_status(base.replace(width=0), dqj.alloc_outputs(8, 8, extras=False))
        assert st == dqj.E_INVALID
        st, _ = srv.submit_status(base.replace(precision=workloads.PREC_FP32),
                                  dqj.alloc_outputs(128, 128, extras=False))
        assert st == dqj.E_INVALID
        # a slow request holds the only in-flight slot; the next ones queue
        slow = base.replace(width=300, height=300, max_iter=64, march_steps=1024)
        t1 = srv.submit(slow, dqj.alloc_outputs(300, 300, extras=False))
        deadline = time.monotonic() + 10.0
        while srv.poll(t1)["t_admit"] < 0:           # the scheduler thread admits it
            assert time.monotonic() < deadline
            time.sleep(0.0002)
        t2 = srv.submit(base, dqj.alloc_outputs(128, 128, extras=False))
        t3 = srv.submit(base, dqj.alloc_outputs(128, 128, extras=False))
        st, _ = srv.submit_status(base, dqj.alloc_outputs(128, 128, extras=False))
        assert st == dqj.E_QUEUE_FULL
        assert srv.wait(t3, timeout_ms=0)["status"] == dqj.E_TIMEOUT
        assert srv.cancel(t3) == dqj.OK
        assert srv.wait(t3, 1000)["status"] == dqj.E_CANCELLED
        assert srv.wait(t1, 60000)["status"] == dqj.OK
        assert srv.wait(t2, 60000)["status"] == dqj.OK
        assert srv.cancel(t2) == dqj.E_STATE
        s = srv.stats()
        assert s["completed"] == 2 and s["cancelled"] == 1 and s["rejected"] >= 2
        assert s["resident_bytes"] == 0


def test_destroy_with_work_in_flight(dqj):
    ps = mix(workloads.PREC_SPLIT, n=6, seed=9)
    srv = dqj.Server(precision=workloads.PREC_SPLIT, epoch_work=1e7)
    outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    for p, o in zip(ps, outs):
        srv.submit(p, o)
    srv.close()     # cancels what is pending, waits for epochs in flight
    import torch
    torch.cuda.synchronize()
