"""GPU checks of the launch configurations the benchmark times, at their full sizes.

* plain_1024 as timed: one batch plan over the 3 frames without extras and without the
  update counter (the non-counting instantiation of the batched refill kernel). Its
  images must equal, bit for bit, the counting plan's and single-frame renders with
  every extra output; sampled pixels and GPU hits are checked against the FP64 oracle.
* split_1080p: the 8 frames at 1920x1080 in one plan, every frame checked against the
  oracle on sampled pixels plus sampled GPU hits.
* sweep_256-shaped frames (real parts U[-0.8, 0.8], max_iter 16, 256 steps, 8 bisection
  steps) in one plan of 64 frames; four frames checked whole against the oracle, with
  the GPU's update count within 0.1 % of the oracle's.
"""
import sys

import numpy as np
import pytest

import workloads
from parity import assert_parity, compare, sample_pixels, to_numpy

pytestmark = pytest.mark.gpu

SPLIT_MIN_AGREE = 0.999
SPLIT_SHADE_FRAC = 0.999


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dqj():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_14827_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


def sampled_with_hits(p, g, n, seed):
    pix = sample_pixels(p, n, seed)
    hits = np.nonzero(g["mask"].reshape(-1))[0]
    if hits.size:
        rng = np.random.default_rng(seed + 1)
        pix = np.union1d(pix, rng.choice(hits, size=min(n // 2, hits.size), replace=False))
    return pix


def test_plain_1024_timed_configuration(dqj, oracle_mod):
    import torch
    ps = workloads.plain_1024()
    say("plain_1024 counting plan")
    counted = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    cplan = dqj.BatchPlan(ps, counted)
    cplan.launch()
    torch.cuda.synchronize()
    cplan.close()
    say("plain_1024 timed plan (no counter, no extras), 3 replays")
    timed = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
              if k != "iters"} for p in ps]
    plan = dqj.BatchPlan(ps, timed)
    for rep in range(3):
        for o in timed:
            o["depth"].fill_(-1.0)
        plan.launch()
        torch.cuda.synchronize()
        for t, c in zip(timed, counted):
            for k in ("mask", "depth", "shade"):
                assert torch.equal(t[k], c[k]), f"replay {rep} {k}"
    plan.close()
    for f, p in enumerate(ps):
        say("single-frame render with extras", f)
        g = to_numpy(dqj.render(p))
        torch.cuda.synchronize()
        t = to_numpy(timed[f])
        for k in ("mask", "depth", "shade"):
            np.testing.assert_array_equal(t[k], g[k], err_msg=f"frame {f} {k}")
        pix = sampled_with_hits(p, g, 3000, 10 + f)
        o = oracle_mod.render(p, pixels=pix)
        rep = compare(p, g, o, pixels=pix)
        say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep)


def test_split_1080p_full_size(dqj, oracle_mod):
    import torch
    ps = workloads.split_1080p()
    outs = [dqj.alloc_outputs(p.width, p.height, extras=True) for p in ps]
    say("split_1080p plan, 8 frames 1920x1080")
    plan = dqj.BatchPlan(ps, outs)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    for f, p in enumerate(ps):
        g = to_numpy(outs[f])
        pix = sampled_with_hits(p, g, 4000, 20 + f)
        o = oracle_mod.render(p, pixels=pix)
        rep = compare(p, g, o, pixels=pix)
        fp64 = int(((g["flags"] & 4) != 0).sum())
        say(" frame", f, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"},
            "fp64 rays", fp64)
        assert_parity(rep, SPLIT_MIN_AGREE, SPLIT_SHADE_FRAC)


def test_sweep_shaped_frames(dqj, oracle_mod):
    import torch
    ps = workloads.sweep_256(64)
    outs = [dqj.alloc_outputs(p.width, p.height, extras=True) for p in ps]
    say("sweep_256 plan, 64 frames")
    plan = dqj.BatchPlan(ps, outs)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    for f in (0, 21, 42, 63):
        p = ps[f]
        g = to_numpy(outs[f])
        o = oracle_mod.render(p)
        rep = compare(p, g, o)
        say(" frame", f, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep)
        rel = abs(int(g["iters"][0]) - o["total_iters"]) / max(o["total_iters"], 1)
        assert rel <= 1e-3, (f, int(g["iters"][0]), o["total_iters"])
