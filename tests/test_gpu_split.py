"""GPU split-precision path (packed FP16 march to a candidate crossing, FP32
continuation + bisection, FP64 re-bisection of rays whose FP32 classes flip) against
the FP64 oracle, at the FP32 path's bar: >= 99.9 % of pixels agree, every mismatch
within one march step of the set's boundary, depth on agreeing hits within 1e-4 of
the box diagonal, shade within 1/255 on >= 99.9 % of agreeing hits.
"""
import sys

import numpy as np
import pytest

import workloads
from parity import assert_parity, compare, to_numpy

SPLIT_MIN_AGREE = 0.999
SPLIT_SHADE_FRAC = 0.999

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


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


def render_np(dqj, p):
    import torch
    out = dqj.render(p)
    torch.cuda.synchronize()
    return to_numpy(out)


@pytest.mark.parametrize("seed", [0, 2, 5])
def test_split_1080p_shape_reduced(dqj, oracle_mod, seed):
    p = workloads.split_1080p([seed])[0].replace(width=320, height=180)
    say("split", seed, p.width, p.height)
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    fp64 = int(((g["flags"] & 4) != 0).sum())
    say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"}, "fp64 rays", fp64)
    assert_parity(rep, SPLIT_MIN_AGREE, SPLIT_SHADE_FRAC)
    miss = g["mask"] == 0
    assert np.all(np.isinf(g["depth"][miss])) and np.all(g["first_hit"][miss] == -1)


def test_split_paper_constant_hits_and_fp64_pass(dqj, oracle_mod):
    # Fig. highres's constant gives a large visible set: many refined rays, some FP64
    p = workloads.split_1080p([0])[0].replace(c=workloads.PAPER_C[7], width=256, height=144,
                                              max_iter=32)
    p.__post_init__()
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"},
        "fp64 rays", int(((g["flags"] & 4) != 0).sum()))
    assert rep["hits_oracle"] > 1000
    assert_parity(rep, SPLIT_MIN_AGREE, SPLIT_SHADE_FRAC)


def test_split_edge_cases(dqj, oracle_mod):
    base = workloads.split_1080p([2])[0].replace(width=97, height=61)
    cases = [base.replace(march_steps=1), base.replace(march_steps=2), base.replace(max_iter=1),
             base.replace(bisect_steps=0), base.replace(norm=workloads.NORM_REALPART),
             base.replace(fp64_window=8), base.replace(fp64_window=1)]
    axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]]
    cases.append(base.replace(slice_axes=axes, c=workloads.PAPER_C[7], max_iter=15))
    for p in cases:
        p.__post_init__()
        say("split edge", p.march_steps, p.max_iter, p.bisect_steps, p.norm, p.fp64_window)
        g = render_np(dqj, p)
        o = oracle_mod.render(p)
        rep = compare(p, g, o)
        say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep, SPLIT_MIN_AGREE, SPLIT_SHADE_FRAC)


def test_split_batch_matches_single(dqj):
    import torch
    ps = [p.replace(width=160, height=90) for p in workloads.split_1080p(range(4))]
    singles = [render_np(dqj, p) for p in ps]
    outs = dqj.render_batch(ps, extras=True)
    torch.cuda.synchronize()
    for o, s in zip(outs, singles):
        o = to_numpy(o)
        for k in ("mask", "depth", "shade", "normal", "first_hit", "flags"):
            np.testing.assert_array_equal(o[k], s[k], err_msg=k)
    plan = dqj.BatchPlan(ps, [dqj.alloc_outputs(p.width, p.height) for p in ps])
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for o, s in zip(plan.outs, singles):
            o = to_numpy(o)
            for k in ("mask", "depth", "shade"):
                np.testing.assert_array_equal(o[k], s[k], err_msg=f"replay {rep} {k}")
    plan.close()
