"""GPU projection ("shadow") rendering (paragraph "Dimension Reduction", approach 2)
against the FP64 oracle, through the C ABI: mask >= 99.9%, depth within 1e-4 of the box
diagonal, update count within 0.1% (the plain path's bar) and shade within 1/255 on
>= 99% of agreeing hits (the normal's potential is a minimum over the fibre points, whose
creases make the central differences of a few hits ill-conditioned), the zero-fibre
reduction to the slice, the c = 0 shadow ball, both normal modes, the refusals, and
sampled pixels at the bench size."""

BAR = (0.999, 0.99)
import math
import sys

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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
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


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_project_128_against_oracle(dqj, oracle_mod, seed):
    p = workloads.project_128(seed)[0]
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(seed, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, *BAR)
    assert abs(int(g["iters"][0]) - o["total_iters"]) <= 1e-3 * o["total_iters"]
    # the shadow covers the slice
    s = oracle_mod.render(workloads.plain_128(seed)[0])
    assert g["mask"].sum() > s["mask"].sum()


def test_zero_fibre_is_the_slice(dqj, oracle_mod):
    p = workloads.plain_128(3)[0]
    q = p.replace(fiber=np.zeros((1, 8)))
    g = render_np(dqj, q)
    rep = compare(p, g, oracle_mod.render(p))
    assert_parity(rep)
    # and the same image as the slice render to the plain path's own bar
    h = render_np(dqj, p)
    agree = (g["mask"] == h["mask"]).mean()
    assert agree >= 0.999


def test_c0_shadow_ball(dqj, oracle_mod):
    N, S, B = 12, 64, 8
    rho = 4.0 ** (2.0 ** -N)
    fib = np.zeros((3, 8))
    fib[:, 3] = (0.3, 0.5, -0.4)
    p = workloads.Params(c=[0.0] * 8, width=64, height=64, max_iter=N, march_steps=S,
                         bisect_steps=B, fiber=fib)
    rs = math.sqrt(rho * rho - float(np.min(np.abs(p.fiber[:, 3]))) ** 2)
    g = render_np(dqj, p)
    checked = 0
    for j in range(0, p.height, 2):
        for i in range(0, p.width, 2):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            b = float(np.dot(o, d))
            disc = b * b - (float(np.dot(o, o)) - rs * rs)
            if disc < 0:
                assert g["mask"][j, i] == 0
                continue
            if 2 * math.sqrt(disc) < 5e-2:
                continue
            assert g["mask"][j, i] == 1
            ts = -b - math.sqrt(disc)
            assert abs(g["depth"][j, i] - ts) <= 2 * (t1 - t0) / S * 2.0 ** -B + 1e-5
            checked += 1
    assert checked > 100


def test_neighbour_normal_projection(dqj, oracle_mod):
    p = workloads.project_128(1)[0].replace(normal_mode=workloads.NORMAL_NEIGHBOUR4)
    g = render_np(dqj, p)
    rep = compare(p, g, oracle_mod.render(p))
    assert_parity(rep, *BAR)


PKEYS = ("mask", "depth", "shade", "normal", "first_hit", "image8", "flags")


def test_projection_batch_equals_single(dqj):
    """A batch of projection frames (one launch, the frames' blocks interleaved) and a
    captured plan of the same frames give every frame bit for bit what dqj_render gives,
    update counts included: frames of different sizes, fibre counts and constants."""
    import torch
    ps = [workloads.project_128(0)[0],
          workloads.project_128(1, fibers=3)[0].replace(width=97, height=61),
          workloads.project_128(2, fibers=16)[0].replace(width=160, height=120, c=workloads.PAPER_C[7],
                                                        max_iter=15),
          workloads.project_128(3, fibers=1)[0].replace(width=33, height=1)]
    for p in ps:
        p.__post_init__()
    singles = []
    for p in ps:
        o = dqj.alloc_outputs(p.width, p.height)
        dqj.render(p, out=o)
        torch.cuda.synchronize()
        singles.append((to_numpy(o), int(o["iters"].item())))
    say("singles done", [s[1] for s in singles])
    outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    dqj.render_batch(ps, outs)
    torch.cuda.synchronize()
    for i, (o, (a, it)) in enumerate(zip(outs, singles)):
        g = to_numpy(o)
        for k in PKEYS:
            np.testing.assert_array_equal(g[k], a[k], err_msg=f"batch frame {i} {k}")
        assert int(o["iters"].item()) == it, (i, int(o["iters"].item()), it)
    say("batch equal")
    outs2 = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height).items() if k != "iters"} for p in ps]
    plan = dqj.BatchPlan(ps, outs2)
    for rep in range(2):
        for o in outs2:
            o["depth"].fill_(-1.0)
        plan.launch()
        torch.cuda.synchronize()
        for i, (o, (a, _)) in enumerate(zip(outs2, singles)):
            g = to_numpy(o)
            for k in PKEYS:
                np.testing.assert_array_equal(g[k], a[k], err_msg=f"plan replay {rep} frame {i} {k}")
    plan.close()


def test_projection_batch_refusals(dqj):
    p = workloads.project_128(0)[0]
    q = workloads.plain_128(0)[0]
    with pytest.raises(Exception, match="projection frames only"):
        dqj.render_batch([p, q])
    with pytest.raises(Exception, match="projection frames only"):
        dqj.render_batch([q, p])
    with pytest.raises(Exception, match="four-neighbour"):
        dqj.render_batch([p, p.replace(normal_mode=workloads.NORMAL_NEIGHBOUR4)])
    with dqj.Server(precision=workloads.PREC_FP32) as srv:
        with pytest.raises(Exception, match="projection"):
            srv.submit(p.replace(precision=workloads.PREC_FP32), dqj.alloc_outputs(p.width, p.height))


def test_project_512_sampled(dqj, oracle_mod):
    """The bench workload (3 frames of 512^2 of the paper's constants, 16 fibre points):
    sampled pixels and a subset of the hits against the oracle, pixel by pixel."""
    for f, p in enumerate(workloads.project_512()):
        g = render_np(dqj, p)
        pix = sample_pixels(p, 1500, f)
        hits = np.nonzero(g["mask"].reshape(-1))[0]
        if hits.size:
            rng = np.random.default_rng(f)
            pix = np.union1d(pix, rng.choice(hits, size=min(800, hits.size), replace=False))
        o = oracle_mod.render(p, pixels=pix)
        rep = compare(p, g, o, pixels=pix)
        say("frame", f, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert rep["hits_oracle"] > 200
        assert_parity(rep, *BAR)


@pytest.mark.parametrize("variant", ["realpart", "dual_slice"])
def test_projection_variants(dqj, oracle_mod, variant):
    """The real-part escape norm, and a slice through the dual scalar axis (W = e4) whose
    fibre offsets lie in other directions (a3, b1, b2)."""
    p = workloads.project_128(2)[0]
    if variant == "realpart":
        p = p.replace(norm=workloads.NORM_REALPART)
    else:
        axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]]
        fib = np.zeros((6, 8))
        rng = np.random.default_rng(11)
        fib[1:, [3, 5, 6]] = rng.uniform(-0.4, 0.4, (5, 3))
        p = p.replace(slice_axes=axes, fiber=fib)
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(variant, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, *BAR)
    assert abs(int(g["iters"][0]) - o["total_iters"]) <= 1e-3 * o["total_iters"]


@pytest.mark.parametrize("case", ["max_fibres", "N1", "N2_ragged", "one_offset"])
def test_projection_edges(dqj, oracle_mod, case):
    """The largest fibre table (32), max_iter 1 and 2 on a ragged frame, and a single
    non-zero offset (the slice shifted in a collapsed direction)."""
    p = workloads.plain_128(4)[0]
    if case == "max_fibres":
        p = p.replace(width=64, height=64, fiber=workloads.fiber_ball(32, 0.5, 3))
    elif case == "N1":
        p = p.replace(width=67, height=45, max_iter=1, fiber=workloads.fiber_ball(5, 0.4, 4))
    elif case == "N2_ragged":
        p = p.replace(width=67, height=45, max_iter=2, fiber=workloads.fiber_ball(5, 0.4, 5))
    else:
        fib = np.zeros((1, 8))
        fib[0, 3] = 0.25
        p = p.replace(fiber=fib)
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(case, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, *BAR)
    assert abs(int(g["iters"][0]) - o["total_iters"]) <= 1e-3 * o["total_iters"]


@pytest.mark.parametrize("side,fibres,lanes", [(1024, 3, 1), (768, 2, 2), (128, 3, 2), (128, 8, 4)])
def test_projection_lane_groups(dqj, oracle_mod, side, fibres, lanes):
    """Each grouping of lanes per pixel: 1, 2 or 4, the least that gives the launch about
    2^20 lanes, at most the fibre count (the grouping leaves the image unchanged; here each
    one is checked against the oracle on a whole frame, with the update count)."""
    group = 1
    while group < 4 and 2 * group <= fibres and side * side * group < (1 << 20):
        group *= 2
    assert group == lanes
    small = side <= 128
    p = workloads.plain_128(4)[0].replace(
        width=side, height=side, max_iter=8 if small else 4, march_steps=128 if small else 16,
        bisect_steps=8 if small else 3, fiber=workloads.fiber_ball(fibres, 0.4, 6))
    g = render_np(dqj, p)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(side, fibres, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert rep["hits_oracle"] > 100
    assert_parity(rep, *BAR)
    assert abs(int(g["iters"][0]) - o["total_iters"]) <= 1e-3 * o["total_iters"]


@pytest.mark.parametrize("side", [128, 1024])
def test_projection_count_off_same_image(dqj, side):
    """Without an update counter the launch takes the non-counting kernels; the image is
    bitwise that of the counting launch (4 lanes per pixel at 128^2, one at 1024^2)."""
    import torch
    p = workloads.plain_128(4)[0].replace(width=side, height=side, max_iter=8, march_steps=32,
                                          bisect_steps=4, fiber=workloads.fiber_ball(8, 0.4, 7))
    a = dqj.alloc_outputs(side, side, extras=False)
    b = {k: v for k, v in dqj.alloc_outputs(side, side, extras=False).items() if k != "iters"}
    a["iters"].zero_()
    dqj.render(p, out=a)
    dqj.render(p, out=b)
    torch.cuda.synchronize()
    assert int(a["iters"].item()) > 0
    for k in ("mask", "depth", "shade"):
        assert torch.equal(a[k], b[k]), k
