"""Renders without an update counter (the kernel instantiation that timed launches use)
against renders with one: both run every sample, bisection point and normal point with
the same arithmetic, so every output must agree bit for bit, whatever the schedule,
the batch composition or the frame's edge cases. The counting renders are themselves
checked against the FP64 oracle by the other GPU tests."""
import sys

import numpy as np
import pytest

import workloads
from parity import to_numpy

pytestmark = pytest.mark.gpu

KEYS = ("mask", "depth", "shade", "normal", "first_hit", "image8", "flags")


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


def counting_ref(dqj, p):
    """Render with the update counter."""
    import torch
    out = dqj.render(p, schedule=dqj.make_schedule(kernel=dqj.KERNEL_REFILL))
    torch.cuda.synchronize()
    return to_numpy(out)


def nocount_render(dqj, p, schedule=None):
    import torch
    out = dqj.alloc_outputs(p.width, p.height)
    del out["iters"]
    dqj.render(p, out=out, schedule=schedule)
    torch.cuda.synchronize()
    return to_numpy(out)


def assert_same(a, b, what):
    for k in KEYS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=f"{what}: {k}")


def cases():
    base = workloads.plain_1024([2])[0].replace(width=160, height=120)
    out = {
        "plain_128_s0": workloads.plain_128(0)[0],
        "plain_128_s1": workloads.plain_128(1)[0],
        "plain_1024_shape": base,
        "paper_const": base.replace(c=workloads.PAPER_C[7], max_iter=15),
        "S1": base.replace(march_steps=1),
        "S2": base.replace(march_steps=2),
        "B0": base.replace(bisect_steps=0),
        "N1": base.replace(max_iter=1),
        "N2": base.replace(max_iter=2),
        "realpart": base.replace(norm=workloads.NORM_REALPART),
        "dual_slice": base.replace(
            slice_axes=[[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]],
            slice_origin=[0, 0, 0.1, 0, 0, 0, 0, 0], c=[-0.39054, -0.58679, 0, 0, 0.0, 0.5632, 0, 0.05],
            max_iter=15),
        "eye_inside_box": base.replace(eye=[0.3, 0.2, 1.4], target=[0.0, 0.0, 0.0], fov_y_deg=90.0,
                                       c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0]),
        "ragged": base.replace(width=97, height=61),
        "one_pixel": base.replace(width=1, height=1),
        "row": base.replace(width=64, height=1),
        "column": base.replace(width=1, height=64),
        "specular_cull": workloads.plain_128(3)[0].replace(k_specular=0.4, shininess=20.0, cull_radius=1.35),
        "large_dual": base.replace(c=[0.1, -0.3, 0.2, 0.05, 0.9, -0.8, 0.7, 0.6]),
    }
    for p in out.values():
        p.__post_init__()
    return out


CASES = cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_nocount_equals_counting(dqj, name):
    p = CASES[name]
    say("case", name, p.width, p.height, "N", p.max_iter, "S", p.march_steps, "B", p.bisect_steps)
    ref = counting_ref(dqj, p)
    got = nocount_render(dqj, p)
    assert_same(got, ref, name)


SCHEDULES = [(8, 8, 4, 8), (5, 3, 4, 8), (1, 64, 2, 4), (32, 32, 8, 2), (16, 4, 1, 16), (3, 1, 16, 1)]


def test_nocount_schedules(dqj):
    p = CASES["paper_const"].replace(width=203, height=151)
    p.__post_init__()
    ref = counting_ref(dqj, p)
    for tw, th, wpb, bpc in SCHEDULES:
        say("schedule", tw, th, wpb, bpc)
        s = dqj.make_schedule(kernel=dqj.KERNEL_REFILL, tile_w=tw, tile_h=th, waves_per_block=wpb,
                              blocks_per_cu=bpc)
        assert_same(nocount_render(dqj, p, s), ref, f"schedule {tw}x{th} {wpb} {bpc}")


def test_nocount_mixed_batch_and_replays(dqj):
    """Frames of different sizes, constants, max_iter, steps, norms' slices and kinds in
    one launch: lanes of one wave hold rays of several frames at once."""
    import torch
    ps = [CASES[n] for n in ("plain_128_s0", "paper_const", "N2", "S2", "B0", "ragged", "one_pixel",
                             "large_dual", "specular_cull", "eye_inside_box")]
    ps += [workloads.sweep_256(1, first_seed=s)[0] for s in (3, 9)]
    refs = [counting_ref(dqj, p) for p in ps]
    say("batch eager")
    outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    for o in outs:
        del o["iters"]
    dqj.render_batch(ps, outs)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(to_numpy(o), r, f"batch frame {i}")
    say("batch plan, 3 replays")
    outs2 = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    for o in outs2:
        del o["iters"]
    plan = dqj.BatchPlan(ps, outs2)
    for rep in range(3):
        for o in outs2:
            o["depth"].fill_(-1.0)
            o["mask"].fill_(7)
        plan.launch()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        for i, (o, r) in enumerate(zip(outs2, refs)):
            assert_same(to_numpy(o), r, f"replay {rep} frame {i}")
    plan.close()


def test_nocount_general_slice_batch(dqj):
    """A batch whose frames are all on general slices (the kernel without the closed-form
    first update) and one on the real-part norm, against single counting renders."""
    import torch
    axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]]
    ps = [workloads.plain_128(s)[0].replace(slice_axes=axes, c=workloads.PAPER_C[7], max_iter=15)
          for s in range(3)]
    ps += [workloads.plain_128(4)[0].replace(slice_origin=[0.1, 0, 0, 0, 0, 0.05, 0, 0])]
    for p in ps:
        p.__post_init__()
    refs = [counting_ref(dqj, p) for p in ps]
    outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    for o in outs:
        del o["iters"]
    dqj.render_batch(ps, outs)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(to_numpy(o), r, f"general batch frame {i}")
    prn = [p.replace(norm=workloads.NORM_REALPART) for p in ps[:2]]
    for p in prn:
        p.__post_init__()
    refs = [counting_ref(dqj, p) for p in prn]
    outs = [dqj.alloc_outputs(p.width, p.height) for p in prn]
    for o in outs:
        del o["iters"]
    dqj.render_batch(prn, outs)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, refs)):
        assert_same(to_numpy(o), r, f"realpart batch frame {i}")


def test_nocount_sweep_plan(dqj):
    """256 sweep frames in one plan: every frame switch happens inside waves."""
    import torch
    ps = workloads.sweep_256(256, first_seed=1000)
    counted = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    cplan = dqj.BatchPlan(ps, counted)
    cplan.launch()
    torch.cuda.synchronize()
    cplan.close()
    timed = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
              if k != "iters"} for p in ps]
    plan = dqj.BatchPlan(ps, timed)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for i, (t, c) in enumerate(zip(timed, counted)):
            for k in ("mask", "depth", "shade"):
                assert torch.equal(t[k], c[k]), f"replay {rep} frame {i} {k}"
    plan.close()


def test_nocount_guided_chunks(dqj):
    """A launch with many tiles per wave takes its tiles in guided chunks (a kernel
    instantiation of its own): up to 8 consecutive tiles per atomic, falling to 1 near the
    end, across frame ends. One wave per CU and 4 x 2 tiles bring 20 sweep frames to 640
    tiles per wave, so every chunk size occurs; the outputs must equal the counting
    plan's, which takes one tile at a time."""
    import torch
    ps = workloads.sweep_256(20, first_seed=3000)
    counted = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
    cplan = dqj.BatchPlan(ps, counted)
    cplan.launch()
    torch.cuda.synchronize()
    cplan.close()
    s = dqj.make_schedule(kernel=dqj.KERNEL_REFILL, tile_w=4, tile_h=2, waves_per_block=1,
                          blocks_per_cu=1)
    timed = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
              if k != "iters"} for p in ps]
    say("guided plan, 20 frames of 256^2, 4x2 tiles, one wave per CU")
    plan = dqj.BatchPlan(ps, timed, schedule=s)
    for rep in range(2):
        for t in timed:
            t["mask"].fill_(7)
        plan.launch()
        torch.cuda.synchronize()
        for i, (t, c) in enumerate(zip(timed, counted)):
            for k in ("mask", "depth", "shade"):
                assert torch.equal(t[k], c[k]), f"replay {rep} frame {i} {k}"
    plan.close()
