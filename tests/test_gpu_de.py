"""GPU distance-estimate march (FP32) against the FP64 oracle's DE march, and the
c = 0 closed form: every hit bisected onto the ball of radius R^(2^-N). Every kernel
runs: the one-thread-per-pixel kernel (KERNEL_DIRECT), the persistent lane-refill kernel
(KERNEL_REFILL) and the persistent point-lock-step kernel (KERNEL_LOCKSTEP).

Mask and depth meet the plain path's bar. Shading is held to 99% of agreeing hits
within 1/255 (DE_SHADE_FRAC): a DE hit is where a chaotic estimate first drops below the
threshold, so the FP32 and FP64 marches can stop one step apart (within the depth
tolerance), which shifts the normal's stencil in dust-like parts of the set."""
import sys

import numpy as np
import pytest

import workloads
from parity import assert_parity, compare, sample_pixels, to_numpy

pytestmark = pytest.mark.gpu
DE_SHADE_FRAC = 0.99


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


KERNELS = ["refill", "direct", "lockstep"]


def sched(dqj, kernel):
    k = {"refill": dqj.KERNEL_REFILL, "direct": dqj.KERNEL_DIRECT,
         "lockstep": dqj.KERNEL_LOCKSTEP}[kernel]
    return dqj.make_schedule(kernel=k)


def render(dqj, p, kernel="direct"):
    import torch
    o = dqj.render(p, schedule=sched(dqj, kernel))
    torch.cuda.synchronize()
    return to_numpy(o)


@pytest.mark.parametrize("kernel", KERNELS)
def test_de_c0_closed_form(dqj, kernel):
    from test_oracle_render import analytic_ball
    import oracle
    N, B = 12, 8
    p = workloads.Params(c=[0.0] * 8, width=48, height=48, max_iter=N, march_steps=400,
                         bisect_steps=B, march=workloads.MARCH_DE)
    g = render(dqj, p, kernel)
    rho = 4.0 ** (2.0 ** -N)
    n = 0
    for j in range(p.height):
        for i in range(p.width):
            hit, o, d, t0, t1 = oracle.ray(p, i, j)
            tstar, chord = analytic_ball(o, d, rho)
            if tstar is None:
                assert g["mask"][j, i] == 0
                continue
            if chord < 1e-2:
                continue
            assert g["mask"][j, i] == 1, (i, j)
            assert abs(float(g["depth"][j, i]) - tstar) <= 2.5e-4 * 2.0 ** -B + 2e-6, (i, j)
            n += 1
    say("c0 hits checked", n)
    assert n > 400


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("norm", [workloads.NORM_EUCLID8, workloads.NORM_REALPART])
def test_de_128_full_frame(dqj, norm, kernel):
    import oracle
    p = workloads.de_128()[0].replace(norm=norm)
    g = render(dqj, p, kernel)
    o = oracle.render(p)
    rep = compare(p, g, o)
    say(norm, {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert rep["hits_oracle"] > 300
    assert_parity(rep, 0.999, DE_SHADE_FRAC)


@pytest.mark.parametrize("kernel", KERNELS)
def test_de_1024_sampled(dqj, kernel):
    """The 1024x1024 DE frame in the benchmark's launch configurations."""
    import oracle
    p = workloads.de_1024()[2]
    g = render(dqj, p, kernel)
    pix = sample_pixels(p, 2500, 3)
    hits = np.nonzero(g["mask"].reshape(-1))[0]
    pix = np.union1d(pix, np.random.default_rng(4).choice(hits, 1500, replace=False))
    o = oracle.render(p, pixels=pix)
    rep = compare(p, g, o, pixels=pix)
    say({k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, 0.999, DE_SHADE_FRAC)


@pytest.mark.parametrize("kernel", KERNELS)
def test_de_paper_constant_and_eye_inside_box(dqj, kernel):
    import oracle
    base = workloads.de_128()[0]
    for p in [base.replace(c=workloads.PAPER_C[1], max_iter=15, width=96, height=72),
              base.replace(eye=[0.4, 0.9, 1.2], width=80, height=80)]:
        g = render(dqj, p, kernel)
        o = oracle.render(p)
        rep = compare(p, g, o)
        say({k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep, 0.999, DE_SHADE_FRAC)


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("case", ["ragged_131x97", "tiny_1x1", "S1", "N1", "B0", "dual_slice",
                                  "steps_clamped_small"])
def test_de_edge_cases(dqj, case, kernel):
    """Degenerate sizes and parameters of the DE march on every kernel: a ragged
    frame over several tiles, one pixel, one march step, one update (every estimate is
    that of z_1), no bisection, a slice through the dual part, and a step range so
    narrow that rays run out of steps inside the box."""
    import oracle
    base = workloads.de_128()[0]
    if case == "ragged_131x97":
        p = base.replace(width=131, height=97)
    elif case == "tiny_1x1":
        p = base.replace(width=1, height=1, eye=[0.0, 0.0, 3.0], c=[-0.2, 0.1, 0, 0, 0, 0, 0, 0])
    elif case == "S1":
        p = base.replace(march_steps=1, c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0])
    elif case == "N1":
        p = base.replace(max_iter=1)
    elif case == "B0":
        p = base.replace(bisect_steps=0)
    elif case == "dual_slice":
        axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]]
        p = base.replace(slice_axes=axes, slice_origin=[0, 0, 0.1, 0, 0, 0, 0, 0],
                         c=[-0.39054, -0.58679, 0, 0, 0.0, 0.5632, 0, 0.05], max_iter=15)
    else:
        p = base.replace(de_min_step=1e-3, de_max_step=2e-3, march_steps=200)
    p.__post_init__()
    say(case, kernel)
    g = render(dqj, p, kernel)
    o = oracle.render(p)
    rep = compare(p, g, o)
    say({k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, 0.999, DE_SHADE_FRAC)


def test_de_batch_matches_single(dqj):
    """A batch of DE frames (one launch over a frame table, also graph-captured) gives the
    single renders' results bit for bit."""
    import torch
    ps = [workloads.de_128()[0], workloads.de_128()[0].replace(c=workloads.PAPER_C[7], max_iter=15),
          workloads.de_128()[0].replace(width=97, height=61, norm=workloads.NORM_REALPART)]
    for p in ps:
        p.__post_init__()
    ps = ps[:2]   # one norm per batch
    singles = [render(dqj, p) for p in ps]
    outs = dqj.render_batch(ps, extras=True)
    torch.cuda.synchronize()
    for o, g in zip(outs, singles):
        o = to_numpy(o)
        for k in ("mask", "depth", "shade", "normal", "first_hit", "iters"):
            np.testing.assert_array_equal(o[k], g[k], err_msg=k)
    outs2 = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    plan = dqj.BatchPlan(ps, outs2)
    for rep in range(3):
        plan.launch()
        torch.cuda.synchronize()
        for o, g in zip(outs2, singles):
            o = to_numpy(o)
            for k in ("mask", "depth", "shade"):
                np.testing.assert_array_equal(o[k], g[k], err_msg=f"replay {rep} {k}")
        if rep < 2:
            for o in outs2:
                o["mask"].zero_()
                o["depth"].zero_()
    plan.close()


def test_de_modes_not_offered(dqj):
    import ctypes
    p = workloads.de_128()[0]
    sp = dqj.make_params(p.replace(precision=workloads.PREC_SPLIT))
    fo = dqj.make_frame_out(dqj.alloc_outputs(128, 128))
    st = dqj.lib().dqj_render(ctypes.byref(sp), ctypes.byref(fo), None)
    assert st == dqj.E_UNSUPPORTED
    # a batch shares one march; DE batches are FP32
    with pytest.raises(Exception):
        dqj.render_batch([p, workloads.plain_128()[0]])
    with pytest.raises(Exception):
        dqj.render_batch([p.replace(precision=workloads.PREC_SPLIT)] * 2)
    # the lock-step kernel runs the DE march only
    fixed = workloads.plain_128()[0]
    st = dqj.lib().dqj_render_scheduled(ctypes.byref(dqj.make_params(fixed)), ctypes.byref(fo),
                                        ctypes.byref(dqj.make_schedule(kernel=dqj.KERNEL_LOCKSTEP)),
                                        None)
    assert st == dqj.E_UNSUPPORTED
    with dqj.Server(precision=workloads.PREC_FP32) as srv:
        st, _ = srv.submit_status(p, dqj.alloc_outputs(128, 128, extras=False))
        assert st == dqj.E_UNSUPPORTED


def test_de_count_off_same_image(dqj):
    """Without an update counter, single renders and batches take the DE kernels with the
    counting compiled out; the images are bitwise those of the counting launches."""
    import torch
    ps = workloads.de_128(0) + workloads.de_128(1)
    def outs(count):
        o = [dqj.alloc_outputs(p.width, p.height, extras=False) for p in ps]
        for x in o:
            x["iters"].zero_()
        return o if count else [{k: v for k, v in x.items() if k != "iters"} for x in o]
    a, b = outs(True), outs(False)
    for p, o in zip(ps, a):
        dqj.render(p, out=o)
    for p, o in zip(ps, b):
        dqj.render(p, out=o)
    ba, bb = outs(True), outs(False)
    dqj.render_batch(ps, ba)
    dqj.render_batch(ps, bb)
    torch.cuda.synchronize()
    for x, y, u, v in zip(a, b, ba, bb):
        assert int(x["iters"].item()) > 0 and int(u["iters"].item()) == int(x["iters"].item())
        for k in ("mask", "depth", "shade"):
            assert torch.equal(x[k], y[k]) and torch.equal(x[k], u[k]) and torch.equal(x[k], v[k]), k


def test_de_batch_spill_matches_single(dqj):
    """Full-size DE frames, where the batch kernel hands the marches of each wave's last
    rays to its resume kernel, and a batch of mixed sizes: every output (counts included)
    equals the single renders' bit for bit, over graph replays too."""
    import torch
    big = workloads.de_1024()
    mixed = [big[1].replace(width=97, height=61), big[0].replace(width=300, height=200),
             big[2].replace(width=1, height=1), big[2]]
    for p in mixed:
        p.__post_init__()
    for name, ps in (("de_1024", big), ("mixed", mixed)):
        say("batch", name, [(p.width, p.height) for p in ps])
        singles = [render(dqj, p) for p in ps]
        outs = dqj.render_batch(ps, extras=True)
        torch.cuda.synchronize()
        for f, (o, g) in enumerate(zip(outs, singles)):
            o = to_numpy(o)
            for k in ("mask", "depth", "shade", "normal", "first_hit", "flags", "iters"):
                np.testing.assert_array_equal(o[k], g[k], err_msg=f"{name} frame {f} {k}")
        timed = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
                  if k != "iters"} for p in ps]
        plan = dqj.BatchPlan(ps, timed)
        for rep in range(2):
            for o in timed:
                o["depth"].fill_(-1.0)
            plan.launch()
            torch.cuda.synchronize()
            for f, (o, g) in enumerate(zip(timed, singles)):
                for k in ("mask", "depth", "shade"):
                    np.testing.assert_array_equal(o[k].cpu().numpy(), g[k], err_msg=f"{name} replay {rep} frame {f} {k}")
        plan.close()
