"""dqj_render_noalloc (the render entry point that allocates no device memory) against
dqj_render: both run the same kernels, so every output must agree bit for bit. Each
case makes two calls in a row, the second on a smaller frame, so the second runs on
the fixed scratch the first one left behind."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads
from parity import to_numpy

pytestmark = pytest.mark.gpu

KEYS = ("mask", "depth", "shade", "normal", "first_hit", "image8", "flags", "iters")


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


def via_render(dqj, p):
    import torch
    out = dqj.alloc_outputs(p.width, p.height)
    dqj.render(p, out=out)
    torch.cuda.synchronize()
    return to_numpy(out)


def via_noalloc(dqj, p, out):
    """Call the C entry point directly with the caller's buffers."""
    import torch
    sp = dqj.make_params(p)
    fo = dqj.make_frame_out(out, p)
    st = dqj.lib().dqj_render_noalloc(C.byref(sp), C.byref(fo), None)
    assert st == dqj.OK, dqj.lib().dqj_last_error().decode()
    torch.cuda.synchronize()
    return to_numpy(out)


def check_pair(dqj, big, small, what):
    import torch
    outs = []
    for p in (big, small):
        o = dqj.alloc_outputs(p.width, p.height)
        for k, v in o.items():   # garbage in the outputs: every element must be written
            if v.dtype.is_floating_point:
                v.fill_(-7.0)
            else:
                v.fill_(3)
        o["iters"].zero_()
        outs.append(o)
    got = []
    for i, (p, o) in enumerate(zip((big, small), outs)):
        say(what, "call", i + 1, p.width, p.height, "precision", p.precision, "march", p.march)
        got.append(via_noalloc(dqj, p, o))
    torch.cuda.synchronize()
    for i, (p, g) in enumerate(zip((big, small), got)):
        ref = via_render(dqj, p)
        for k in KEYS:
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"{what} call {i + 1}: {k}")
        assert int(g["mask"].sum()) > 0, f"{what} call {i + 1} has no hits"


def test_noalloc_fp32(dqj):
    big = workloads.plain_1024([1])[0].replace(width=320, height=240)
    small = workloads.plain_128(0)[0].replace(width=97, height=61)
    for p in (big, small):
        p.__post_init__()
    check_pair(dqj, big, small, "fp32")


def test_noalloc_split(dqj):
    big = workloads.split_1080p([3])[0].replace(width=512, height=512)   # the largest split frame
    small = workloads.split_1080p([5])[0].replace(width=200, height=120)
    for p in (big, small):
        p.__post_init__()
    assert big.width * big.height == dqj.NOALLOC_MAX_SPLIT_PIXELS
    check_pair(dqj, big, small, "split")


def test_noalloc_distance_estimate(dqj):
    big = workloads.plain_128(2)[0].replace(width=192, height=160, march=workloads.MARCH_DE)
    small = workloads.plain_128(4)[0].replace(width=64, height=33, march=workloads.MARCH_DE)
    for p in (big, small):
        p.__post_init__()
    check_pair(dqj, big, small, "de")


def test_noalloc_rejects_split_beyond_limit(dqj):
    """A split frame over the limit is refused on the host, before any launch."""
    import torch
    p = workloads.split_1080p([0])[0].replace(width=512, height=513)
    p.__post_init__()
    out = dqj.alloc_outputs(p.width, p.height)
    sp = dqj.make_params(p)
    fo = dqj.make_frame_out(out, p)
    st = dqj.lib().dqj_render_noalloc(C.byref(sp), C.byref(fo), None)
    assert st == dqj.E_INVALID
    assert "fixed scratch" in dqj.lib().dqj_last_error().decode()
    torch.cuda.synchronize()
    # and a frame within the limit still renders afterwards
    ok = workloads.plain_128(0)[0]
    check_pair(dqj, ok, ok.replace(width=40, height=40), "after_refusal")
