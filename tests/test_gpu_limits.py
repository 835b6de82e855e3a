"""GPU parity at the limits the public header allows, through the C ABI.

* Largest sides (16384): a 16384 x 1 row and a 1 x 16384 column, every pixel against the
  FP64 oracle, for the FP32, split and distance-estimate paths.
* A 16384 x 16384 frame with every extra output (7.2 GB on the device; the normal's float
  offsets reach 3 x 2^28): sampled pixels, the four corners and sampled GPU hits.
* Large max_iter: 64 (the request stream's largest), 200 and 4096 (the largest allowed),
  whole frames against the oracle in every precision and kernel, both marches and
  projection. The normal's stencil is formed relative to its least escape index; without
  that, its terms or their squares flush to zero in FP32 beyond about m = 53, and such
  hits would fall back to the reversed ray direction. The frames locate their hits far
  more precisely than the stencil step, as every workload does; with coarse bisection all
  six stencil points of a hit can stay inside, and at large max_iter the normal of such a
  hit is rounding noise on either side.
* Largest march_steps (2^20, with max_iter 2 under the (S + B + 8) N <= 2^30 rule) and the
  largest bisect_steps (64).
* Voxel grids: 4096 x 4096 x 512 (8.6e9 voxels, past 2^32, so the kernel's 64-bit voxel
  indices run; 43 GB of mask and escape indices) on sampled voxels, the extreme ones among
  them, with the update counter against the escape indices summed on the device; and a
  48^3 grid at max_iter 4096, whole.
"""
import sys

import numpy as np
import pytest

import workloads
from parity import assert_parity, compare, sample_pixels, to_numpy

pytestmark = pytest.mark.gpu

FIXED_BAR = (0.999, 0.999)
LOOSE_SHADE_BAR = (0.999, 0.99)   # distance-estimate march and projection, as their own tests


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


def as_mode(dqj, p, mode):
    """(params, schedule, bar) of a render mode."""
    if mode == "split":
        return p.replace(precision=workloads.PREC_SPLIT), None, FIXED_BAR
    if mode == "direct":
        return p, dqj.make_schedule(kernel=dqj.KERNEL_DIRECT), FIXED_BAR
    if mode.startswith("de_"):
        k = {"de_direct": dqj.KERNEL_DIRECT, "de_refill": dqj.KERNEL_REFILL,
             "de_lockstep": dqj.KERNEL_LOCKSTEP}[mode]
        return p.replace(march=workloads.MARCH_DE), dqj.make_schedule(kernel=k), LOOSE_SHADE_BAR
    if mode == "project":
        return p.replace(fiber=workloads.fiber_ball(8, 0.5, 100)), None, LOOSE_SHADE_BAR
    return p, None, FIXED_BAR   # "refill", "batch"


def render_mode(dqj, p, mode, schedule):
    import torch
    if mode == "batch":   # the timed instantiation: a plan without extras or counter
        outs = [{k: v for k, v in dqj.alloc_outputs(p.width, p.height, extras=False).items()
                 if k != "iters"}]
        plan = dqj.BatchPlan([p], outs)
        plan.launch()
        torch.cuda.synchronize()
        plan.close()
        return to_numpy(outs[0])
    out = dqj.render(p, schedule=schedule)
    torch.cuda.synchronize()
    return to_numpy(out)


def check_whole(dqj, oracle_mod, p, mode, name):
    q, schedule, bar = as_mode(dqj, p, mode)
    say("limits", name, mode, q.width, "x", q.height, "N", q.max_iter, "S", q.march_steps,
        "B", q.bisect_steps)
    g = render_mode(dqj, q, mode, schedule)
    o = oracle_mod.render(q)
    rep = compare(q, g, o)
    say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep, *bar)
    # (the split path counts its FP16 march and re-checks, not the oracle's updates). A
    # point that FP32 and FP64 classify differently, within rounding of the boundary, moves
    # the count by up to max_iter updates: at max_iter 4096 a few such points exceed 0.1%.
    if mode != "split" and "iters" in g and o["total_iters"] > 0:
        diff = abs(int(g["iters"][0]) - o["total_iters"])
        assert diff <= max(1e-3 * o["total_iters"], 4 * q.max_iter), (int(g["iters"][0]),
                                                                        o["total_iters"])
    if "flags" in g and rep["hits_gpu"] and mode in ("refill", "direct", "split"):
        # no hit of these frames falls back to the reversed ray direction
        assert not np.any((g["flags"] & 8) != 0), "normal fell back on a hit"
    return g, o, rep


# ---------------------------------------------------------------- large max_iter

BIG_N = {
    "N64": lambda: workloads.plain_128(2)[0].replace(width=96, height=96, max_iter=64,
                                                     march_steps=256, bisect_steps=8),
    "N200": lambda: workloads.plain_128(0)[0].replace(width=64, height=64, c=workloads.PAPER_C[0],
                                                      max_iter=200, march_steps=64, bisect_steps=8),
    "N4096": lambda: workloads.plain_128(0)[0].replace(width=32, height=32,
                                                       c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0],
                                                       max_iter=4096, march_steps=128, bisect_steps=10),
}
MODES = ["refill", "batch", "direct", "split", "de_direct", "de_refill", "de_lockstep", "project"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", list(BIG_N))
def test_large_max_iter(dqj, oracle_mod, case, mode):
    g, o, rep = check_whole(dqj, oracle_mod, BIG_N[case](), mode, case)
    assert rep["hits_oracle"] >= 15, rep   # the frames have hits to shade



# ---------------------------------------------------------------- largest sides

SIDES = {
    # (with a vertical field of 60/16384 degrees the row spans about 60 degrees across)
    "row_16384": lambda: workloads.plain_128(2)[0].replace(width=16384, height=1,
                                                           fov_y_deg=60.0 / 16384),
    "column_16384": lambda: workloads.plain_128(2)[0].replace(width=1, height=16384),
}


@pytest.mark.parametrize("mode", ["refill", "split", "de_direct"])
@pytest.mark.parametrize("case", list(SIDES))
def test_largest_side(dqj, oracle_mod, case, mode):
    g, o, rep = check_whole(dqj, oracle_mod, SIDES[case](), mode, case)
    assert rep["hits_oracle"] > 0, rep


def test_largest_frame_sampled(dqj, oracle_mod):
    """16384 x 16384 with every extra output, compared on sampled pixels gathered on the
    device (the full outputs are 7.2 GB)."""
    import torch
    p = workloads.plain_128(2)[0].replace(width=16384, height=16384)
    W, H = p.width, p.height
    say("limits 16384^2: render")
    out = dqj.render(p)
    torch.cuda.synchronize()
    pix = sample_pixels(p, 3000, 7)
    corners = np.array([0, W - 1, (H - 1) * W, H * W - 1])
    hit_idx = torch.nonzero(out["mask"].reshape(-1)).reshape(-1)
    say("  GPU hits", int(hit_idx.numel()))
    rng = np.random.default_rng(7)
    hits = hit_idx[torch.from_numpy(rng.choice(int(hit_idx.numel()), size=1500, replace=False))
                   .to(hit_idx.device)].cpu().numpy() if hit_idx.numel() > 1500 else \
        hit_idx.cpu().numpy()
    pix = np.union1d(np.union1d(pix, corners), hits)
    sel = torch.from_numpy(pix).to(out["mask"].device)
    g = {k: out[k].reshape(-1)[sel].cpu().numpy() for k in ("mask", "depth", "shade", "first_hit")}
    normal = out["normal"].reshape(-1, 3)[sel].cpu().numpy()
    o = oracle_mod.render(p, pixels=pix)
    rep = compare(p, g, o, pixels=pix, gathered=True)
    say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert rep["hits_oracle"] > 500, rep
    assert_parity(rep, *FIXED_BAR)
    hit = g["mask"] == 1
    assert np.all(np.abs(np.linalg.norm(normal[hit], axis=1) - 1.0) < 1e-5)
    assert np.all(normal[~hit] == 0)


# ---------------------------------------------------------------- march and bisection steps

@pytest.mark.parametrize("mode", ["refill", "split"])
def test_largest_march_steps(dqj, oracle_mod, mode):
    p = workloads.plain_128(2)[0].replace(width=6, height=6, max_iter=2, march_steps=1 << 20,
                                          bisect_steps=8, target=[0.2, 0.1, 0.0], fov_y_deg=30.0)
    check_whole(dqj, oracle_mod, p, mode, "S2^20")


@pytest.mark.parametrize("mode", ["refill", "batch", "split"])
def test_largest_bisect_steps(dqj, oracle_mod, mode):
    p = workloads.plain_128(2)[0].replace(width=64, height=64, bisect_steps=64)
    g, o, rep = check_whole(dqj, oracle_mod, p, mode, "B64")
    assert rep["hits_oracle"] > 100, rep
    assert rep["depth_err_max_E"] <= 1e-6, rep   # 64 halvings: limited by the FP32 depth only


# ---------------------------------------------------------------- voxel grids

def test_grid_past_32_bit_indices(dqj, oracle_mod):
    import torch
    p, _ = workloads.voxel_grid(8)
    dims = (4096, 4096, 512)
    nvox = dims[0] * dims[1] * dims[2]
    assert nvox > 1 << 32
    say("limits grid", dims)
    r = dqj.classify_grid(p, *dims, extras=True)
    torch.cuda.synchronize()
    mask, esc = r["mask"].reshape(-1), r["escape"].reshape(-1)
    # the counter is the escape indices (max_iter inside) summed, here in slices on the device
    total = 0
    step = 1 << 30
    for a in range(0, nvox, step):
        m, e = mask[a:a + step], esc[a:a + step]
        total += int(torch.where(m == 1, torch.full_like(e, p.max_iter), e).sum(dtype=torch.int64))
    say("  counter", int(r["iters"][0]), "sum", total, "inside", int(mask.sum(dtype=torch.int64)))
    assert int(r["iters"][0]) == total
    rng = np.random.default_rng(9)
    lo = nvox // 2 - (1 << 29)   # inside voxels of the middle slices, across voxel 2^32
    inside = torch.nonzero(mask[lo:lo + (1 << 30)]).reshape(-1)
    pick = inside[torch.from_numpy(rng.choice(int(inside.numel()), 3000, replace=False))
                  .to(inside.device)].cpu().numpy() + lo
    extremes = np.array([0, dims[0] - 1, dims[0] * dims[1] - 1, (1 << 32) - 1, 1 << 32, (1 << 32) + 1,
                         nvox - dims[0], nvox - 1], dtype=np.int64)
    idx = np.unique(np.concatenate([rng.integers(0, nvox, 20000, dtype=np.int64), pick, extremes]))
    sel = torch.from_numpy(idx).to(mask.device)
    g = {"mask": mask[sel].cpu().numpy(), "escape": esc[sel].cpu().numpy()}
    import test_gpu_grid as T
    o = oracle_mod.classify_grid(p, *dims, voxels=idx)
    agree = float(np.mean(g["mask"] == o["inside"]))
    agree_m = float(np.mean(g["escape"] == o["m"]))
    bad = np.nonzero(g["mask"] != o["inside"])[0]
    far = 0
    if bad.size:
        x = T.centres(p, *dims, idx[bad[:200]])
        far = int(np.sum(~T.near_boundary(oracle_mod, p, x, o["inside"][bad[:200]])))
    say("  ", {"voxels": int(idx.size), "inside_oracle": int(o["inside"].sum()), "class_agree": agree,
               "escape_index_agree": agree_m, "class_mismatch": int(bad.size), "far": far})
    assert agree >= 0.999 and agree_m >= 0.999 and far == 0
    assert int(o["inside"].sum()) > 2000


def test_grid_max_iter_4096(dqj):
    from test_gpu_grid import check_against_oracle
    p, _ = workloads.voxel_grid(8)
    p = p.replace(c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0], max_iter=4096)
    say("limits grid N4096")
    g, o, rep = check_against_oracle(dqj, p, (48, 48, 48))
    assert rep["inside_oracle"] > 1000, rep
    gm, ge = g["mask"].reshape(-1), g["escape"].reshape(-1)
    assert int(g["iters"][0]) == int(np.where(gm == 1, p.max_iter, ge).sum())


# ---------------------------------------------------------------- empty inputs

def test_empty_inputs(dqj):
    """Zero-sized inputs on the device: a batch or a plan of no frames and a grid with a
    zero side are refused as invalid, and nothing is launched; zero points classify to
    nothing."""
    import ctypes as C
    import torch
    p = workloads.plain_128(0)[0]
    arr_p = (dqj.dqj_params * 1)(dqj.make_params(p))
    arr_o = (dqj.dqj_frame_out * 1)()
    assert dqj.lib().dqj_render_batch(arr_p, arr_o, 0, None) == dqj.E_INVALID
    plan = C.c_void_p()
    assert dqj.lib().dqj_batch_plan_create(arr_p, arr_o, 0, None, None, C.byref(plan)) == \
        dqj.E_INVALID
    assert not plan.value
    mask = torch.zeros(16, dtype=torch.uint8, device="cuda")
    sp = dqj.make_params(p)
    for dims in ((0, 4, 4), (4, 0, 4), (4, 4, 0)):
        assert dqj.lib().dqj_classify_grid(C.byref(sp), *dims, C.c_void_p(mask.data_ptr()), None,
                                           None, None) == dqj.E_INVALID
    torch.cuda.synchronize()
    assert int(mask.sum()) == 0   # untouched
    esc, n2 = dqj.classify_points(torch.empty((0, 8), dtype=torch.float32, device="cuda"), p)
    torch.cuda.synchronize()
    assert esc.numel() == 0 and n2.numel() == 0
