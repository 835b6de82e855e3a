"""GPU parity of the FP32 path against the FP64 oracle (through the C ABI).

Bar (per frame): >= 99.9 % of pixels agree (both miss, or both hit with depth within
1e-4 of the box diagonal); every mismatch within one march step of the boundary;
shade within 1/255 on >= 99.9 % of agreeing hits; executed-work counter within
0.1 % of the oracle's. Images must be bit-identical across schedules, between a
batched and a single-frame launch, and across graph replays.
"""
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
    info = m.device_info(0)
    assert info["arch"].startswith("gfx950"), info
    return m


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


def render_np(dqj, p, schedule=None):
    import torch
    out = dqj.render(p, schedule=schedule)
    torch.cuda.synchronize()
    return to_numpy(out)


def check_frame(dqj, oracle_mod, p, schedule=None, iters_rel=1e-3):
    say("render", p.width, p.height, "N", p.max_iter, "S", p.march_steps, "B", p.bisect_steps,
        "c", p.c[:2], "sched", None if schedule is None else schedule.kernel)
    g = render_np(dqj, p, schedule)
    o = oracle_mod.render(p)
    rep = compare(p, g, o)
    say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
    assert_parity(rep)
    if o["total_iters"] > 0:
        rel = abs(int(g["iters"][0]) - o["total_iters"]) / o["total_iters"]
        assert rel <= iters_rel, (int(g["iters"][0]), o["total_iters"])
    # outputs that have exact meanings
    miss = g["mask"] == 0
    assert np.all(np.isinf(g["depth"][miss])) and np.all(g["shade"][miss] == 0)
    assert np.all(g["first_hit"][miss] == -1)
    hit = ~miss
    if hit.any():
        nl = np.linalg.norm(g["normal"][hit], axis=-1)
        assert np.all(np.abs(nl - 1) < 1e-5)
        expect8 = np.floor(255.0 * g["shade"].astype(np.float64) + 0.5)
        assert np.all(np.abs(g["image8"].astype(np.float64) - expect8) <= 1)
    return g, o, rep


# ---------------------------------------------------------------- classify

@pytest.mark.parametrize("seed", [0, 2])
def test_classify_points_fp32_fp64(dqj, oracle_mod, seed):
    import torch
    rng = np.random.default_rng(100 + seed)
    p = workloads.plain_1024([seed])[0]
    pts = np.zeros((20000, 8))
    pts[:10000, :3] = rng.uniform(-1.5, 1.5, (10000, 3))
    pts[10000:] = rng.uniform(-1.0, 1.0, (10000, 8))
    pts = pts.astype(np.float32).astype(np.float64)   # the same FP32 points on both sides
    o = oracle_mod.classify(p, pts)
    o_esc = np.where(o["inside"] == 1, 0, o["m"])
    say("classify fp32", seed)
    esc32, _ = dqj.classify_points(torch.tensor(pts, dtype=torch.float32, device="cuda"), p,
                                   dqj.PREC_FP32)
    esc32 = esc32.cpu().numpy()
    assert (esc32 == o_esc).mean() >= 0.999
    say("classify fp64", seed)
    esc64, n2 = dqj.classify_points(torch.tensor(pts, dtype=torch.float64, device="cuda"), p,
                                    dqj.PREC_FP64)
    esc64 = esc64.cpu().numpy()
    assert (esc64 == o_esc).mean() >= 0.9999
    assert np.all((esc64 == 0) <= (esc64 >= 0))


def test_classify_mirror_bitwise(dqj):
    import torch
    c = [0.2, -0.55, 0, 0, 0.3, 0.25, 0, 0]
    p = workloads.plain_128()[0].replace(c=c, max_iter=14)
    p.__post_init__()
    rng = np.random.default_rng(7)
    xyz = rng.uniform(-1.5, 1.5, (5000, 3)).astype(np.float32)
    a = np.zeros((5000, 8), np.float32)
    a[:, :3] = xyz
    b = a.copy()
    b[:, 2] = -b[:, 2]
    ea, na = dqj.classify_points(torch.tensor(a, device="cuda"), p, dqj.PREC_FP32)
    eb, nb = dqj.classify_points(torch.tensor(b, device="cuda"), p, dqj.PREC_FP32)
    assert torch.equal(ea, eb) and torch.equal(na, nb)


# ---------------------------------------------------------------- frames

def test_plain_128_refill_and_direct(dqj, oracle_mod):
    p = workloads.plain_128()[0]
    check_frame(dqj, oracle_mod, p)
    check_frame(dqj, oracle_mod, p, schedule=dqj.make_schedule(kernel=dqj.KERNEL_DIRECT))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_1024_shape_at_256(dqj, oracle_mod, seed):
    p = workloads.plain_1024([seed])[0].replace(width=256, height=256)
    check_frame(dqj, oracle_mod, p)


def test_c0_sphere_closed_form(dqj, oracle_mod):
    N, S, B = 12, 128, 8
    p = workloads.Params(c=[0.0] * 8, width=96, height=96, max_iter=N, march_steps=S,
                         bisect_steps=B)
    g = render_np(dqj, p)
    rho = 4.0 ** (2.0 ** -N)
    l = np.array(p.light_dir) / np.linalg.norm(p.light_dir)
    n_checked = 0
    for j in range(0, 96, 3):
        for i in range(0, 96, 3):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            b = np.dot(o, d)
            disc = b * b - (np.dot(o, o) - rho * rho)
            dt = (t1 - t0) / S
            if disc < 0:
                assert g["mask"][j, i] == 0
                continue
            if 2 * math.sqrt(disc) < dt + 1e-6:
                continue
            assert g["mask"][j, i] == 1
            ts = -b - math.sqrt(disc)
            assert abs(g["depth"][j, i] - ts) <= dt * 2.0 ** -(B + 1) + 2e-6
            ph = o + g["depth"][j, i] * d
            nrm = ph / np.linalg.norm(ph)
            assert np.max(np.abs(g["normal"][j, i] - nrm)) < 2e-3
            sh = min(1.0, p.k_ambient + p.k_diffuse * max(0.0, float(np.dot(nrm, l))))
            assert abs(g["shade"][j, i] - sh) <= 1.0 / 255.0
            n_checked += 1
    assert n_checked > 200


@pytest.mark.parametrize("case", [
    "ragged_131x97", "tiny_1x1", "strip_1x64", "B0", "S1", "N1", "realpart", "dual_slice",
    "eye_inside_box", "paper_highres", "paper_test2_0",
])
def test_edge_cases(dqj, oracle_mod, case):
    base = workloads.plain_128()[0]
    if case == "ragged_131x97":
        p = base.replace(width=131, height=97)
    elif case == "tiny_1x1":
        p = base.replace(width=1, height=1, eye=[0.0, 0.0, 3.0], c=[-0.2, 0.1, 0, 0, 0, 0, 0, 0])
    elif case == "strip_1x64":
        p = base.replace(width=1, height=64)
    elif case == "B0":
        p = base.replace(bisect_steps=0)
    elif case == "S1":
        p = base.replace(march_steps=1, c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0])
    elif case == "N1":
        p = base.replace(max_iter=1)
    elif case == "realpart":
        p = base.replace(norm=workloads.NORM_REALPART)
    elif case == "dual_slice":
        axes = [[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1.0, 0, 0, 0]]
        p = base.replace(slice_axes=axes, slice_origin=[0, 0, 0.1, 0, 0, 0, 0, 0],
                         c=[-0.39054, -0.58679, 0, 0, 0.0, 0.5632, 0, 0.05], max_iter=15)
    elif case == "eye_inside_box":
        p = base.replace(eye=[0.3, 0.2, 1.4], target=[0.0, 0.0, 0.0], fov_y_deg=90.0,
                         c=[-0.2, 0.1, 0, 0, 0.1, 0, 0, 0])
    elif case == "paper_highres":
        p = base.replace(c=workloads.PAPER_C[7], max_iter=15)
    else:
        p = base.replace(c=workloads.PAPER_C[0])
    p.__post_init__()
    check_frame(dqj, oracle_mod, p)


def test_plain_1024_full_size_sampled(dqj, oracle_mod):
    """The 1024x1024 frame in the benchmark's launch configuration, checked on sampled
    pixels (all of them for the oracle would take minutes) plus sampled GPU hits."""
    for seed in (0, 2):
        p = workloads.plain_1024([seed])[0]
        say("render 1024", seed)
        g = render_np(dqj, p)
        pix = sample_pixels(p, 3000, seed)
        hits = np.nonzero(g["mask"].reshape(-1))[0]
        if hits.size:
            rng = np.random.default_rng(seed)
            pix = np.union1d(pix, rng.choice(hits, size=min(1500, hits.size), replace=False))
        o = oracle_mod.render(p, pixels=pix)
        rep = compare(p, g, o, pixels=pix)
        say(" ", {k: v for k, v in rep.items() if k != "mismatch_far_from_boundary"})
        assert_parity(rep)


# ---------------------------------------------------------------- schedules, batch, graph

SCHEDULES = [(8, 8, 4, 8), (16, 4, 1, 16), (4, 16, 2, 4), (32, 32, 8, 2), (1, 64, 4, 8)]


def test_schedule_invariance_bitwise(dqj):
    p = workloads.plain_1024([2])[0].replace(width=257, height=131)
    ref = None
    for tw, th, wpb, bpc in SCHEDULES:
        s = dqj.make_schedule(kernel=dqj.KERNEL_REFILL, tile_w=tw, tile_h=th, waves_per_block=wpb,
                              blocks_per_cu=bpc)
        say("schedule", tw, th, wpb, bpc)
        g = render_np(dqj, p, schedule=s)
        if ref is None:
            ref = g
            continue
        for k in ("mask", "depth", "shade", "normal", "first_hit", "image8", "flags", "iters"):
            np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    # the variant compiled without the work counter gives the same image
    import torch
    out = dqj.alloc_outputs(p.width, p.height)
    del out["iters"]
    dqj.render(p, out=out)
    torch.cuda.synchronize()
    g = to_numpy(out)
    for k in ("mask", "depth", "shade", "normal", "first_hit", "image8", "flags"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg="no-count " + k)


def test_batch_matches_single_and_graph_replays(dqj):
    import torch
    ps = [workloads.plain_128(s)[0] for s in range(3)]
    ps += [workloads.plain_1024([2])[0].replace(width=200, height=120),
           workloads.sweep_256(1, first_seed=6)[0],
           # the specular term and the bounding sphere on the batched kernel
           workloads.plain_128(3)[0].replace(k_specular=0.4, shininess=20.0, cull_radius=1.35)]
    for p in ps:
        p.__post_init__()
    singles = [render_np(dqj, p) for p in ps]
    say("batch eager")
    outs = dqj.render_batch(ps, extras=True)
    torch.cuda.synchronize()
    for o, s in zip(outs, singles):
        o = to_numpy(o)
        for k in ("mask", "depth", "shade", "normal", "first_hit", "iters"):
            np.testing.assert_array_equal(o[k], s[k], err_msg=k)
    say("batch plan")
    outs2 = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    plan = dqj.BatchPlan(ps, outs2)
    for rep in range(3):
        for o in outs2:
            o["depth"].fill_(-1.0)
            o["iters"].zero_()
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
        for o, s in zip(outs2, singles):
            o = to_numpy(o)
            for k in ("mask", "depth", "shade", "iters"):
                np.testing.assert_array_equal(o[k], s[k], err_msg=f"replay {rep} {k}")
    plan.close()


def test_autotune_remembers_and_keeps_images(dqj, tmp_path):
    import torch
    ps = workloads.sweep_256(6, first_seed=200)
    ref = [render_np(dqj, p) for p in ps]
    outs = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    cache = tmp_path / "tune.jsonl"
    best = dqj.autotune(ps, outs, str(cache))
    say("autotuned", best.tile_w, best.tile_h, best.waves_per_block, best.blocks_per_cu)
    line = cache.read_text().strip().splitlines()[-1]
    assert "W=256,H=256,N=16,S=256,B=8" in line and f'"tile_w": {best.tile_w}' in line
    # a plan without an explicit schedule now uses the tuned one; images are unchanged
    outs2 = [dqj.alloc_outputs(p.width, p.height) for p in ps]
    plan = dqj.BatchPlan(ps, outs2)
    plan.launch()
    torch.cuda.synchronize()
    for o, r in zip(outs2, ref):
        o = to_numpy(o)
        for k in ("mask", "depth", "shade", "normal", "iters"):
            np.testing.assert_array_equal(o[k], r[k], err_msg=k)
    plan.close()
