"""GPU voxel-grid classification (dqj_classify_grid) against the FP64 oracle.

FP32 and FP64 can classify a voxel differently only where the set's boundary passes
within rounding reach of its centre. The bar: >= 99.9% of voxels agree in class and in
escape index, and every voxel whose class differs has an FP64 class change among points
5e-4 (1e-4 of the box diagonal) away from its centre. The c = 0 case is checked against
its closed form: the ball of radius R^(2^-N) and the escape index of |p|^(2^n) > R.
"""
import math
import sys

import numpy as np
import pytest

import workloads

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


def gpu_grid(dqj, p, nx, ny, nz, extras=True):
    import torch
    r = dqj.classify_grid(p, nx, ny, nz, extras=extras)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in r.items()}


def centres(p, nx, ny, nz, idx):
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    lo, hi = np.asarray(p.box_min, float), np.asarray(p.box_max, float)
    return np.stack([lo[0] + (i + 0.5) * (hi[0] - lo[0]) / nx,
                     lo[1] + (j + 0.5) * (hi[1] - lo[1]) / ny,
                     lo[2] + (k + 0.5) * (hi[2] - lo[2]) / nz], axis=-1)


def near_boundary(oracle, p, x, cls, h=5e-4):
    """True where some point at distance h (26 directions) has the other FP64 class."""
    dirs = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                     if (a, b, c) != (0, 0, 0)], float)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    pts = (x[:, None, :] + h * dirs[None]).reshape(-1, 3)
    z = np.zeros((len(pts), 8))
    for q in range(len(pts)):
        z[q] = oracle.slice_map(p, pts[q])
    ins = oracle.classify(p, z)["inside"].reshape(len(x), -1)
    return np.any(ins != cls[:, None], axis=1)


def check_against_oracle(dqj, p, dims, idx=None, g=None):
    import oracle
    nx, ny, nz = dims
    if g is None:
        g = gpu_grid(dqj, p, nx, ny, nz)
    gm, ge = g["mask"].reshape(-1), g["escape"].reshape(-1)
    if idx is None:
        o = oracle.classify_grid(p, nx, ny, nz)
        om, oe = o["inside"].reshape(-1), o["m"].reshape(-1)
        idx = np.arange(gm.size)
    else:
        o = oracle.classify_grid(p, nx, ny, nz, voxels=idx)
        om, oe = o["inside"], o["m"]
    gm, ge = gm[idx], ge[idx]
    agree = float(np.mean(gm == om))
    agree_m = float(np.mean(ge == oe))
    bad = np.nonzero(gm != om)[0]
    far = 0
    if bad.size:
        x = centres(p, nx, ny, nz, idx[bad[:200]])
        far = int(np.sum(~near_boundary(oracle, p, x, om[bad[:200]])))
    rep = {"voxels": int(idx.size), "inside_oracle": int(om.sum()), "class_agree": agree,
           "escape_index_agree": agree_m, "class_mismatch": int(bad.size),
           "mismatch_far_from_boundary": far}
    say(rep)
    assert agree >= 0.999 and agree_m >= 0.999 and far == 0, rep
    return g, o, rep


@pytest.mark.parametrize("case", ["paper_c_ragged", "seeded_c", "realpart", "componentwise",
                                  "dual_slice", "N1", "N2"])
def test_grid_small_full(dqj, case):
    p, _ = workloads.voxel_grid(8)
    dims = (67, 45, 33)      # ragged runs (67 = 64 + 3) and several chunks
    if case == "seeded_c":
        p = p.replace(c=workloads.seeded_c(3, 0.6), max_iter=24)
    elif case == "realpart":
        p = p.replace(norm=workloads.NORM_REALPART)
    elif case == "componentwise":
        p = p.replace(algebra=workloads.ALGEBRA_COMPONENTWISE, c=[-0.2, 0.5, 0.1, 0.0, 0.2, -0.3, 0.1, 0.0])
    elif case == "dual_slice":
        p = p.replace(slice_axes=[[1.0, 0, 0, 0, 0, 0, 0, 0], [0, 1.0, 0, 0, 0, 0, 0, 0],
                                  [0, 0, 0, 0, 1.0, 0, 0, 0]],
                      slice_origin=[0, 0, 0.1, 0, 0, 0, 0, 0])
    elif case == "N1":
        p = p.replace(max_iter=1)
    elif case == "N2":
        p = p.replace(max_iter=2)
    p.__post_init__()
    say(case)
    g, o, rep = check_against_oracle(dqj, p, dims)
    # the update counter is the escape indices (max_iter inside) summed
    gm, ge = g["mask"].reshape(-1), g["escape"].reshape(-1)
    assert int(g["iters"][0]) == int(np.where(gm == 1, p.max_iter, ge).sum())
    assert abs(int(g["iters"][0]) - o["total_iters"]) <= 2 * p.max_iter * rep["class_mismatch"] + \
        int(0.001 * o["total_iters"])
    # without extras the mask is the same
    g2 = gpu_grid(dqj, p, *dims, extras=False)
    np.testing.assert_array_equal(g2["mask"], g["mask"])


@pytest.mark.parametrize("N", [6, 12])
def test_grid_c0_closed_form(dqj, N):
    n = 96
    p, _ = workloads.voxel_grid(n, c=[0.0] * 8, max_iter=N)
    g = gpu_grid(dqj, p, n, n, n)
    x = centres(p, n, n, n, np.arange(n ** 3))
    r = np.linalg.norm(x, axis=1)
    R = p.escape_radius
    rho = R ** (2.0 ** -N)
    away = np.abs(r - rho) > 1e-5
    np.testing.assert_array_equal(g["mask"].reshape(-1)[away], (r <= rho)[away])
    out = (r > 1.0) & (g["mask"].reshape(-1) == 0)
    e = np.log2(math.log(R) / np.log(r[out]))
    ok = np.abs(e - np.round(e)) > 2e-3          # away from escape-index ties (FP32 reach)
    ns = np.maximum(np.floor(e) + 1, 1)
    np.testing.assert_array_equal(g["escape"].reshape(-1)[out][ok], ns[ok].astype(np.int32))


def test_grid_1024_sampled(dqj):
    """The benchmark's 1024^3 grid of the paper's high-detail constant, on sampled voxels
    (random ones plus GPU-inside ones) and the update count against the stored oracle total."""
    import json
    import os
    p, dims = workloads.voxel_1024()
    g = gpu_grid(dqj, p, *dims)
    n = int(np.prod(dims))
    rng = np.random.default_rng(5)
    inside = np.nonzero(g["mask"].reshape(-1))[0]
    idx = np.union1d(rng.integers(0, n, 20000), rng.choice(inside, 5000, replace=False))
    check_against_oracle(dqj, p, dims, idx=idx, g=g)
    with open(os.path.join(os.path.dirname(__file__), "golden", "ialg_voxel_1024.json")) as f:
        gold = json.load(f)
    say("gpu iters", int(g["iters"][0]), "oracle", gold["total_iters"], "inside gpu", inside.size,
        "oracle", gold["inside"])
    assert abs(int(g["iters"][0]) - gold["total_iters"]) < 1e-4 * gold["total_iters"]
    assert abs(inside.size - gold["inside"]) < 1e-4 * gold["inside"]


def test_grid_rejections(dqj):
    import ctypes
    import torch
    p, _ = workloads.voxel_grid(8)
    sp = dqj.make_params(p)
    m = torch.empty(8, dtype=torch.uint8, device="cuda")
    L = dqj.lib()
    for dims in [(0, 2, 2), (4097, 1, 1), (2, -1, 2)]:
        assert L.dqj_classify_grid(ctypes.byref(sp), *dims, ctypes.c_void_p(m.data_ptr()), None,
                                   None, None) == dqj.E_INVALID
    assert L.dqj_classify_grid(ctypes.byref(sp), 2, 2, 2, None, None, None, None) == dqj.E_INVALID
    sp2 = dqj.make_params(p.replace(precision=workloads.PREC_SPLIT))
    assert L.dqj_classify_grid(ctypes.byref(sp2), 2, 2, 2, ctypes.c_void_p(m.data_ptr()), None,
                               None, None) == dqj.E_UNSUPPORTED
    # a render does not take the component-wise algebra
    o = dqj.alloc_outputs(16, 16)
    pr = workloads.plain_128()[0].replace(width=16, height=16, algebra=workloads.ALGEBRA_COMPONENTWISE)
    st = L.dqj_render(ctypes.byref(dqj.make_params(pr)), ctypes.byref(dqj.make_frame_out(o)), None)
    assert st == dqj.E_UNSUPPORTED
    # the smallest grid
    g = gpu_grid(dqj, p, 1, 1, 1)
    assert g["mask"].shape == (1, 1, 1)


def test_grid_paper_size_100(dqj):
    """The paper's larger voxel prototype, 100^3, in full."""
    p, dims = workloads.voxel_100()
    check_against_oracle(dqj, p, dims)
