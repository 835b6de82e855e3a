"""Pins of the oracle's iteration and escape rule (Eq. dqjulia2, "Practical Considerations").

* c = 0 with zero dual part: ||z_n|| = ||z_0||^(2^n), so the escape index has a
  closed form and the inside set is the ball of radius R^(2^-N).
* Strict escape test, z_0 never tested: exact binary cases.
* Zero dual part and c_d = 0 reduce to quaternion Julia (Eq. dqjulia); further
  restricted to span(1, i) they reduce to complex Julia, brute-forced with numpy
  complex128 (a library routine that knows nothing of the oracle).
* Symmetries: rotation about the real axis, and the mirror z -> -z.
* Dual numbers are forward-mode derivatives: the dual part of the orbit equals
  the derivative of the real orbit along c_d (finite differences).
* Reading "real part only": the mask cannot depend on c_d.
"""
import math

import numpy as np
import pytest

import workloads


def P(c, N=12, R=4.0, norm=workloads.NORM_EUCLID8):
    # parameters for classify only; c is FP32-rounded by Params like every input
    return workloads.Params(c=c, width=8, height=8, max_iter=N, march_steps=8, bisect_steps=0,
                            escape_radius=R, norm=norm)


def pts8(xyz):
    xyz = np.atleast_2d(np.asarray(xyz, float))
    out = np.zeros((xyz.shape[0], 8))
    out[:, :xyz.shape[1]] = xyz
    return out


def closed_form_escape_c0(r, R):
    """Escape index for c = 0, zero dual part, ||z_0|| = r > 1 (ties excluded by caller)."""
    x = math.log(R) / math.log(r)
    return max(1, math.floor(math.log2(x)) + 1)


def test_escape_index_closed_form_c0(oracle_mod):
    rng = np.random.default_rng(10)
    p = P([0.0] * 8, N=30, R=4.0)
    dirs = rng.normal(size=(400, 4))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    radii = np.exp(rng.uniform(math.log(1.0005), math.log(3.0), 400))
    pts = np.zeros((400, 8))
    pts[:, :4] = dirs * radii[:, None]
    r = oracle_mod.classify(p, pts)
    checked = 0
    for q in range(400):
        rad = np.linalg.norm(pts[q, :4])
        x = math.log(4.0) / math.log(rad)
        if abs(math.log2(x) - round(math.log2(x))) < 1e-6:
            continue   # near-tie: ||z_n|| within rounding of R
        n_star = closed_form_escape_c0(rad, 4.0)
        if n_star > 30:
            assert r["inside"][q] == 1 and r["m"][q] == 30
        else:
            assert r["inside"][q] == 0 and r["m"][q] == n_star, (rad, n_star, r["m"][q])
        checked += 1
    assert checked > 350


def test_inside_set_c0_is_ball(oracle_mod):
    for N in (6, 12, 24):
        rho = 4.0 ** (2.0 ** -N)
        p = P([0.0] * 8, N=N)
        rng = np.random.default_rng(N)
        dirs = rng.normal(size=(200, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        inner = oracle_mod.classify(p, pts8(dirs * rho * (1 - 1e-6)))
        outer = oracle_mod.classify(p, pts8(dirs * rho * (1 + 1e-6)))
        assert inner["inside"].all()
        assert not outer["inside"].any()


def test_escape_is_strict_and_z0_untested(oracle_mod):
    # z0 = 2: z1 = 4, ||z1||^2 = 16 = R^2 exactly -> not escaped; z2 = 16 escapes.
    p1 = P([0.0] * 8, N=1)
    r = oracle_mod.classify(p1, pts8([2.0]))
    assert r["inside"][0] == 1 and r["m"][0] == 1
    p2 = P([0.0] * 8, N=5)
    r = oracle_mod.classify(p2, pts8([2.0]))
    assert r["inside"][0] == 0 and r["m"][0] == 2
    # ||z0||^2 = 25 > R^2 is never tested: with c0 = -25, z1 = 0 and z2 = c escapes at 2.
    p3 = P([-25.0, 0, 0, 0, 0, 0, 0, 0], N=5)
    r = oracle_mod.classify(p3, pts8([5.0]))
    assert r["m"][0] == 2 and r["inside"][0] == 0


def quaternion_escape_eqquatsq(q0, c, N, R2):
    """Independent 4D classifier using Eq. quatsq directly (vectorised numpy)."""
    q = np.array(q0, float).copy()
    m = np.full(q.shape[0], N)
    inside = np.ones(q.shape[0], bool)
    for n in range(1, N + 1):
        x, y, z, w = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
        q = np.stack([x * x - y * y - z * z - w * w + c[0], 2 * x * y + c[1],
                      2 * x * z + c[2], 2 * x * w + c[3]], axis=1)
        esc = inside & ((q * q).sum(1) > R2)
        m[esc] = n
        inside &= ~esc
    return inside, m


def test_zero_dual_reduces_to_quaternion_julia(oracle_mod):
    rng = np.random.default_rng(11)
    n_inside = 0
    for trial in range(5):
        c = list(rng.uniform(-0.6, 0.6, 4)) + [0.0] * 4
        p = P(c, N=15)
        pts = np.zeros((3000, 8))
        pts[:, :4] = rng.uniform(-1.5, 1.5, (3000, 4))
        r = oracle_mod.classify(p, pts)
        ins, m = quaternion_escape_eqquatsq(pts[:, :4], p.c[:4], 15, 16.0)
        agree = (r["m"] == m) & (r["inside"].astype(bool) == ins)
        # the two formulas round differently; a disagreement needs a norm within
        # rounding of R^2 at some step, which is vanishingly rare
        assert agree.mean() >= 0.999
        n_inside += int(r["inside"].sum())
    assert n_inside > 0


def test_complex_plane_reduces_to_complex_julia_bruteforce(oracle_mod):
    c = complex(-0.39054, -0.58679)            # the complex part of Fig. highres's c
    p = P([c.real, c.imag, 0, 0, 0, 0, 0, 0], N=15)
    cr = complex(p.c[0], p.c[1])               # FP32-rounded, as the oracle sees it
    xs = np.linspace(-1.6, 1.6, 64)
    X, Y = np.meshgrid(xs, xs)
    z = (X + 1j * Y).ravel()
    m_ref = np.full(z.shape, 15)
    alive = np.ones(z.shape, bool)
    tie = np.zeros(z.shape, bool)
    zz = z.copy()
    for n in range(1, 16):
        zz = np.where(alive, zz * zz + cr, zz)
        a2 = np.abs(zz) ** 2
        tie |= alive & (np.abs(a2 - 16.0) < 1e-9)
        esc = alive & (a2 > 16.0)
        m_ref[esc] = n
        alive &= ~esc
    pts = np.zeros((z.size, 8))
    pts[:, 0], pts[:, 1] = z.real, z.imag
    r = oracle_mod.classify(p, pts)
    ok = ~tie
    assert ok.sum() > 4000
    np.testing.assert_array_equal(r["m"][ok], m_ref[ok])
    np.testing.assert_array_equal(r["inside"][ok].astype(bool), alive[ok])
    assert alive.any() and (~alive).any()


def test_revolution_symmetry_real_c(oracle_mod):
    # c in span(1): the iteration commutes with rotations of the (i, j, k) space.
    c0 = -0.7
    p = P([c0, 0, 0, 0, 0.0, 0, 0, 0], N=12)
    rng = np.random.default_rng(12)
    xyz = rng.uniform(-1.5, 1.5, (2000, 3))
    rot = np.zeros_like(xyz)
    rot[:, 0] = xyz[:, 0]
    rot[:, 1] = np.hypot(xyz[:, 1], xyz[:, 2])
    a = oracle_mod.classify(p, pts8(xyz))
    b = oracle_mod.classify(p, pts8(rot))
    near = np.abs(a["norm2"] - 16.0) < 1e-6
    agree = (a["m"] == b["m"]) | near
    assert agree.mean() >= 0.999


def test_mirror_symmetry_bitwise(oracle_mod):
    # c and the slice in span(1, i) for both parts: negating the j slot of zeta_0 maps
    # every iterate to its mirror image exactly (only signs change), so escape indices
    # and final norms agree bit for bit.
    c = [0.2, -0.55, 0, 0, 0.3, 0.25, 0, 0]
    p = P(c, N=14)
    rng = np.random.default_rng(13)
    xyz = rng.uniform(-1.5, 1.5, (3000, 3))
    mir = xyz * np.array([1, 1, -1])
    a = oracle_mod.classify(p, pts8(xyz))
    b = oracle_mod.classify(p, pts8(mir))
    np.testing.assert_array_equal(a["m"], b["m"])
    np.testing.assert_array_equal(a["norm2"], b["norm2"])


def test_dual_part_is_derivative_along_cd(oracle_mod):
    """Dual numbers are forward-mode AD: with b_0 = 0, b_n = d a_n / d c_r along c_d."""
    rng = np.random.default_rng(14)
    checked = 0
    for _ in range(60):
        cr = rng.uniform(-0.3, 0.3, 4)
        cd = rng.normal(size=4)
        a0 = rng.uniform(-0.5, 0.5, 4)
        n = 8
        z = oracle_mod.orbit(np.concatenate([a0, np.zeros(4)]), np.concatenate([cr, cd]), n)
        if not np.all(np.isfinite(z)) or np.linalg.norm(z[:4]) > 2:
            continue
        h = 1e-6
        ap = oracle_mod.orbit(np.concatenate([a0, np.zeros(4)]), np.concatenate([cr + h * cd, np.zeros(4)]), n)
        am = oracle_mod.orbit(np.concatenate([a0, np.zeros(4)]), np.concatenate([cr - h * cd, np.zeros(4)]), n)
        fd = (ap[:4] - am[:4]) / (2 * h)
        scale = max(1.0, np.max(np.abs(fd)))
        assert np.max(np.abs(z[4:] - fd)) <= 1e-6 * scale, (z[4:], fd)
        checked += 1
    assert checked >= 20


def test_realpart_norm_mask_independent_of_cd(oracle_mod):
    rng = np.random.default_rng(15)
    cr = list(rng.uniform(-0.5, 0.5, 4))
    pts = np.zeros((3000, 8))
    pts[:, :3] = rng.uniform(-1.5, 1.5, (3000, 3))
    base = oracle_mod.classify(P(cr + [0.0] * 4, norm=workloads.NORM_REALPART), pts)
    for _ in range(3):
        cd = list(rng.uniform(-0.5, 0.5, 4))
        r = oracle_mod.classify(P(cr + cd, norm=workloads.NORM_REALPART), pts)
        np.testing.assert_array_equal(r["m"], base["m"])
        np.testing.assert_array_equal(r["inside"], base["inside"])
    # under the 8-component norm the dual part does change the set
    e8 = oracle_mod.classify(P(cr + [0.45, -0.4, 0.3, 0.2]), pts)
    assert (e8["inside"] != base["inside"]).any()
