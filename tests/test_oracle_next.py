"""Pins of the oracle's extensions: the printed component-wise square, dense grid
classification, the bounding sphere, the specular term and the four-neighbour normal.

* Component-wise square a^2 + b^2 e (printed with Eq. dqjulia2): checked against an
  independent iteration that squares each quaternion with the closed form of Eq. quatsq,
  (s, v)^2 = (s^2 - |v|^2, 2 s v), instead of the oracle's Hamilton product.
* Grid: voxel centres and the (k ny + j) nx + i layout against point classification;
  c = 0 gives the ball of radius R^(2^-N) and the closed-form escape index.
* Bounding sphere (section "Ray-Marching"): a sphere inside the c = 0 ball makes every
  ray that meets it hit at the sphere's entry point (the textbook ray/sphere root); a
  sphere around the ball leaves the hits on the ball, and rays missing it are misses.
* Specular (Eq. phong): on the c = 0 ball with only the specular term the brightest hit
  faces the half vector of the light and view directions (the mirror condition r = v).
* Four-neighbour normal (paragraph "Lighting/Illumination"): on the c = 0 ball it is
  radial to within the sampling error, faces the eye, and the pixel-list and full-frame
  forms agree; no update is spent on it.
"""
import math

import numpy as np
import pytest

import workloads
from test_oracle_render import analytic_ball, frame


def quat_sq_closed_form(q):
    s, v = q[..., :1], q[..., 1:]
    return np.concatenate([s * s - np.sum(v * v, axis=-1, keepdims=True), 2.0 * s * v], axis=-1)


def componentwise_escape(z0, c, N, R2):
    """Escape index (0 = inside) of a <- a^2 + c_r, b <- b^2 + c_d, 8-square norm."""
    a, b = z0[:, :4].copy(), z0[:, 4:].copy()
    m = np.zeros(len(z0), np.int32)
    live = np.ones(len(z0), bool)
    for n in range(1, N + 1):
        a = quat_sq_closed_form(a) + c[:4]
        b = quat_sq_closed_form(b) + c[4:]
        esc = live & (np.sum(a * a, axis=1) + np.sum(b * b, axis=1) > R2)
        m[esc] = n
        live &= ~esc
    return m


def test_componentwise_square_against_quatsq_iteration(oracle_mod):
    rng = np.random.default_rng(11)
    for trial in range(4):
        c = np.concatenate([rng.uniform(-0.6, 0.6, 4), rng.uniform(-0.5, 0.5, 4)])
        p = frame(c=list(c), N=20, algebra=workloads.ALGEBRA_COMPONENTWISE)
        pts = np.zeros((3000, 8))
        pts[:, :3] = rng.uniform(-1.5, 1.5, (3000, 3))
        if trial % 2:   # a slice through the dual part as well
            pts[:, 4:7] = rng.uniform(-0.3, 0.3, (3000, 3))
        ref = componentwise_escape(pts, np.asarray(p.c), p.max_iter, p.escape_radius ** 2)
        got = oracle_mod.classify(p, pts)
        m = np.where(got["inside"] == 1, 0, got["m"])
        # rounding differs between the two formulations: allow a few chaotic boundary points
        assert np.mean(m == ref) > 0.995, np.mean(m == ref)
        assert np.mean(m != ref) * 3000 < 15


def test_componentwise_dual_orbit_ignores_the_point(oracle_mod):
    """With b_0 = 0 on every point, b_n is the orbit of 0 under b <- b^2 + c_d for all
    points: the final dual parts of points that stay inside coincide."""
    rng = np.random.default_rng(12)
    c = [0.1, -0.2, 0.05, 0.0, 0.2, 0.1, -0.15, 0.05]
    p = frame(c=c, N=10, algebra=workloads.ALGEBRA_COMPONENTWISE)
    pts = np.zeros((400, 8))
    pts[:, :3] = rng.uniform(-0.4, 0.4, (400, 3))
    got = oracle_mod.classify(p, pts)
    ins = got["inside"] == 1
    assert ins.sum() > 50
    bd = got["zfinal"][ins, 4:]
    assert np.max(np.abs(bd - bd[0])) == 0.0


def grid_centres(p, nx, ny, nz):
    lo, hi = np.asarray(p.box_min, float), np.asarray(p.box_max, float)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = lo[0] + (i + 0.5) * (hi[0] - lo[0]) / nx
    y = lo[1] + (j + 0.5) * (hi[1] - lo[1]) / ny
    z = lo[2] + (k + 0.5) * (hi[2] - lo[2]) / nz
    return np.stack([x, y, z], axis=-1)


def test_grid_layout_and_centres(oracle_mod):
    p = workloads.plain_128()[0].replace(box_min=[-1.5, -1.2, -0.9], box_max=[1.5, 1.0, 1.3])
    nx, ny, nz = 7, 5, 4
    g = oracle_mod.classify_grid(p, nx, ny, nz)
    pts = np.zeros((nz, ny, nx, 8))
    pts[..., :3] = grid_centres(p, nx, ny, nz)
    r = oracle_mod.classify(p, pts.reshape(-1, 8))
    np.testing.assert_array_equal(g["inside"].reshape(-1), r["inside"])
    np.testing.assert_array_equal(g["m"].reshape(-1), np.where(r["inside"] == 1, 0, r["m"]))
    assert g["total_iters"] == int(r["m"].sum())
    sel = np.array([0, 5, 17, 139, nx * ny * nz - 1])
    gs = oracle_mod.classify_grid(p, nx, ny, nz, voxels=sel)
    np.testing.assert_array_equal(gs["inside"], g["inside"].reshape(-1)[sel])


@pytest.mark.parametrize("N", [6, 12])
def test_grid_c0_ball_and_escape_index(oracle_mod, N):
    n = 40
    p = frame(N=N)
    g = oracle_mod.classify_grid(p, n, n, n)
    r = np.linalg.norm(grid_centres(p, n, n, n), axis=-1)
    R = p.escape_radius
    rho = R ** (2.0 ** -N)
    away = np.abs(r - rho) > 1e-9
    np.testing.assert_array_equal(g["inside"][away], (r <= rho)[away])
    out = (r > 1.0) & away & (g["inside"] == 0)
    ns = np.floor(np.log2(math.log(R) / np.log(r[out]))) + 1
    ns = np.maximum(ns, 1)
    tie = np.abs(np.log2(math.log(R) / np.log(r[out])) - np.round(np.log2(math.log(R) / np.log(r[out])))) < 1e-9
    np.testing.assert_array_equal(g["m"][out][~tie], ns[~tie].astype(np.int32))
    assert g["inside"].sum() > 100


def test_sphere_inside_the_ball_gives_its_entry_point(oracle_mod):
    p = frame(W=24, H=24, N=12, cull_radius=0.8)
    r = oracle_mod.render(p)
    hits = 0
    for j in range(p.height):
        for i in range(p.width):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            ts, chord = analytic_ball(np.asarray(o), np.asarray(d), p.cull_radius)
            if ts is None:
                assert not hit and r["mask"][j, i] == 0
                continue
            assert hit and r["mask"][j, i] == 1 and r["first_hit"][j, i] == 0
            assert abs(r["depth"][j, i] - ts) < 1e-12
            hits += 1
    assert hits > 100


def test_sphere_around_the_ball_keeps_the_hits(oracle_mod):
    N, B = 12, 8
    rho = 4.0 ** (2.0 ** -N)
    p0 = frame(W=32, H=32, N=N, S=64, B=B)
    p1 = p0.replace(cull_radius=1.25)
    r0, r1 = oracle_mod.render(p0), oracle_mod.render(p1)
    np.testing.assert_array_equal(r0["mask"], r1["mask"])
    for j in range(p1.height):
        for i in range(p1.width):
            if not r1["mask"][j, i]:
                continue
            hit, o, d, t0, t1 = oracle_mod.ray(p1, i, j)
            ts, chord = analytic_ball(np.asarray(o), np.asarray(d), rho)
            if chord < 1e-2:
                continue
            assert abs(r1["depth"][j, i] - ts) <= (t1 - t0) / p1.march_steps * 2.0 ** -B + 1e-9
    # fewer updates: the sphere discards empty space of the box
    assert r1["total_iters"] < r0["total_iters"]


def test_specular_peak_faces_the_half_vector(oracle_mod):
    W = H = 96
    p = frame(W=W, H=H, N=12, k_ambient=0.0, k_diffuse=0.0, k_specular=1.0, shininess=64.0,
              light_dir=[0.3, 0.8, 0.6])
    r = oracle_mod.render(p)
    assert r["mask"].sum() > 1000
    shade = np.where(r["mask"] == 1, r["shade"], -1.0)
    j, i = np.unravel_index(np.argmax(shade), shade.shape)
    hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
    pt = np.asarray(o) + r["depth"][j, i] * np.asarray(d)
    n = pt / np.linalg.norm(pt)
    l = np.asarray(p.light_dir) / np.linalg.norm(p.light_dir)
    h = l - np.asarray(d)
    h /= np.linalg.norm(h)
    # within a few pixels' worth of surface angle of the mirror direction
    assert math.degrees(math.acos(min(1.0, float(np.dot(n, h))))) < 3.0
    assert r["shade"][j, i] > 0.95
    # with k_s = 0 the shade is the ambient + diffuse one, unchanged
    q = frame(W=24, H=24, N=12)
    np.testing.assert_array_equal(oracle_mod.render(q)["shade"],
                                  oracle_mod.render(q.replace(shininess=3.0))["shade"])


def test_neighbour_normal_on_the_ball(oracle_mod):
    W = H = 64
    N = 12
    p = frame(W=W, H=H, N=N, S=96, B=12, normal_mode=workloads.NORMAL_NEIGHBOUR4)
    r = oracle_mod.render(p)
    r0 = oracle_mod.render(p.replace(normal_mode=workloads.NORMAL_POTENTIAL))
    np.testing.assert_array_equal(r["mask"], r0["mask"])
    np.testing.assert_array_equal(r["depth"], r0["depth"])
    rho = 4.0 ** (2.0 ** -N)
    interior = 0
    radial = []
    for j in range(H):
        for i in range(W):
            if not r["mask"][j, i]:
                assert r["iters"][j, i] == r0["iters"][j, i]
                continue
            # the normal costs no updates in this mode
            assert r["iters"][j, i] < r0["iters"][j, i]
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            n = r["normal"][j, i]
            assert abs(np.linalg.norm(n) - 1.0) < 1e-12
            assert np.dot(n, d) < 0.0
            nb = [(i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)]
            if all(0 <= a < W and 0 <= b < H and r["mask"][b, a] for a, b in nb):
                # the same construction from the analytic hit points of the five pixels
                P = []
                for a, b in [(i, j)] + nb:
                    _, oo, dd, _, _ = oracle_mod.ray(p, a, b)
                    ts, _ = analytic_ball(np.asarray(oo), np.asarray(dd), rho)
                    P.append(np.asarray(oo) + ts * np.asarray(dd))
                ref = np.cross(P[2] - P[1], P[3] - P[4])
                ref /= np.linalg.norm(ref)
                if np.dot(ref, d) > 0:
                    ref = -ref
                assert math.acos(min(1.0, float(np.dot(n, ref)))) < 2e-3, (i, j)
                pt = P[0]
                radial.append(math.acos(min(1.0, float(np.dot(n, pt / np.linalg.norm(pt))))))
                interior += 1
    assert interior > 500
    # radial up to the sampling error of chords across two pixels
    assert np.mean(radial) < 0.02 and np.max(radial) < 0.15
    pix = np.array([5 * W + 30, 32 * W + 32, 40 * W + 10, 63 * W + 63])
    rs = oracle_mod.render(p, pixels=pix)
    np.testing.assert_array_equal(rs["normal"], r["normal"].reshape(-1, 3)[pix])
    np.testing.assert_array_equal(rs["shade"], r["shade"].reshape(-1)[pix])


# ---- projection ("shadow") rendering: paragraph "Dimension Reduction", approach (2)

def test_projection_with_the_zero_fibre_is_the_slice(oracle_mod):
    p = workloads.plain_128(1)[0].replace(width=48, height=40)
    a = oracle_mod.render(p)
    b = oracle_mod.render(p.replace(fiber=np.zeros((1, 8))))
    for k in ("mask", "depth", "shade", "normal", "first_hit", "iters"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_projection_grows_the_set_and_moves_hits_forward(oracle_mod):
    p = workloads.plain_128(2)[0].replace(width=48, height=48)
    a = oracle_mod.render(p)
    fib = workloads.fiber_ball(6, 0.5, 7)
    b = oracle_mod.render(p.replace(fiber=fib))
    assert np.all(b["mask"] >= a["mask"]) and b["mask"].sum() > a["mask"].sum()
    both = (a["mask"] == 1) & (b["mask"] == 1)
    assert np.all(b["first_hit"][both] <= a["first_hit"][both])
    # the order of the fibre points does not change the image
    c = oracle_mod.render(p.replace(fiber=fib[::-1].copy()))
    for k in ("mask", "depth", "first_hit"):
        np.testing.assert_array_equal(b[k], c[k], err_msg=k)


@pytest.mark.parametrize("ws", [(0.3, 0.5, -0.4), (0.62,), (0.0, 0.9)])
def test_projection_c0_shadow_is_a_smaller_ball(oracle_mod, ws):
    """c = 0: a point (x, y, z, w | 0) stays inside for N updates iff x^2 + y^2 + z^2 + w^2
    <= rho^2 with rho = R^(2^-N) (the quaternion norm squares with every update). With
    fibre offsets w e3, the shadow is the ball of radius sqrt(rho^2 - min w^2)."""
    N, S, B = 12, 64, 8
    rho = 4.0 ** (2.0 ** -N)
    fib = np.zeros((len(ws), 8))
    fib[:, 3] = ws
    p = frame(W=32, H=32, N=N, S=S, B=B, fiber=fib)
    wmin = min(abs(w) for w in p.fiber[:, 3])
    rs = math.sqrt(rho * rho - wmin * wmin)
    r = oracle_mod.render(p)
    hits = 0
    for j in range(p.height):
        for i in range(p.width):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            ts, chord = analytic_ball(np.asarray(o), np.asarray(d), rs)
            if ts is None or chord < 2e-2:
                if ts is None:
                    assert r["mask"][j, i] == 0
                continue
            assert r["mask"][j, i] == 1
            assert abs(r["depth"][j, i] - ts) <= (t1 - t0) / S * 2.0 ** -B + 1e-9
            hits += 1
    assert hits > 50
