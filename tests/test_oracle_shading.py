"""Pin of the oracle's normal and shade for c != 0 (section "Lighting/Illumination",
Eq. phong), where no closed form exists.

The traced surface fixes its own normal. Zoomed in until neighbouring pixels' hits lie
about 1e-3 apart, the cross product of the central differences of the four neighbours'
hit points is the surface normal, up to the pixel spacing times the curvature. The hit
points come from the march and bisection, which the dense-scan and c = 0 pins cover.

The render's normal is the central difference of the escape potential ln||z_m||^2 / 2^m.
It follows the surface only where that potential is smooth across it. Where every
stencil point of the five pixels escapes at max_iter or stays inside, the potential
near the hit is the one function ln||z_N||^2 / 2^N. The traced surface is then its level
set ||z_N|| = R, so its gradient is the surface normal. Elsewhere the potential can
jump across the surface. Under the 8-square norm an orbit whose norm nearly reached R
in its dual part can fall back, so the inside neighbour's ||z_N|| is far below R while
the outside one escaped early. A stencil axis that straddles such a jump tilts the
normal; that is the method's normal as defined, and this pin leaves those pixels out.

A swapped or sign-flipped gradient component, a stencil step on the wrong axis, or a
shade formed from another vector than the normal is off by O(1) radians on generic
views, against the 2e-2 allowed here.
"""
import math

import numpy as np

import workloads

ANGLE_TOL = 2e-2    # rad: the cross product's O(spacing x curvature) error, about 1e-2 at worst
SHADE_TOL = 1e-2


def zoomed_views(oracle_mod, seed, N, count, rng):
    """Views 1 degree wide, aimed at hit points of a 64 x 64 render of the seeded frame."""
    base = workloads.plain_128(seed)[0].replace(width=64, height=64, max_iter=N, march_steps=256,
                                                bisect_steps=22)
    r = oracle_mod.render(base, nthreads=8)
    hits = np.argwhere((r["mask"] == 1) & (r["first_hit"] > 0))
    views = []
    for jj, ii in hits[rng.choice(len(hits), min(count, len(hits)), replace=False)]:
        _, o, d, _, _ = oracle_mod.ray(base, int(ii), int(jj))
        target = np.asarray(o) + r["depth"][jj, ii] * np.asarray(d)
        views.append(base.replace(target=[float(v) for v in target], fov_y_deg=1.0, width=24,
                                  height=24))
    return views


def surface_checks(oracle_mod, p):
    """(angle, shade difference) for every pixel of a view where the pin applies."""
    r = oracle_mod.render(p, nthreads=8)
    W, H, N = p.width, p.height, p.max_iter
    light = np.asarray(p.light_dir, dtype=np.float64)
    light /= np.linalg.norm(light)
    X = np.zeros((H, W, 3))
    D = np.zeros((H, W, 3))
    for j in range(H):
        for i in range(W):
            _, o, d, _, _ = oracle_mod.ray(p, i, j)
            X[j, i] = np.asarray(o) + r["depth"][j, i] * np.asarray(d)
            D[j, i] = d
    smooth = {}

    def smooth_at(a, b):
        # every stencil point of the pixel's hit escapes at max_iter or stays inside
        if (a, b) not in smooth:
            smooth[(a, b)] = all(
                oracle_mod.potential(p, X[b, a] + s * p.normal_h * e)[1] == N
                for e in np.eye(3) for s in (1.0, -1.0))
        return smooth[(a, b)]

    out = []
    for j in range(1, H - 1):
        for i in range(1, W - 1):
            five = [(i, j), (i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)]
            # hits in the march (not on the box face), on one smooth sheet
            if not all(r["mask"][b, a] and r["first_hit"][b, a] > 0 for a, b in five):
                continue
            tu = X[j, i + 1] - X[j, i - 1]
            tv = X[j + 1, i] - X[j - 1, i]
            bend_u = np.linalg.norm(X[j, i + 1] - 2 * X[j, i] + X[j, i - 1]) / np.linalg.norm(tu)
            bend_v = np.linalg.norm(X[j + 1, i] - 2 * X[j, i] + X[j - 1, i]) / np.linalg.norm(tv)
            if max(bend_u, bend_v) >= 0.05:
                continue
            if not all(smooth_at(a, b) for a, b in five):
                continue
            nf = np.cross(tu, tv)
            nf /= np.linalg.norm(nf)
            if nf @ D[j, i] > 0:
                nf = -nf
            angle = math.acos(min(1.0, max(-1.0, float(r["normal"][j, i] @ nf))))
            shade = p.k_ambient + p.k_diffuse * max(0.0, float(nf @ light))
            out.append((angle, abs(r["shade"][j, i] - shade)))
    return out


def test_nonzero_c_normal_and_shade_follow_the_traced_surface(oracle_mod):
    rng = np.random.default_rng(11)
    used = 0
    checks = []
    for seed in range(4):
        for N in (8, 12):
            for p in zoomed_views(oracle_mod, seed, N, 3, rng):
                assert any(abs(v) > 0.05 for v in p.c)   # a c far from 0
                got = surface_checks(oracle_mod, p)
                if len(got) >= 100:
                    used += 1
                    checks.extend(got)
    assert used >= 8 and len(checks) >= 2000, (used, len(checks))
    angles = np.array([a for a, _ in checks])
    shades = np.array([s for _, s in checks])
    assert angles.max() < ANGLE_TOL, angles.max()
    assert shades.max() < SHADE_TOL, shades.max()
    # most pixels agree far more closely than the curvature bound
    assert np.median(angles) < 2e-3, np.median(angles)
