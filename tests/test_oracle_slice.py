"""Pins of the oracle's general slice map and of the projection's fibre minimum
(paragraph "Dimension Reduction"), each against closed forms that do not use the
oracle's own formulas.

* General slice: with c = 0 a point z0 of the real quaternion part stays inside for N
  updates iff |z0| <= rho = R^(2^-N) (the quaternion norm squares with every update). A
  world point x maps to z0 = O + A x (A = [U V W], 8 x 3), so the set is the quadric
  |O + A x|^2 <= rho^2, met by the ray o + t d where |u + t v|^2 = rho^2 with u = O + A o,
  v = A d. The escape potential is 2 ln|O + A x| exactly, so the normal is A^T (O + A x)
  normalised. The origin, axes and slots are chosen so that swapping two axes, dropping
  the origin or reordering the axes moves the quadric's centre by 0.16 or more.
* Fibre minimum: with fibre offsets w_f along the scalar slot (identity slice), the
  shadow is the union of the balls of radius rho centred at X = -w_f. The union's hit is
  the nearest ball entry, and its normal is radial about the centre of the ball entered
  first: the least potential over the fibre picks that ball (the greatest would pick the
  farthest centre)."""
import math

import numpy as np
import pytest

from test_oracle_render import analytic_ball, frame

N, S, B = 12, 96, 10
RHO = 4.0 ** (2.0 ** -N)


def slice_frame(**kw):
    # slot 0 <- 0.3 + 1.25 Z, slot 1 <- X, slot 2 <- -0.2 + 0.8 Y, slot 3 <- 0.6 Y
    O = [0.3, 0.0, -0.2, 0.0, 0.0, 0.0, 0.0, 0.0]
    U = [0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    V = [0.0, 0.0, 0.8, 0.6, 0.0, 0.0, 0.0, 0.0]
    W = [1.25, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]
    return frame(W=40, H=40, N=N, S=S, B=B, slice_origin=O, slice_axes=[U, V, W], **kw)


def quadric_hit(O, A, o, d, rho):
    u = O + A @ o
    v = A @ d
    a, b, c = v @ v, 2.0 * (u @ v), u @ u - rho * rho
    disc = b * b - 4.0 * a * c
    if disc < 0:
        return None, 0.0
    s = math.sqrt(disc)
    return (-b - s) / (2.0 * a), s / a      # entry parameter, chord length along the ray


def test_general_slice_map_is_affine(oracle_mod):
    p = slice_frame()
    O = np.asarray(p.slice_origin, float)
    A = np.asarray(p.slice_axes, float).T
    rng = np.random.default_rng(3)
    for x in rng.uniform(-1.5, 1.5, (20, 3)):
        np.testing.assert_allclose(oracle_mod.slice_map(p, x), O + A @ x, rtol=0, atol=1e-15)


def test_general_slice_c0_quadric_depth_and_normal(oracle_mod):
    p = slice_frame()
    O = np.asarray(p.slice_origin, float)
    A = np.asarray(p.slice_axes, float).T
    r = oracle_mod.render(p)
    hits = 0
    for j in range(p.height):
        for i in range(p.width):
            _, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            dt = (t1 - t0) / S
            ts, chord = quadric_hit(O, A, np.asarray(o), np.asarray(d), RHO)
            if ts is None:
                assert r["mask"][j, i] == 0, (i, j)
                continue
            if chord < 2.0 * dt:   # grazing: the march may step over it
                continue
            assert r["mask"][j, i] == 1, (i, j)
            assert abs(r["depth"][j, i] - ts) <= dt * 2.0 ** -B + 1e-9, (i, j)
            x = np.asarray(o) + r["depth"][j, i] * np.asarray(d)
            g = A.T @ (O + A @ x)
            g /= np.linalg.norm(g)
            n = r["normal"][j, i]
            assert math.acos(min(1.0, float(n @ g))) < 1e-4, (i, j)
            hits += 1
    assert hits > 300


def test_general_slice_centre_is_not_the_origin(oracle_mod):
    """The quadric's centre, -(A^T A)^-1 A^T O, sits at (0, 0.16, -0.24): the render's
    hits lie around it, not around the world origin."""
    p = slice_frame()
    O = np.asarray(p.slice_origin, float)
    A = np.asarray(p.slice_axes, float).T
    centre = -np.linalg.solve(A.T @ A, A.T @ O)
    np.testing.assert_allclose(centre, [0.0, 0.16, -0.24], atol=1e-6)
    r = oracle_mod.render(p)
    pts = []
    for j in range(0, p.height, 3):
        for i in range(0, p.width, 3):
            if r["mask"][j, i]:
                _, o, d, _, _ = oracle_mod.ray(p, i, j)
                pts.append(np.asarray(o) + r["depth"][j, i] * np.asarray(d))
    pts = np.asarray(pts)
    assert len(pts) > 20
    # every hit lies on the quadric: |O + A x| = rho up to the bisection error
    res = np.abs(np.linalg.norm(pts @ A.T + O, axis=1) - RHO)
    assert res.max() < 1e-3


@pytest.mark.parametrize("ws", [(0.45, -0.45), (-0.45, 0.25, 0.4)])   # balls inside the box
def test_fibre_union_of_shifted_balls(oracle_mod, ws):
    fib = np.zeros((len(ws), 8))
    fib[:, 0] = ws
    p = frame(W=40, H=40, N=N, S=S, B=B, fiber=fib)
    centres = [np.array([-w, 0.0, 0.0]) for w in p.fiber[:, 0]]
    r = oracle_mod.render(p)
    hits = 0
    for j in range(p.height):
        for i in range(p.width):
            _, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            o, d = np.asarray(o), np.asarray(d)
            dt = (t1 - t0) / S
            entries = []
            for cf in centres:
                ts, chord = analytic_ball(o - cf, d, RHO)
                if ts is not None:
                    entries.append((ts, chord, cf))
            if not entries:
                assert r["mask"][j, i] == 0, (i, j)
                continue
            ts, chord, cf = min(entries, key=lambda e: e[0])
            if chord < 2.0 * dt or any(abs(e[0] - ts) < 4.0 * dt for e in entries if e[2] is not cf):
                continue   # grazing, or two balls entered within a few steps
            assert r["mask"][j, i] == 1, (i, j)
            assert abs(r["depth"][j, i] - ts) <= dt * 2.0 ** -B + 1e-9, (i, j)
            x = o + r["depth"][j, i] * d
            g = (x - cf) / np.linalg.norm(x - cf)
            n = r["normal"][j, i]
            assert math.acos(min(1.0, float(n @ g))) < 1e-4, (i, j)
            hits += 1
    assert hits > 300


def test_fibre_potential_is_the_least_over_the_fibre(oracle_mod):
    """c = 0: the potential of fibre point f is 2 ln|x + w_f e0| (no cancellation), so the
    fibre's potential is 2 ln of the distance to the nearest centre."""
    fib = np.zeros((3, 8))
    fib[:, 0] = [0.6, -0.6, 0.1]
    p = frame(W=8, H=8, N=N, S=S, B=B, fiber=fib)
    rng = np.random.default_rng(5)
    tried = 0
    for x in rng.uniform(-1.4, 1.4, (400, 3)):
        ds = [np.linalg.norm(x + np.array([w, 0.0, 0.0])) for w in p.fiber[:, 0]]
        if min(ds) < 0.995:
            continue   # deep inside: |z_N|^2 falls below the potential's 1e-30 floor
        tried += 1
        want = 2.0 * math.log(min(ds))
        got, _ = oracle_mod.potential(p, x)
        assert abs(got - want) < 1e-9 * max(1.0, abs(want)), (x, got, want)
    assert tried > 100
