"""Pins of the oracle's distance-estimate march (section "Ray-Marching", Eq. distfract,
Eq. distfract2), independent of its own code.

* c = 0, zero dual part: z_n = z_0^(2^n), so |z_n| = |p|^(2^n) and, from
  |z'_{n+1}| = 2 |z_n| |z'_n| with |z'_0| = 1, |z'_n| = 2^n |p|^(2^n - 1). The estimate
  0.5 |z_m| ln|z_m| / |z'_m| is therefore 0.5 |p| ln|p| whatever the escape index m.
* c = 0 render, N = 12: the inside set is the ball of radius rho = R^(2^-N) = 1.000338.
  Near its surface the estimate 0.5 |p| ln|p| ~ (|p| - 1)/2 stays above the hit threshold
  (1e-4) until |p| < 1.0002 < rho, so every hit comes from a step landing inside the
  ball. Bisection then puts the hit within one step / 2^B of the analytic entry point.
* c = 0 render, N = 24: rho = 1 + 8e-8 lies inside the threshold shell, so the march
  stops at the first point where 0.5 |p| ln|p| < 1e-4. That point satisfies
  1 <= |p| < 1.0002, and the point one step earlier does not.
* A march that never meets the set misses, with the update count of every step.
"""
import math

import numpy as np
import pytest

import workloads
from test_oracle_render import analytic_ball, frame


def de_frame(**kw):
    kw.setdefault("march", workloads.MARCH_DE)
    return frame(**kw)


def test_distance_estimate_c0_closed_form(oracle_mod):
    rng = np.random.default_rng(4)
    for N, norm in [(12, workloads.NORM_EUCLID8), (24, workloads.NORM_EUCLID8),
                    (12, workloads.NORM_REALPART)]:
        p = de_frame(N=N, norm=norm)
        dirs = rng.normal(size=(40, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        r = rng.uniform(1.001, 3.0, size=40)
        pts = np.zeros((40, 8))
        pts[:, :3] = dirs * r[:, None]
        d = oracle_mod.distance(p, pts)
        assert not d["inside"].any()
        np.testing.assert_allclose(d["de"], 0.5 * r * np.log(r), rtol=1e-12)
        # the escape index itself follows |p|^(2^m) > R
        m = np.maximum(1, np.floor(np.log2(np.log(4.0) / np.log(r))) + 1)
        np.testing.assert_array_equal(d["m"], m.astype(np.int32))
    # inside points carry no estimate
    p = de_frame(N=12)
    d = oracle_mod.distance(p, np.zeros((1, 8)))
    assert d["inside"][0] == 1 and d["de"][0] == 0.0


@pytest.mark.parametrize("B", [8, 0])
def test_de_render_c0_bisects_onto_the_ball(oracle_mod, B):
    W = H = 40
    N = 12
    p = de_frame(W=W, H=H, N=N, S=400, B=B)
    rho = 4.0 ** (2.0 ** -N)
    r = oracle_mod.render(p)
    n_hit = 0
    for j in range(H):
        for i in range(W):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            tstar, chord = analytic_ball(o, d, rho)
            if tstar is None:
                assert r["mask"][j, i] == 0
                continue
            if chord < 1e-2:
                continue   # grazing rays may pass between steps
            assert r["mask"][j, i] == 1, (i, j)
            n_hit += 1
            # the bracket is one step, at most max(de, min_step) <= 0.5 (1.0004 - 1) + ...;
            # bisection leaves step / 2^(B+1) (B = 0: the bracket's midpoint)
            assert abs(r["depth"][j, i] - tstar) <= 2.5e-4 * 2.0 ** -B, (i, j)
    assert n_hit > 300


def test_de_render_c0_stops_on_the_threshold_shell(oracle_mod):
    W = H = 32
    p = de_frame(W=W, H=H, N=24, S=400, B=8)
    eps = p.de_hit_eps
    r = oracle_mod.render(p)
    n_hit = 0
    for j in range(H):
        for i in range(W):
            hit, o, d, t0, t1 = oracle_mod.ray(p, i, j)
            tstar, chord = analytic_ball(o, d, 1.0)
            if tstar is None or chord < 2e-2:
                continue
            assert r["mask"][j, i] == 1, (i, j)
            n_hit += 1
            ph = o + r["depth"][j, i] * d
            rad = float(np.linalg.norm(ph))
            assert 0.5 * rad * math.log(rad) < eps + 1e-12
            assert 1.0 - 1e-7 <= rad < 1.0 + 2.01 * eps
    assert n_hit > 200


def test_de_render_miss_counts_every_step(oracle_mod):
    # c = 0, the camera looking away from the ball: every point escapes on update 1 at
    # |p| > 2 (p in the far corner region); the march steps to the box exit
    p = de_frame(W=4, H=4, N=12, S=400, B=8, eye=[1.4, 1.4, 1.4], target=[3.0, 3.0, 3.0],
                 fov_y_deg=5.0)
    r = oracle_mod.render(p)
    assert r["mask"].sum() == 0
    assert r["total_iters"] > 0
