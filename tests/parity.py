"""Test-side comparison of GPU frames with the FP64 oracle.

A pixel AGREES if both miss, or both hit with |depth_gpu - depth_oracle| <= 1e-4 E,
E the box diagonal. Every other pixel is a mismatch; at most 0.1 % may mismatch,
and each must lie within one march step of the set's boundary: the FP64 fine scan
(64 points) of [t - dt, t + dt] around the disputed sample t must change class.
The disputed sample is the earlier first-inside sample of the two sides (the one
whose class the two sides disagree on).

On agreeing hits the shade must be within 1/255, except where the oracle's own shade
takes the GPU's value (within 1/255) at some depth between the two hits, widened by 4
FP32 ulps on each side: the normal is the gradient of the escape potential sampled by a
stencil, and that gradient jumps where a stencil point's escape index changes, so two
hits within the depth tolerance can lie on the two sides of a jump. Every exception
must be explained that way, and at least 99 % of agreeing hits must be within 1/255
(the fraction within, the maximum and the 99.9th percentile are returned).
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np

import oracle
import workloads


def to_numpy(out: Dict) -> Dict[str, np.ndarray]:
    r = {}
    for k, v in out.items():
        if hasattr(v, "detach"):
            v = v.detach().cpu().numpy()
        r[k] = v
    return r


def shade_explained(p, pix: int, t_gpu: float, t_ora: float, s_gpu: float, n: int = 65) -> bool:
    """True when the oracle's shade equals s_gpu within 1/255 at some depth of
    [min(t_gpu, t_ora) - 4u, max(t_gpu, t_ora) + 4u], u one FP32 ulp of the depth."""
    i, j = pix % p.width, pix // p.width
    u = float(np.spacing(np.float32(max(t_gpu, t_ora))))
    lo, hi = min(t_gpu, t_ora) - 4.0 * u, max(t_gpu, t_ora) + 4.0 * u
    for t in np.linspace(lo, hi, n):
        _, s = oracle.shade_at(p, i, j, float(t))
        if abs(s - s_gpu) <= 1.0 / 255.0:
            return True
    return False


def compare(p, gpu: Dict[str, np.ndarray], ora: Dict[str, np.ndarray],
            pixels: Optional[np.ndarray] = None, scan: bool = True, max_scan: int = 400,
            gathered: bool = False):
    """Compare GPU outputs (full images; with ``gathered``, flat arrays already taken at
    the listed ``pixels``) with oracle outputs (full images, or flat arrays for the listed
    ``pixels``). Returns a report dict."""
    E = workloads.scene_extent(p)
    tol = 1e-4 * E
    if pixels is None:
        g = {k: np.asarray(v).reshape(-1, *np.asarray(v).shape[2:]) for k, v in gpu.items()
             if k in ("mask", "depth", "shade", "first_hit", "normal")}
        o = {k: np.asarray(ora[k]).reshape(g[k].shape) for k in g}
        idx = np.arange(p.width * p.height)
    else:
        idx = np.asarray(pixels)
        if gathered:
            g = {k: np.asarray(gpu[k]).reshape(idx.size) for k in
                 ("mask", "depth", "shade", "first_hit") if k in gpu}
        else:
            g = {k: np.asarray(gpu[k]).reshape(-1, *np.asarray(gpu[k]).shape[2:])[idx] for k in
                 ("mask", "depth", "shade", "first_hit") if k in gpu}
        o = {k: np.asarray(ora[k]) for k in g}
    gm = g["mask"].astype(bool)
    om = o["mask"].astype(bool)
    both_hit = gm & om
    with np.errstate(invalid="ignore"):   # misses carry +inf depths on both sides
        ddepth = np.where(both_hit, np.abs(g["depth"].astype(np.float64) - o["depth"]), 0.0)
    agree = (~gm & ~om) | (both_hit & (ddepth <= tol))
    mism = np.nonzero(~agree)[0]
    rep = {
        "pixels": int(idx.size),
        "hits_gpu": int(gm.sum()),
        "hits_oracle": int(om.sum()),
        "agree_frac": float(agree.mean()),
        "mismatches": int(mism.size),
        "depth_err_max_E": float(ddepth[both_hit & agree].max() / E) if (both_hit & agree).any() else 0.0,
    }
    sh_ok = both_hit & agree
    rep["shade_exceptions"] = 0
    rep["shade_unexplained"] = []
    if sh_ok.any():
        ds = np.abs(g["shade"].astype(np.float64) - o["shade"])[sh_ok]
        rep["shade_err_max"] = float(ds.max())
        rep["shade_within_frac"] = float((ds <= 1.0 / 255.0).mean())
        rep["shade_err_p999"] = float(np.quantile(ds, 0.999))
        # diagnose every shade exception against the oracle's shade between the two hits
        if getattr(p, "normal_mode", 0) == 0 and getattr(p, "march", 0) == 0 \
                and getattr(p, "fiber", None) is None:
            exc = np.nonzero(sh_ok)[0][ds > 1.0 / 255.0]
            rep["shade_exceptions"] = int(exc.size)
            for q in exc[:max_scan]:
                if not shade_explained(p, int(idx[q]), float(g["depth"][q]), float(o["depth"][q]),
                                       float(g["shade"][q])):
                    rep["shade_unexplained"].append(int(idx[q]))
    else:
        rep["shade_err_max"] = 0.0
        rep["shade_within_frac"] = 1.0
        rep["shade_err_p999"] = 0.0
    # mismatch diagnosis: the disputed sample must sit within one march step of a class change
    far = []
    if scan and getattr(p, "march", workloads.MARCH_FIXED) == workloads.MARCH_DE:
        # Distance-estimate march: the disputed point is the nearer of the two hits; the
        # ray must pass close to the set there (inside, or an FP64 estimate below 10 eps)
        for q in mism[:max_scan]:
            pix = int(idx[q])
            i, j = pix % p.width, pix // p.width
            hit, o3, d3, t0, t1 = oracle.ray(p, i, j)
            ts = [float(t) for t in (g["depth"][q], o["depth"][q]) if np.isfinite(t)]
            if not hit or not ts:
                far.append(pix)
                continue
            x = np.asarray(o3) + min(ts) * np.asarray(d3)
            dd = oracle.distance(p, oracle.slice_map(p, x).reshape(1, 8))
            if not (dd["inside"][0] or dd["de"][0] < 10.0 * p.de_hit_eps):
                far.append(pix)
    elif scan and "first_hit" in g:
        for q in mism[:max_scan]:
            pix = int(idx[q])
            i, j = pix % p.width, pix // p.width
            hit, o3, d3, t0, t1 = oracle.ray(p, i, j)
            if not hit:
                far.append(pix)
                continue
            dt = (t1 - t0) / p.march_steps
            ks = [int(k) for k in (g["first_hit"][q], o["first_hit"][q]) if k >= 0]
            if not ks:
                far.append(pix)
                continue
            kd = min(ks)
            td = t0 + kd * dt
            _, changes = oracle.scan_ray(p, i, j, td - dt, td + dt, 64)
            if changes == 0:
                far.append(pix)
    rep["mismatch_far_from_boundary"] = far
    return rep


def assert_parity(rep, min_agree=0.999, shade_frac=0.999):
    """The bar of the module docstring. shade_frac is the fraction of agreeing hits
    that must shade within 1/255 when exceptions are not diagnosed (distance-estimate
    march, neighbour normal, projection); with the diagnosis every exception must be
    explained and 99 % is the floor."""
    assert rep["agree_frac"] >= min_agree, rep
    assert not rep["mismatch_far_from_boundary"], rep
    assert rep["depth_err_max_E"] <= 1e-4, rep
    assert not rep.get("shade_unexplained"), rep
    if rep.get("shade_exceptions") and rep["shade_within_frac"] < shade_frac:
        assert rep["shade_within_frac"] >= min(shade_frac, 0.99), rep
    else:
        assert rep["shade_within_frac"] >= shade_frac, rep


def sample_pixels(p, n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(p.width * p.height, size=min(n, p.width * p.height), replace=False))
