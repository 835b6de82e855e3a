"""ctypes wrapper of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check the GPU library. The GPU library never imports
it and it imports nothing from the GPU library; the two share only the seeded
input records of ``workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

from . import build as _build

_lib = None


class _Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("c", C.c_double * 8),
        ("slice_origin", C.c_double * 8),
        ("slice_axes", (C.c_double * 8) * 3),
        ("box_min", C.c_double * 3),
        ("box_max", C.c_double * 3),
        ("eye", C.c_double * 3),
        ("target", C.c_double * 3),
        ("up", C.c_double * 3),
        ("fov_y_deg", C.c_double),
        ("width", C.c_int32),
        ("height", C.c_int32),
        ("max_iter", C.c_int32),
        ("march_steps", C.c_int32),
        ("bisect_steps", C.c_int32),
        ("escape_radius", C.c_double),
        ("norm", C.c_int32),
        ("precision", C.c_int32),
        ("fp64_window", C.c_int32),
        ("normal_h", C.c_double),
        ("light_dir", C.c_double * 3),
        ("k_ambient", C.c_double),
        ("k_diffuse", C.c_double),
        ("march", C.c_int32),
        ("de_hit_eps", C.c_double),
        ("de_min_step", C.c_double),
        ("de_max_step", C.c_double),
        ("algebra", C.c_int32),
        ("normal_mode", C.c_int32),
        ("k_specular", C.c_double),
        ("shininess", C.c_double),
        ("cull_radius", C.c_double),
        ("fiber_count", C.c_int32),
        ("fiber_reserved", C.c_int32),
        ("fiber", C.POINTER(C.c_double)),
    ]


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        D = C.POINTER(C.c_double)
        P = C.POINTER(_Params)
        L.dqjo_quat_mul.argtypes = [D, D, D]
        L.dqjo_quat_square_eq.argtypes = [D, D]
        L.dqjo_dq_add.argtypes = [D, D, D]
        L.dqjo_dq_mul.argtypes = [D, D, D]
        L.dqjo_dq_square.argtypes = [D, D]
        L.dqjo_orbit.argtypes = [D, D, C.c_int32, D]
        L.dqjo_classify.argtypes = [P, D, C.POINTER(C.c_int32), D, D]
        L.dqjo_classify.restype = C.c_int32
        L.dqjo_classify_many.argtypes = [P, D, C.c_int64, C.POINTER(C.c_uint8),
                                         C.POINTER(C.c_int32), D, D]
        L.dqjo_distance.argtypes = [P, D, C.POINTER(C.c_int32), D]
        L.dqjo_distance.restype = C.c_int32
        L.dqjo_slice_map.argtypes = [P, D, D]
        L.dqjo_ray.argtypes = [P, C.c_int32, C.c_int32, D, D, D, D]
        L.dqjo_ray.restype = C.c_int32
        L.dqjo_potential.argtypes = [P, D, C.POINTER(C.c_int32)]
        L.dqjo_potential.restype = C.c_double
        L.dqjo_render.argtypes = [P, C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_uint8), D, D,
                                  D, C.POINTER(C.c_int32), C.POINTER(C.c_uint64), C.c_int32]
        L.dqjo_render.restype = C.c_uint64
        L.dqjo_scan_ray.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                    C.POINTER(C.c_uint8)]
        L.dqjo_scan_ray.restype = C.c_int32
        L.dqjo_classify_grid.argtypes = [P, C.c_int32, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_uint8),
                                         C.POINTER(C.c_int32), C.c_int32]
        L.dqjo_classify_grid.restype = C.c_uint64
        L.dqjo_shade_at.argtypes = [P, C.c_int32, C.c_int32, C.c_double, D, D]
        L.dqjo_shade_at.restype = C.c_int32
        L.dqjo_params_size.restype = C.c_uint32
        _lib = L
    return _lib


def make_params(p) -> _Params:
    """Fill the oracle's parameter record from a ``workloads.Params``-like object."""
    s = _Params()
    s.struct_size = C.sizeof(_Params)
    s.c[:] = [float(x) for x in p.c]
    s.slice_origin[:] = [float(x) for x in p.slice_origin]
    for a in range(3):
        s.slice_axes[a][:] = [float(x) for x in p.slice_axes[a]]
    s.box_min[:] = list(p.box_min)
    s.box_max[:] = list(p.box_max)
    s.eye[:] = list(p.eye)
    s.target[:] = list(p.target)
    s.up[:] = list(p.up)
    s.fov_y_deg = p.fov_y_deg
    s.width, s.height = p.width, p.height
    s.max_iter, s.march_steps, s.bisect_steps = p.max_iter, p.march_steps, p.bisect_steps
    s.escape_radius = p.escape_radius
    s.norm, s.precision, s.fp64_window = p.norm, p.precision, p.fp64_window
    s.normal_h = p.normal_h
    s.light_dir[:] = list(p.light_dir)
    s.k_ambient, s.k_diffuse = p.k_ambient, p.k_diffuse
    s.march = getattr(p, "march", 0)
    s.de_hit_eps = getattr(p, "de_hit_eps", 1e-4)
    s.de_min_step = getattr(p, "de_min_step", 1e-4)
    s.de_max_step = getattr(p, "de_max_step", 0.25)
    s.algebra = getattr(p, "algebra", 0)
    s.normal_mode = getattr(p, "normal_mode", 0)
    s.k_specular = getattr(p, "k_specular", 0.0)
    s.shininess = getattr(p, "shininess", 16.0)
    s.cull_radius = getattr(p, "cull_radius", 0.0)
    fib = getattr(p, "fiber", None)
    if fib is not None and len(fib):
        # the array must be C-contiguous float64 and outlive the call (the Params
        # object holds it)
        assert isinstance(fib, np.ndarray) and fib.dtype == np.float64 and fib.flags.c_contiguous
        s.fiber_count = int(fib.shape[0])
        s.fiber = fib.ctypes.data_as(C.POINTER(C.c_double))
    return s


# ---- algebra -------------------------------------------------------------

def _vec(x, n):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))
    return a


def quat_mul(a, b) -> np.ndarray:
    out = np.zeros(4)
    lib().dqjo_quat_mul(_dptr(_vec(a, 4)), _dptr(_vec(b, 4)), _dptr(out))
    return out


def quat_square_eq(q) -> np.ndarray:
    out = np.zeros(4)
    lib().dqjo_quat_square_eq(_dptr(_vec(q, 4)), _dptr(out))
    return out


def dq_add(x, y) -> np.ndarray:
    out = np.zeros(8)
    lib().dqjo_dq_add(_dptr(_vec(x, 8)), _dptr(_vec(y, 8)), _dptr(out))
    return out


def dq_mul(x, y) -> np.ndarray:
    out = np.zeros(8)
    lib().dqjo_dq_mul(_dptr(_vec(x, 8)), _dptr(_vec(y, 8)), _dptr(out))
    return out


def dq_square(z) -> np.ndarray:
    out = np.zeros(8)
    lib().dqjo_dq_square(_dptr(_vec(z, 8)), _dptr(out))
    return out


def orbit(z0, c, n: int) -> np.ndarray:
    out = np.zeros(8)
    lib().dqjo_orbit(_dptr(_vec(z0, 8)), _dptr(_vec(c, 8)), int(n), _dptr(out))
    return out


# ---- iteration, camera, render ---------------------------------------------

def classify(p, points) -> Dict[str, np.ndarray]:
    """Classify points of R^8 (shape (n, 8)): inside, m, norm2, zfinal."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 8))
    n = pts.shape[0]
    inside = np.zeros(n, np.uint8)
    m = np.zeros(n, np.int32)
    n2 = np.zeros(n)
    zf = np.zeros((n, 8))
    sp = make_params(p)
    lib().dqjo_classify_many(C.byref(sp), _dptr(pts), n,
                             inside.ctypes.data_as(C.POINTER(C.c_uint8)),
                             m.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(n2), _dptr(zf))
    return {"inside": inside, "m": m, "norm2": n2, "zfinal": zf}


def distance(p, points) -> Dict[str, np.ndarray]:
    """Distance estimate of points of R^8 (shape (n, 8)): inside, m, de (0 when inside)."""
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 8))
    n = pts.shape[0]
    inside = np.zeros(n, np.uint8)
    m = np.zeros(n, np.int32)
    de = np.zeros(n)
    sp = make_params(p)
    for q in range(n):
        mi = C.c_int32()
        d = np.zeros(1)
        inside[q] = lib().dqjo_distance(C.byref(sp), _dptr(pts[q]), C.byref(mi), _dptr(d))
        m[q] = mi.value
        de[q] = d[0]
    return {"inside": inside, "m": m, "de": de}


def slice_map(p, x) -> np.ndarray:
    out = np.zeros(8)
    sp = make_params(p)
    lib().dqjo_slice_map(C.byref(sp), _dptr(_vec(x, 3)), _dptr(out))
    return out


def ray(p, i: int, j: int):
    """(hit_box, o, d, t0, t1) for pixel column i, row j."""
    o = np.zeros(3)
    d = np.zeros(3)
    t0 = C.c_double(0.0)
    t1 = C.c_double(0.0)
    sp = make_params(p)
    hit = lib().dqjo_ray(C.byref(sp), int(i), int(j), _dptr(o), _dptr(d), C.byref(t0), C.byref(t1))
    return bool(hit), o, d, t0.value, t1.value


def potential(p, x):
    m = C.c_int32(0)
    sp = make_params(p)
    v = lib().dqjo_potential(C.byref(sp), _dptr(_vec(x, 3)), C.byref(m))
    return v, m.value


def shade_at(p, i: int, j: int, t: float):
    """(normal, shade) at depth t on pixel (i, j)'s ray, as a render's hit would get them."""
    n = np.zeros(3)
    sh = C.c_double(0.0)
    sp = make_params(p)
    if not lib().dqjo_shade_at(C.byref(sp), int(i), int(j), float(t), _dptr(n), C.byref(sh)):
        raise ValueError("the ray misses the box")
    return n, sh.value


def render(p, pixels: Optional[Sequence[int]] = None, nthreads: int = 0) -> Dict[str, np.ndarray]:
    """Render all pixels (image-shaped outputs) or a list of pixel indices (flat outputs)."""
    sp = make_params(p)
    if pixels is None:
        npix = p.width * p.height
        pix_ptr = None
        shape = (p.height, p.width)
    else:
        pix = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64))
        npix = pix.shape[0]
        pix_ptr = pix.ctypes.data_as(C.POINTER(C.c_int64))
        shape = (npix,)
    mask = np.zeros(npix, np.uint8)
    depth = np.zeros(npix)
    shade = np.zeros(npix)
    normal = np.zeros((npix, 3))
    first_hit = np.zeros(npix, np.int32)
    iters = np.zeros(npix, np.uint64)
    total = lib().dqjo_render(C.byref(sp), pix_ptr, npix,
                              mask.ctypes.data_as(C.POINTER(C.c_uint8)), _dptr(depth),
                              _dptr(shade), _dptr(normal),
                              first_hit.ctypes.data_as(C.POINTER(C.c_int32)),
                              iters.ctypes.data_as(C.POINTER(C.c_uint64)), int(nthreads))
    return {"mask": mask.reshape(shape), "depth": depth.reshape(shape),
            "shade": shade.reshape(shape), "normal": normal.reshape(shape + (3,)),
            "first_hit": first_hit.reshape(shape), "iters": iters.reshape(shape),
            "total_iters": int(total)}


def classify_grid(p, nx: int, ny: int, nz: int, voxels: Optional[Sequence[int]] = None,
                  nthreads: int = 0) -> Dict[str, np.ndarray]:
    """Classify the voxel centres of the box (all of them, shape (nz, ny, nx), or the
    listed linear voxel indices (k*ny + j)*nx + i, flat): inside, escape index m (0 when
    inside) and the total update count."""
    sp = make_params(p)
    if voxels is None:
        n = nx * ny * nz
        vptr = None
        shape = (nz, ny, nx)
    else:
        vox = np.ascontiguousarray(np.asarray(voxels, dtype=np.int64))
        n = vox.shape[0]
        vptr = vox.ctypes.data_as(C.POINTER(C.c_int64))
        shape = (n,)
    inside = np.zeros(n, np.uint8)
    m = np.zeros(n, np.int32)
    total = lib().dqjo_classify_grid(C.byref(sp), int(nx), int(ny), int(nz), vptr, n,
                                     inside.ctypes.data_as(C.POINTER(C.c_uint8)),
                                     m.ctypes.data_as(C.POINTER(C.c_int32)), int(nthreads))
    return {"inside": inside.reshape(shape), "m": m.reshape(shape), "total_iters": int(total)}


def scan_ray(p, i: int, j: int, ta: float, tb: float, n: int = 64):
    """Classes of n evenly spaced samples on [ta, tb] of pixel (i, j)'s ray; (classes, changes)."""
    cls = np.zeros(n, np.uint8)
    sp = make_params(p)
    ch = lib().dqjo_scan_ray(C.byref(sp), int(i), int(j), float(ta), float(tb), int(n),
                             cls.ctypes.data_as(C.POINTER(C.c_uint8)))
    return cls, int(ch)


def params_size() -> int:
    return int(lib().dqjo_params_size())
