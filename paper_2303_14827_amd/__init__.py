"""Python binding of libdqj (dual-quaternion Julia ray marching on MI355X / gfx950).

Argument marshalling only: every step of the render runs in the library's HIP
kernels. PyTorch provides device memory and the current HIP stream. The library
is built in-tree (``python -m paper_2303_14827_amd.build``); importing this module
does not load it, the first call does, and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import os
from typing import Dict, List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdqj.so")

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_BUDGET, E_QUEUE_FULL, E_DEVICE = -1, -2, -3, -4, -5
E_TIMEOUT, E_CANCELLED, E_UNSUPPORTED, E_STATE = -6, -7, -8, -9
SERVE_FAIR, SERVE_OLDEST = 0, 1
MARCH_FIXED, MARCH_DE = 0, 1
ALGEBRA_DUAL, ALGEBRA_COMPONENTWISE = 0, 1
NORMAL_POTENTIAL, NORMAL_NEIGHBOUR4 = 0, 1

NORM_EUCLID8, NORM_REALPART = 0, 1
PREC_FP32, PREC_SPLIT, PREC_FP64 = 0, 1, 2
KERNEL_AUTO, KERNEL_REFILL, KERNEL_DIRECT, KERNEL_LOCKSTEP = 0, 1, 2, 3
FLAG_BOX, FLAG_HIT, FLAG_FP64, FLAG_FALLBACK = 1, 2, 4, 8
NOALLOC_MAX_SPLIT_PIXELS = 262144   # DQJ_NOALLOC_MAX_SPLIT_PIXELS


class DQJError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_str(status)}: {msg}")
        self.status = status


class dqj_params(C.Structure):
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


class dqj_frame_out(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("mask", C.c_void_p),
        ("depth", C.c_void_p),
        ("shade", C.c_void_p),
        ("image8", C.c_void_p),
        ("normal", C.c_void_p),
        ("first_hit", C.c_void_p),
        ("flags", C.c_void_p),
        ("iters", C.c_void_p),
    ]


class dqj_schedule(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("kernel", C.c_int32),
        ("tile_w", C.c_int32),
        ("tile_h", C.c_int32),
        ("waves_per_block", C.c_int32),
        ("blocks_per_cu", C.c_int32),
    ]


class dqj_serve_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("hbm_budget_bytes", C.c_uint64),
        ("max_inflight", C.c_int32),
        ("max_pending", C.c_int32),
        ("precision", C.c_int32),
        ("norm", C.c_int32),
        ("slots", C.c_int32),
        ("count_iters", C.c_int32),
        ("epoch_pixels", C.c_int64),
        ("epoch_work", C.c_double),
        ("sched", dqj_schedule),
        ("policy", C.c_int32),
    ]


class dqj_request_result(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("status", C.c_int32),
        ("t_submit", C.c_double),
        ("t_admit", C.c_double),
        ("t_first_launch", C.c_double),
        ("t_done", C.c_double),
        ("chunks", C.c_int32),
    ]


class dqj_serve_stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("submitted", C.c_uint64),
        ("admitted", C.c_uint64),
        ("completed", C.c_uint64),
        ("cancelled", C.c_uint64),
        ("failed", C.c_uint64),
        ("rejected", C.c_uint64),
        ("epochs", C.c_uint64),
        ("pending", C.c_int32),
        ("active", C.c_int32),
        ("resident_bytes", C.c_uint64),
        ("p50_latency_s", C.c_double),
        ("p99_latency_s", C.c_double),
        ("max_latency_s", C.c_double),
        ("mean_latency_s", C.c_double),
    ]


class dqj_device_info(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32),
        ("arch", C.c_char * 64),
        ("compute_units", C.c_int32),
        ("clock_khz", C.c_int32),
        ("memory_clock_khz", C.c_int32),
        ("total_mem_bytes", C.c_uint64),
        ("fp32_vector_peak_tflops", C.c_double),
        ("fp32_unpacked_peak_tflops", C.c_double),
    ]


_lib = None

# symbol -> (restype, argtypes)
_SIGS = {
    "dqj_render": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out), C.c_void_p]),
    "dqj_render_noalloc": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out),
                                       C.c_void_p]),
    "dqj_render_scheduled": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out),
                                         C.POINTER(dqj_schedule), C.c_void_p]),
    "dqj_render_batch": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out), C.c_int32,
                                     C.c_void_p]),
    "dqj_batch_plan_create": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out),
                                          C.c_int32, C.POINTER(dqj_schedule), C.c_void_p,
                                          C.POINTER(C.c_void_p)]),
    "dqj_batch_plan_launch": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "dqj_batch_plan_destroy": (C.c_int32, [C.c_void_p]),
    "dqj_classify_points": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(dqj_params),
                                        C.c_void_p, C.c_void_p, C.c_void_p]),
    "dqj_classify_grid": (C.c_int32, [C.POINTER(dqj_params), C.c_int32, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dqj_device_info_get": (C.c_int32, [C.c_int32, C.POINTER(dqj_device_info)]),
    "dqj_measure_engine_clock": (C.c_int32, [C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "dqj_autotune": (C.c_int32, [C.POINTER(dqj_params), C.POINTER(dqj_frame_out), C.c_int32,
                                 C.c_char_p, C.POINTER(dqj_schedule)]),
    "dqj_serve_create": (C.c_int32, [C.POINTER(dqj_serve_config), C.POINTER(C.c_void_p)]),
    "dqj_serve_submit": (C.c_int32, [C.c_void_p, C.POINTER(dqj_params), C.POINTER(dqj_frame_out),
                                     C.POINTER(C.c_uint64)]),
    "dqj_serve_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(dqj_request_result)]),
    "dqj_serve_wait": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_int32,
                                   C.POINTER(dqj_request_result)]),
    "dqj_serve_cancel": (C.c_int32, [C.c_void_p, C.c_uint64]),
    "dqj_serve_stats_get": (C.c_int32, [C.c_void_p, C.POINTER(dqj_serve_stats)]),
    "dqj_serve_destroy": (C.c_int32, [C.c_void_p]),
    "dqj_last_error": (C.c_char_p, []),
    "dqj_status_str": (C.c_char_p, [C.c_int32]),
}


def lib():
    """Load libdqj.so. Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2303_14827_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    if _lib is None:
        return str(s)
    return _lib.dqj_status_str(int(s)).decode()


def _check(status: int):
    if status != OK:
        raise DQJError(status, lib().dqj_last_error().decode())


def make_params(p) -> dqj_params:
    """Fill a dqj_params from a ``workloads.Params``-like object."""
    s = dqj_params()
    s.struct_size = C.sizeof(dqj_params)
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


def make_schedule(kernel=0, tile_w=0, tile_h=0, waves_per_block=0, blocks_per_cu=0) -> dqj_schedule:
    s = dqj_schedule()
    s.struct_size = C.sizeof(dqj_schedule)
    s.kernel, s.tile_w, s.tile_h = kernel, tile_w, tile_h
    s.waves_per_block, s.blocks_per_cu = waves_per_block, blocks_per_cu
    return s


def alloc_outputs(width: int, height: int, device="cuda", extras: bool = True):
    """Device output tensors for one frame (torch, caller-owned)."""
    import torch
    o = {
        "mask": torch.empty((height, width), dtype=torch.uint8, device=device),
        "depth": torch.empty((height, width), dtype=torch.float32, device=device),
        "shade": torch.empty((height, width), dtype=torch.float32, device=device),
        "iters": torch.zeros((1,), dtype=torch.int64, device=device),
    }
    if extras:
        o["image8"] = torch.empty((height, width), dtype=torch.uint8, device=device)
        o["normal"] = torch.empty((height, width, 3), dtype=torch.float32, device=device)
        o["first_hit"] = torch.empty((height, width), dtype=torch.int32, device=device)
        o["flags"] = torch.empty((height, width), dtype=torch.uint8, device=device)
    return o


# dtype and elements per pixel of each output buffer ("iters" is one counter per frame)
_OUT_SPEC = {"mask": ("uint8", 1), "depth": ("float32", 1), "shade": ("float32", 1),
             "image8": ("uint8", 1), "normal": ("float32", 3), "first_hit": ("int32", 1),
             "flags": ("uint8", 1), "iters": ("int64", 0)}
_REQUIRED_OUT = ("mask", "depth", "shade")


def check_device_tensor(name: str, t, dtype: str, min_numel: int, where: bool = True):
    """Raise ValueError unless t is a contiguous torch tensor of the given dtype on the
    current GPU with at least min_numel elements. The C ABI receives raw device
    pointers, so this is the only place a wrong buffer can be refused before a kernel
    writes through it."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.{dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if t.numel() < min_numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {min_numel} needed")
    if where:
        check_on_current_gpu(name, t)


def check_on_current_gpu(name: str, t):
    import torch
    if t.device.type != "cuda":
        raise ValueError(f"{name}: tensor is on {t.device}, not on the GPU")
    cur = torch.cuda.current_device()
    if t.device.index is not None and t.device.index != cur:
        raise ValueError(f"{name}: tensor is on cuda:{t.device.index}, current device is cuda:{cur}")


def make_frame_out(o: Dict, p=None) -> dqj_frame_out:
    """Marshal an output dict. With the frame's parameters p, every tensor is checked
    (device, dtype, contiguity, size) before its pointer is passed on."""
    f = dqj_frame_out()
    f.struct_size = C.sizeof(dqj_frame_out)
    npix = int(p.width) * int(p.height) if p is not None else 0
    if p is not None:   # format of every buffer first, then where each one lives
        for name in _REQUIRED_OUT:
            if o.get(name) is None:
                raise ValueError(f"output '{name}' is required")
        for name, (dtype, per_px) in _OUT_SPEC.items():
            if o.get(name) is not None:
                check_device_tensor(name, o[name], dtype, per_px * npix if per_px else 1,
                                    where=False)
        for name in _OUT_SPEC:
            if o.get(name) is not None:
                check_on_current_gpu(name, o[name])
    for name in _OUT_SPEC:
        t = o.get(name)
        setattr(f, name, t.data_ptr() if t is not None else None)
    return f


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def render(p, out: Optional[Dict] = None, stream=None, schedule: Optional[dqj_schedule] = None,
           extras: bool = True) -> Dict:
    """Enqueue one frame on the stream; returns the output tensor dict."""
    if out is None:
        out = alloc_outputs(p.width, p.height, extras=extras)
    sp = make_params(p)
    fo = make_frame_out(out, p)
    if schedule is None:
        _check(lib().dqj_render(C.byref(sp), C.byref(fo), _stream(stream)))
    else:
        _check(lib().dqj_render_scheduled(C.byref(sp), C.byref(fo), C.byref(schedule),
                                          _stream(stream)))
    return out


def render_noalloc(p, out: Dict, stream=None) -> Dict:
    """dqj_render_noalloc: one frame into the caller's outputs, with the library's fixed
    per-GPU scratch instead of device memory allocated per stream. Split frames are
    limited to NOALLOC_MAX_SPLIT_PIXELS; calls that overlap on one GPU race."""
    sp = make_params(p)
    fo = make_frame_out(out, p)
    _check(lib().dqj_render_noalloc(C.byref(sp), C.byref(fo), _stream(stream)))
    return out


def render_batch(ps: Sequence, outs: Optional[List[Dict]] = None, stream=None,
                 extras: bool = False) -> List[Dict]:
    """Enqueue n frames as one persistent launch; returns the output dicts."""
    n = len(ps)
    if outs is None:
        outs = [alloc_outputs(p.width, p.height, extras=extras) for p in ps]
    if len(outs) != n:
        raise ValueError(f"{n} frames but {len(outs)} output dicts")
    arr_p = (dqj_params * n)(*[make_params(p) for p in ps])
    arr_o = (dqj_frame_out * n)(*[make_frame_out(o, p) for p, o in zip(ps, outs)])
    _check(lib().dqj_render_batch(arr_p, arr_o, n, _stream(stream)))
    return outs


class BatchPlan:
    """A batch captured into a HIP graph once and replayed with launch()."""

    def __init__(self, ps: Sequence, outs: List[Dict], schedule: Optional[dqj_schedule] = None,
                 stream=None):
        n = len(ps)
        if len(outs) != n:
            raise ValueError(f"{n} frames but {len(outs)} output dicts")
        self.outs = outs
        arr_p = (dqj_params * n)(*[make_params(p) for p in ps])
        arr_o = (dqj_frame_out * n)(*[make_frame_out(o, p) for p, o in zip(ps, outs)])
        h = C.c_void_p()
        _check(lib().dqj_batch_plan_create(arr_p, arr_o, n,
                                           C.byref(schedule) if schedule is not None else None,
                                           _stream(stream), C.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().dqj_batch_plan_launch(self._h, _stream(stream)))

    def close(self):
        if self._h:
            _check(lib().dqj_batch_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ps: Sequence, outs: List[Dict], cache_path: Optional[str] = None) -> dqj_schedule:
    """Pick the fastest schedule for frames like ps (renders them into outs)."""
    n = len(ps)
    if len(outs) != n:
        raise ValueError(f"{n} frames but {len(outs)} output dicts")
    arr_p = (dqj_params * n)(*[make_params(p) for p in ps])
    arr_o = (dqj_frame_out * n)(*[make_frame_out(o, p) for p, o in zip(ps, outs)])
    best = make_schedule()
    _check(lib().dqj_autotune(arr_p, arr_o, n, cache_path.encode() if cache_path else None,
                              C.byref(best)))
    return best


def classify_points(pts, p, precision: int = PREC_FP32, stream=None):
    """Classify device points (n x 8, float32 or float64). Returns (escape_iter, final_norm2)."""
    import torch
    if pts.dim() != 2 or pts.shape[1] != 8:
        raise ValueError(f"points: shape {tuple(pts.shape)}, expected (n, 8)")
    check_device_tensor("points", pts, "float64" if precision == PREC_FP64 else "float32",
                        pts.shape[0] * 8)
    n = pts.shape[0]
    esc = torch.empty((n,), dtype=torch.int32, device=pts.device)
    n2 = torch.empty((n,), dtype=torch.float32, device=pts.device)
    sp = make_params(p)
    _check(lib().dqj_classify_points(C.c_void_p(pts.data_ptr()), n, precision, C.byref(sp),
                                     C.c_void_p(esc.data_ptr()), C.c_void_p(n2.data_ptr()),
                                     _stream(stream)))
    return esc, n2


def classify_grid(p, nx: int, ny: int, nz: int, mask=None, escape=None, iters=None,
                  extras: bool = False, stream=None) -> Dict:
    """Classify the nx x ny x nz voxel centres of p's box (dqj_classify_grid). Outputs
    are device tensors of shape (nz, ny, nx): ``mask`` (u8) and, with ``extras``, the
    escape index (i32) and a one-element update counter (int64, added to)."""
    import torch
    if mask is None:
        mask = torch.empty((nz, ny, nx), dtype=torch.uint8, device="cuda")
    if extras and escape is None:
        escape = torch.empty((nz, ny, nx), dtype=torch.int32, device="cuda")
    if extras and iters is None:
        iters = torch.zeros((1,), dtype=torch.int64, device="cuda")
    nvox = int(nx) * int(ny) * int(nz)
    check_device_tensor("mask", mask, "uint8", nvox)
    if escape is not None:
        check_device_tensor("escape", escape, "int32", nvox)
    if iters is not None:
        check_device_tensor("iters", iters, "int64", 1)
    sp = make_params(p)
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
    _check(lib().dqj_classify_grid(C.byref(sp), nx, ny, nz, ptr(mask), ptr(escape), ptr(iters),
                                   _stream(stream)))
    out = {"mask": mask}
    if escape is not None:
        out["escape"] = escape
    if iters is not None:
        out["iters"] = iters
    return out


def _result_dict(r: dqj_request_result) -> Dict:
    return {"status": r.status, "t_submit": r.t_submit, "t_admit": r.t_admit,
            "t_first_launch": r.t_first_launch, "t_done": r.t_done, "chunks": r.chunks}


class Server:
    """The library's request server (continuous batching over epoch slots).

    submit() takes a Params-like record and a dict of caller-owned device tensors
    (alloc_outputs); the tensors must stay alive until the request is final.
    """

    def __init__(self, precision: int = PREC_SPLIT, norm: int = NORM_EUCLID8,
                 hbm_budget_bytes: int = 0, max_inflight: int = 0, max_pending: int = 0,
                 slots: int = 0, epoch_pixels: int = 0, epoch_work: float = 0.0,
                 count_iters: bool = False, schedule: Optional[dqj_schedule] = None,
                 policy: int = SERVE_FAIR):
        cfg = dqj_serve_config()
        cfg.struct_size = C.sizeof(dqj_serve_config)
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.max_inflight, cfg.max_pending = max_inflight, max_pending
        cfg.precision, cfg.norm, cfg.slots = precision, norm, slots
        cfg.count_iters = 1 if count_iters else 0
        cfg.epoch_pixels, cfg.epoch_work = epoch_pixels, epoch_work
        cfg.policy = policy
        if schedule is not None:
            cfg.sched = schedule
        h = C.c_void_p()
        _check(lib().dqj_serve_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, p, out: Dict) -> int:
        sp = make_params(p)
        fo = make_frame_out(out, p)
        t = C.c_uint64()
        _check(lib().dqj_serve_submit(self._h, C.byref(sp), C.byref(fo), C.byref(t)))
        self._keep[t.value] = out
        return t.value

    def submit_status(self, p, out: Dict):
        """(status, ticket) without raising: for tests of refusals."""
        sp = make_params(p)
        fo = make_frame_out(out, p)
        t = C.c_uint64()
        st = lib().dqj_serve_submit(self._h, C.byref(sp), C.byref(fo), C.byref(t))
        if st == OK:
            self._keep[t.value] = out
        return st, t.value

    def poll(self, ticket: int):
        r = dqj_request_result()
        r.struct_size = C.sizeof(dqj_request_result)
        st = lib().dqj_serve_poll(self._h, ticket, C.byref(r))
        if st == E_INVALID:
            _check(st)
        d = _result_dict(r)
        d["status"] = st
        return d

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = dqj_request_result()
        r.struct_size = C.sizeof(dqj_request_result)
        st = lib().dqj_serve_wait(self._h, ticket, timeout_ms, C.byref(r))
        if st == E_INVALID:
            _check(st)
        d = _result_dict(r)
        d["status"] = st
        if st not in (PENDING, E_TIMEOUT):
            self._keep.pop(ticket, None)
        return d

    def cancel(self, ticket: int) -> int:
        return lib().dqj_serve_cancel(self._h, ticket)

    def stats(self) -> Dict:
        s = dqj_serve_stats()
        s.struct_size = C.sizeof(dqj_serve_stats)
        _check(lib().dqj_serve_stats_get(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dqj_serve_stats._fields_ if k != "struct_size"}

    def close(self):
        if self._h:
            _check(lib().dqj_serve_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_info(device: int = 0) -> Dict:
    d = dqj_device_info()
    d.struct_size = C.sizeof(dqj_device_info)
    _check(lib().dqj_device_info_get(device, C.byref(d)))
    return {"arch": d.arch.decode(), "compute_units": d.compute_units, "clock_khz": d.clock_khz,
            "memory_clock_khz": d.memory_clock_khz, "total_mem_bytes": d.total_mem_bytes,
            "fp32_vector_peak_tflops": d.fp32_vector_peak_tflops,
            "fp32_unpacked_peak_tflops": d.fp32_unpacked_peak_tflops}


def measure_engine_clock(seconds: float = 0.2, device: int = 0) -> float:
    """Engine clock (MHz) the device sustains under an FP32 FMA load of about `seconds`
    (dqj_measure_engine_clock, include/dqj_measure.h)."""
    mhz = C.c_double(0.0)
    _check(lib().dqj_measure_engine_clock(int(device), float(seconds), C.byref(mhz)))
    return mhz.value


def exported_symbols() -> List[str]:
    return sorted(_SIGS)
