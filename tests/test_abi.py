"""The C ABI library: it loads, exports every function include/*.h declares, its
record layouts match the header, and validation rejects bad input before any
device work (these run without a GPU)."""
import ctypes as C
import glob
import os
import re
import subprocess

import pytest

import paper_2303_14827_amd as dqj
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dqj.h")
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(dqj_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_function():
    L = dqj.lib()
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding covers every one of them
    assert set(names) <= set(dqj.exported_symbols()) | {"dqj_last_error", "dqj_status_str"}


def test_record_sizes_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "dqj.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n",'
                   'sizeof(dqj_params), sizeof(dqj_frame_out), sizeof(dqj_schedule),'
                   'sizeof(dqj_device_info), sizeof(dqj_serve_config), sizeof(dqj_request_result),'
                   'sizeof(dqj_serve_stats)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                            check=True).stdout.split()]
    assert sizes == [C.sizeof(dqj.dqj_params), C.sizeof(dqj.dqj_frame_out),
                     C.sizeof(dqj.dqj_schedule), C.sizeof(dqj.dqj_device_info),
                     C.sizeof(dqj.dqj_serve_config), C.sizeof(dqj.dqj_request_result),
                     C.sizeof(dqj.dqj_serve_stats)]


def _render_status(p, **out_overrides):
    sp = dqj.make_params(p)
    fo = dqj.dqj_frame_out()
    fo.struct_size = C.sizeof(dqj.dqj_frame_out)
    fo.mask = fo.depth = fo.shade = 0x1000   # never dereferenced: validation fails first
    for k, v in out_overrides.items():
        setattr(fo, k, v)
    return dqj.lib().dqj_render(C.byref(sp), C.byref(fo), None), dqj.lib().dqj_last_error().decode()


BASE = workloads.plain_128()[0]


@pytest.mark.parametrize("field,value", [
    ("width", 0), ("height", 16385), ("max_iter", 0), ("max_iter", 5000), ("march_steps", 0),
    ("bisect_steps", -1), ("escape_radius", 0.0), ("escape_radius", float("inf")),
    ("fov_y_deg", 0.0), ("fov_y_deg", 180.0), ("normal_h", 0.0), ("norm", 2), ("precision", 7),
])
def test_validation_rejects(field, value):
    p = BASE.replace(**{field: value})
    st, msg = _render_status(p)
    assert st == dqj.E_INVALID, (st, msg)
    assert msg


def test_validation_rejects_geometry():
    for kw in (dict(eye=[0.0, 0.0, 0.0]), dict(up=list(BASE.eye)),
               dict(box_min=[1.5, -1.5, -1.5]), dict(light_dir=[0.0, 0.0, 0.0]),
               dict(c=[float("nan")] + [0.0] * 7)):
        p = BASE.replace(**kw)
        p.__post_init__()
        st, msg = _render_status(p)
        assert st == dqj.E_INVALID, (kw, st, msg)


def test_missing_required_output():
    st, msg = _render_status(BASE, depth=None)
    assert st == dqj.E_INVALID and "required" in msg


def test_bad_struct_size():
    sp = dqj.make_params(BASE)
    sp.struct_size = 12
    fo = dqj.dqj_frame_out()
    fo.struct_size = C.sizeof(dqj.dqj_frame_out)
    assert dqj.lib().dqj_render(C.byref(sp), C.byref(fo), None) == dqj.E_INVALID


def test_status_strings():
    L = dqj.lib()
    assert L.dqj_status_str(dqj.E_BUDGET) == b"DQJ_E_BUDGET"
    assert L.dqj_status_str(12345) == b"DQJ_E_UNKNOWN"


def test_batch_validation():
    n = 2
    arr_p = (dqj.dqj_params * n)(*[dqj.make_params(BASE), dqj.make_params(BASE.replace(width=0))])
    arr_o = (dqj.dqj_frame_out * n)()
    st = dqj.lib().dqj_render_batch(arr_p, arr_o, n, None)
    assert st in (dqj.E_INVALID, dqj.E_UNSUPPORTED, dqj.E_DEVICE)
    assert dqj.lib().dqj_render_batch(arr_p, arr_o, 0, None) in (dqj.E_INVALID, dqj.E_UNSUPPORTED,
                                                                 dqj.E_DEVICE)


def test_projection_validation():
    """Fibre tables are checked before any device work: count 0..32, a table when the
    count is positive, finite offsets; projection runs the FP32 fixed-step march only."""
    import numpy as np
    fib = np.zeros((33, 8))
    st, msg = _render_status(BASE.replace(fiber=fib))
    assert st == dqj.E_INVALID and "fiber_count" in msg, msg
    bad = np.zeros((2, 8))
    bad[1, 5] = float("nan")
    st, msg = _render_status(BASE.replace(fiber=bad))
    assert st == dqj.E_INVALID and "fiber" in msg, msg
    sp = dqj.make_params(BASE)
    sp.fiber_count = 3          # with no table
    fo = dqj.dqj_frame_out()
    fo.struct_size = C.sizeof(dqj.dqj_frame_out)
    fo.mask = fo.depth = fo.shade = 0x1000
    assert dqj.lib().dqj_render(C.byref(sp), C.byref(fo), None) == dqj.E_INVALID
    ok = np.zeros((4, 8))
    for kw in (dict(march=workloads.MARCH_DE), dict(precision=workloads.PREC_FP64),
               dict(precision=workloads.PREC_SPLIT)):
        st, msg = _render_status(BASE.replace(fiber=ok, **kw))
        assert st == dqj.E_UNSUPPORTED and "projection" in msg, (kw, st, msg)


def test_engine_clock_rejects_bad_arguments():
    L = dqj.lib()
    mhz = C.c_double(-1.0)
    assert L.dqj_measure_engine_clock(0, 0.0, C.byref(mhz)) == dqj.E_INVALID
    assert L.dqj_measure_engine_clock(0, 11.0, C.byref(mhz)) == dqj.E_INVALID
    assert L.dqj_measure_engine_clock(0, 0.1, None) == dqj.E_INVALID
    assert mhz.value == -1.0   # untouched on failure
