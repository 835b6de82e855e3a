"""The Python binding refuses output buffers the kernels would write outside of, or
scramble, before any pointer reaches the C ABI (these run without a GPU: every
refusal below is raised before a launch)."""
import pytest
import torch

import paper_2303_14827_amd as dqj
import workloads

P = workloads.plain_128()[0]


def good_outputs(width, height):
    return {
        "mask": torch.empty((height, width), dtype=torch.uint8),
        "depth": torch.empty((height, width), dtype=torch.float32),
        "shade": torch.empty((height, width), dtype=torch.float32),
        "normal": torch.empty((height, width, 3), dtype=torch.float32),
        "iters": torch.zeros((1,), dtype=torch.int64),
    }


def test_cpu_tensor_refused():
    with pytest.raises(ValueError, match="not on the GPU"):
        dqj.make_frame_out(good_outputs(P.width, P.height), P)


@pytest.mark.parametrize("name,bad,msg", [
    ("mask", torch.empty((128, 128), dtype=torch.int32), "dtype"),
    ("depth", torch.empty((128, 128), dtype=torch.float64), "dtype"),
    ("iters", torch.zeros((1,), dtype=torch.int32), "dtype"),
    ("shade", torch.empty((128, 127), dtype=torch.float32), "elements"),
    ("normal", torch.empty((128, 128), dtype=torch.float32), "elements"),
    ("depth", torch.empty((128, 256), dtype=torch.float32)[:, ::2], "contiguous"),
    ("mask", [0] * (128 * 128), "torch tensor"),
])
def test_bad_buffer_refused(name, bad, msg):
    o = good_outputs(P.width, P.height)
    o[name] = bad
    with pytest.raises(ValueError, match=msg):
        dqj.make_frame_out(o, P)


def test_required_output_missing_refused():
    o = good_outputs(P.width, P.height)
    del o["shade"]
    with pytest.raises(ValueError, match="required"):
        dqj.make_frame_out(o, P)


def test_batch_length_mismatch_refused():
    ps = workloads.plain_1024()
    with pytest.raises(ValueError, match="output dicts"):
        dqj.render_batch(ps, [good_outputs(p.width, p.height) for p in ps[:2]])


def test_points_shape_refused():
    with pytest.raises(ValueError, match="expected \\(n, 8\\)"):
        dqj.classify_points(torch.zeros((4, 7), dtype=torch.float32), P)
    with pytest.raises(ValueError, match="dtype"):
        dqj.classify_points(torch.zeros((4, 8), dtype=torch.float64), P, dqj.PREC_FP32)


def test_grid_buffer_refused():
    with pytest.raises(ValueError, match="elements"):
        dqj.classify_grid(P, 8, 8, 8, mask=torch.empty((8, 8, 7), dtype=torch.uint8))
