"""The engine clock probe (include/dqj_measure.h) on the GPU: it returns a clock in the
range of what an MI355X runs at, and leaves the current device as it was."""
import pytest

pytestmark = pytest.mark.gpu


def test_engine_clock_in_range():
    import torch
    import paper_2303_14827_amd as dqj
    before = torch.cuda.current_device()
    mhz = dqj.measure_engine_clock(0.05)
    print("engine clock MHz", mhz, flush=True)
    assert 500.0 < mhz < 3000.0
    assert torch.cuda.current_device() == before
