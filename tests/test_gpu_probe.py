"""The VALU issue-rate probe the VALU rooflines are taken against: a
plausible rate on the device, stable across calls, and refused while the
stream is being captured (it synchronises)."""
import ctypes

import pytest

from gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


def _rate(hg, stream=None):
    r = ctypes.c_double(0.0)
    st = hg._lib.load().hgsr_probe_valu_rate(ctypes.byref(r), stream)
    return st, r.value


def test_rate_is_plausible_and_stable(hg):
    import torch
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    rates = []
    for k in range(3):
        log(f"case: probe call {k}")
        st, v = _rate(hg)
        assert st == 0, hg._lib.load().hgsr_last_error()
        rates.append(v)
    per_cu_cycle = [v / (cus * 2.4e9) for v in rates]
    log("wave64 FMA per CU per nominal cycle", [round(x, 3) for x in per_cu_cycle])
    # at least half a wave64 FMA per CU per cycle, at most two (two 32-lane
    # passes per cycle on each of the four SIMDs) at the nominal clock
    assert all(0.5 < x < 2.0 for x in per_cu_cycle), per_cu_cycle
    assert max(rates) / min(rates) < 1.3, rates


def test_refused_while_capturing(hg):
    import torch
    r = hg.Renderer()
    s = torch.cuda.Stream()
    xi = torch.zeros((1, 6), device="cuda")
    poses = torch.zeros((1, 12), device="cuda")
    out = torch.empty_like(poses)
    torch.cuda.synchronize()
    log("case: probe during capture")
    with torch.cuda.stream(s):
        r.graph_begin(s)
        hg.pose_retract(poses, xi, out=out, stream=s)
        st, _ = _rate(hg, hg._stream_ptr(s))
        r.graph_end()
    torch.cuda.synchronize()
    assert st == 5, st  # HGSR_ERR_STATE
    st, v = _rate(hg)
    assert st == 0 and v > 0
